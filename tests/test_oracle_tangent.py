"""Pins of the oracle's tangent build (exact directional derivatives).

The tangent build runs the oracle's own code on forward-mode dual numbers
(oracle/tangent.hpp): J d of the right-hand side and of the TVD RK3
trajectory, with every branch (facet neighbour of the centre's smallest
indicator, pivots, rank) held at the point.  It is pinned against things
outside itself:

* its values are bitwise those of the FP64 build (same operations);
* with unit weights the scheme is linear in u, so J d is the scheme applied
  to d (Sec. 3.1.1: plain least squares is a linear map of the averages);
* with the WLS-ENO weights (Sec. 3.1.2) it matches central differences of the
  extended-precision (x87) build on data without ties, for the right-hand
  side and over two RK3 steps (Sec. 4.2.1);
* where the data has exact ties (plateaus, where two facet neighbours give
  the centre the same smallest indicator) the map has kinks; there the
  tangent equals the forward or the backward one-sided difference, i.e. the
  derivative of one branch.
"""

import numpy as np
import pytest

from workloads import configs, fields, periodic_line


def _pair(oracle_lib, mesh, periodic=False, **kw):
    ot = oracle_lib.Oracle(mesh.dim, mesh.verts, mesh.cells, periodic, tangent=True, **kw)
    ox = oracle_lib.Oracle(mesh.dim, mesh.verts, mesh.cells, periodic, extended=True, **kw)
    return ot, ox


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


SQUARE_KW = {
    "advection": dict(p=3, n_lo=12, n_hi=20, flux="advection", velocity=(1.0, 0.5, 0.0), bc=1),
    "burgers": dict(p=3, n_lo=12, n_hi=20, flux="burgers"),
    "burgers-local": dict(p=3, n_lo=12, n_hi=20, flux="burgers", lf_alpha=1),
}


@pytest.mark.parametrize("case", ["advection", "burgers", "euler", "line", "cube"])
def test_tangent_values_bitwise_fp64(oracle_lib, case):
    """The dual numbers' values are the FP64 oracle's, bit for bit."""
    from workloads import jittered_cube

    rng = np.random.default_rng(11)
    periodic = False
    if case in ("advection", "burgers"):
        wl = configs.square_advection_adjoint(20, 5001)
        mesh, u0, kw = wl.mesh, wl.u0, SQUARE_KW[case]
    elif case == "euler":
        wl = configs.square_advection_adjoint(14, 5001)
        mesh = wl.mesh
        u0 = fields.cell_averages(mesh, fields.euler_quadrants(4125))
        kw = dict(p=3, n_lo=12, n_hi=20, flux="euler")
    elif case == "line":
        mesh = periodic_line(40, 0.1, 1001)
        periodic = True
        u0 = fields.square_wave_sine_1d(mesh)
        kw = dict(p=3, n_lo=5, n_hi=5, flux="burgers")
    else:
        mesh = jittered_cube(4, 0.15, 4001)
        u0 = fields.cell_averages(mesh, fields.sine_with_sphere_3d)
        kw = dict(p=2, n_lo=8, n_hi=16, flux="advection", velocity=(1.0, 0.5, 0.25))
    o = oracle_lib.Oracle(mesh.dim, mesh.verts, mesh.cells, periodic, **kw)
    ot = oracle_lib.Oracle(mesh.dim, mesh.verts, mesh.cells, periodic, tangent=True, **kw)
    D = rng.standard_normal((2, np.size(u0)))
    L, _ = o.rhs(u0)
    Lt, _ = ot.rhs_tangent(u0, D)
    assert np.array_equal(L, Lt)
    uT = o.step(u0, 1e-3, 2)
    uTt, _ = ot.step_tangent(u0, D, 1e-3, 2)
    assert np.array_equal(uT, uTt)


def test_tangent_of_linear_scheme(oracle_lib):
    """Unit weights make advection linear: J(u) d = L(d) and the trajectory's
    tangent is the trajectory of d."""
    wl = configs.square_advection_adjoint(20, 5001)
    kw = dict(SQUARE_KW["advection"], weight_mode=1)
    o = oracle_lib.Oracle(2, wl.mesh.verts, wl.mesh.cells, **kw)
    ot = oracle_lib.Oracle(2, wl.mesh.verts, wl.mesh.cells, tangent=True, **kw)
    D = np.random.default_rng(12).standard_normal((3, wl.mesh.n_cell))
    _, JR = ot.rhs_tangent(wl.u0, D)
    _, JT = ot.step_tangent(wl.u0, D, 2e-3, 5)
    for k in range(3):
        assert _rel(JR[k], o.rhs(D[k])[0][0]) <= 1e-14
        assert _rel(JT[k], o.step(D[k], 2e-3, 5)[0]) <= 1e-14


@pytest.mark.parametrize("case", ["advection", "burgers", "burgers-local"])
def test_tangent_matches_extended_differences(oracle_lib, case):
    """Smooth data without ties (a sum of Gaussians): J d against central
    differences of the extended-precision build at step 1e-8, norm-wise, for
    L and for two RK3 steps.  Measured: 5e-9 to 9e-8 (rounding of the
    differenced fluxes and the occasional near-tie within the step)."""
    wl = configs.square_advection_adjoint(24, 5001)
    ot, ox = _pair(oracle_lib, wl.mesh, **SQUARE_KW[case])
    u0 = wl.u0
    D = np.random.default_rng(13).standard_normal((2, wl.mesh.n_cell))
    h, dt = 1e-8, 2e-3
    _, JR = ot.rhs_tangent(u0, D)
    _, JT = ot.step_tangent(u0, D, dt, 2)
    for k in range(2):
        fd = (ox.rhs(u0 + h * D[k])[0] - ox.rhs(u0 - h * D[k])[0])[0] / (2 * h)
        assert _rel(fd, JR[k]) <= 2e-7, (case, k, _rel(fd, JR[k]))
        fs = ((ox.step(u0 + h * D[k], dt, 2) - ox.step(u0 - h * D[k], dt, 2)) / (2 * h))[0]
        assert _rel(fs, JT[k]) <= 2e-7, (case, k, _rel(fs, JT[k]))


def test_tangent_on_line(oracle_lib):
    """1-D periodic, smooth data: three RK3 steps against central differences."""
    mesh = periodic_line(60, 0.1, 1001)
    x = 0.5 * (mesh.verts[mesh.cells[:, 0], 0] + mesh.verts[mesh.cells[:, 1], 0])
    u0 = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x)
    d = np.random.default_rng(14).standard_normal((1, mesh.n_cell))
    for flux in ("advection", "burgers"):
        ot, ox = _pair(oracle_lib, mesh, True, p=3, n_lo=5, n_hi=5, flux=flux)
        _, JT = ot.step_tangent(u0, d, 2e-3, 3)
        h = 1e-8
        fs = ((ox.step(u0 + h * d[0], 2e-3, 3) - ox.step(u0 - h * d[0], 2e-3, 3)) / (2 * h))[0]
        assert _rel(fs, JT[0]) <= 2e-7


@pytest.mark.parametrize("flux", ["advection", "burgers"])
def test_tangent_at_ties_is_one_sided(oracle_lib, flux):
    """Bump-and-step data has plateaus, so some cells have two facet
    neighbours tied for the smallest indicator and L has a kink there (the
    forward and backward differences disagree).  At every such cell the
    tangent is the derivative of one side; elsewhere it is the central
    difference."""
    wl = configs.square_advection_adjoint(30, 5001)
    mesh = wl.mesh
    u0 = fields.cell_averages(mesh, fields.gaussian_bump_with_step_2d)
    ot, ox = _pair(oracle_lib, mesh, **SQUARE_KW[flux])
    D = np.random.default_rng(15).standard_normal((2, mesh.n_cell))
    _, J = ot.rhs_tangent(u0, D)
    h = 1e-8
    f0 = ox.rhs(u0)[0][0]
    kinks = 0
    for k in range(2):
        fp, fm = ox.rhs(u0 + h * D[k])[0][0], ox.rhs(u0 - h * D[k])[0][0]
        fw, bw, ce = (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)
        sc = np.max(np.abs(J[k]))
        kink = np.abs(fw - bw) > 1e-4 * sc
        kinks += int(kink.sum())
        assert np.max(np.abs(ce - J[k])[~kink]) <= 1e-6 * sc
        one_sided = np.minimum(np.abs(fw - J[k]), np.abs(bw - J[k]))[kink]
        assert np.all(one_sided <= 1e-5 * sc)
    assert kinks > 0          # the case does exercise the kinks
