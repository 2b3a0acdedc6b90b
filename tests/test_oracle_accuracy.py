"""Accuracy and non-oscillation pins of the oracle (convergence studies).

* Sec. 4.1 (accuracy theorem): on smooth data the degree p-1 reconstruction
  is p-th order accurate at the facet points.
* Sec. 5.1.2 / 5.1.3: the 1-D wave and Burgers solutions converge at the
  scheme's order while the solution is smooth (Burgers: exact solution by
  characteristics before the shock time 1/0.7).
* Sec. 5.2.1: on irregular triangle meshes p = 3 gives only second order for
  the wave equation.
* Sec. 5.1.2 (piecewise initial data): the weighted scheme stays
  non-oscillatory where plain least squares overshoots.
"""

import numpy as np
import pytest
from scipy.optimize import brentq

from workloads import periodic_line, jittered_square, jittered_cube, fields, configs


def _slopes(hs, errs):
    hs, errs = np.log(np.asarray(hs)), np.log(np.asarray(errs))
    return np.diff(errs) / np.diff(hs)


def _fit_slope(hs, errs):
    return float(np.polyfit(np.log(hs), np.log(errs), 1)[0])


@pytest.mark.parametrize("p,n", [(3, 5), (5, 7)])
def test_reconstruction_order_1d(p, n):
    import oracle

    hs, errs = [], []
    for N in (40, 80, 160, 320):
        mesh = periodic_line(N, 0.1, 100 + N)
        ubar = fields.line_cell_averages(mesh, lambda x: -np.cos(2 * np.pi * x) / (2 * np.pi))
        o = oracle.Oracle(1, mesh.verts, mesh.cells, True, p=p, n_lo=n, n_hi=n)
        fv = o.reconstruct(ubar)["fval"][0]
        exact = np.sin(2 * np.pi * o.mesh.qx[..., 0])
        errs.append(np.max(np.abs(fv - exact)))
        hs.append(1.0 / N)
    assert np.all(_slopes(hs, errs) >= p - 0.3), (errs, _slopes(hs, errs))


def test_reconstruction_order_2d_p3():
    import oracle

    fn = lambda x: np.sin(2 * x[:, 0] + 1.0) * np.cos(3 * x[:, 1])
    hs, errs = [], []
    for P in (16, 32, 64):
        mesh = jittered_square(P, 0.3, 200 + P)
        ubar = fields.cell_averages(mesh, fn)
        o = oracle.Oracle(2, mesh.verts, mesh.cells, p=3, n_lo=12, n_hi=20)
        fv = o.reconstruct(ubar)["fval"][0]
        exact = fn(o.mesh.qx.reshape(-1, 2)).reshape(fv.shape)
        errs.append(np.max(np.abs(fv - exact)))
        hs.append(o.mesh.h)
    assert _fit_slope(hs, errs) >= 3 - 0.3 and _slopes(hs, errs)[-1] >= 3 - 0.3, (errs, _slopes(hs, errs))


@pytest.mark.slow
def test_reconstruction_order_2d_p5():
    """Degree-4 reconstruction on 24-30 cell stencils: fifth order at the
    facet points (3-point Gauss-Legendre edges), interior cells."""
    import oracle

    fn = lambda x: np.sin(2 * x[:, 0] + 1.0) * np.cos(3 * x[:, 1])
    hs, errs = [], []
    for P in (12, 24, 48):
        mesh = jittered_square(P, 0.3, 210 + P)
        ubar = fields.cell_averages(mesh, fn)
        o = oracle.Oracle(2, mesh.verts, mesh.cells, p=5, n_lo=24, n_hi=30)
        fv = o.reconstruct(ubar)["fval"][0]
        exact = fn(o.mesh.qx.reshape(-1, 2)).reshape(fv.shape)
        inner = np.all((o.mesh.cv > 0.2) & (o.mesh.cv < 0.8), axis=(1, 2))
        errs.append(np.max(np.abs(fv - exact)[inner]))
        hs.append(o.mesh.h)
    assert _fit_slope(hs, errs) >= 5 - 0.5, (errs, _slopes(hs, errs))


@pytest.mark.slow
def test_reconstruction_order_3d_p3():
    import oracle

    fn = lambda x: np.sin(2 * x[:, 0] + 1.0) * np.cos(x[:, 1] - 0.5 * x[:, 2])
    hs, errs = [], []
    for P in (5, 8, 12):
        mesh = jittered_cube(P, 0.15, 300 + P)
        ubar = fields.cell_averages(mesh, fn)
        o = oracle.Oracle(3, mesh.verts, mesh.cells, p=3, n_lo=30, n_hi=50)
        fv = o.reconstruct(ubar)["fval"][0]
        exact = fn(o.mesh.qx.reshape(-1, 3)).reshape(fv.shape)
        # interior cells (all vertices off the boundary) to avoid one-sided stencils
        inner = np.all((o.mesh.cv > 0.15) & (o.mesh.cv < 0.85), axis=(1, 2))
        errs.append(np.max(np.abs(fv - exact)[inner]))
        hs.append(o.mesh.h)
    assert _fit_slope(hs, errs) >= 3 - 0.4, (errs, _slopes(hs, errs))


def test_wave_equation_order_1d():
    """u_t + u_x = 0, periodic, smooth data, jittered grid, t = 0.25."""
    import oracle

    hs, errs = [], []
    T = 0.25
    for N in (20, 40, 80):
        mesh = periodic_line(N, 0.1, 400 + N)
        F = lambda x: -np.cos(2 * np.pi * x) / (2 * np.pi)
        ubar = fields.line_cell_averages(mesh, F)
        o = oracle.Oracle(1, mesh.verts, mesh.cells, True, p=5, n_lo=7, n_hi=7)
        nsteps = int(np.ceil(T / (0.4 / N)))
        dt = T / nsteps
        u = o.step(ubar, dt, nsteps)[0]
        exact = fields.line_cell_averages(mesh, lambda x: F(x - T))
        errs.append(np.max(np.abs(u - exact)))
        hs.append(1.0 / N)
    # fifth-order space, third-order time with dt ~ h: the observed order is >= 3
    assert np.all(_slopes(hs, errs) >= 3.0), (errs, _slopes(hs, errs))
    assert errs[-1] < 1e-5


def _burgers_exact(x, t):
    """u = 0.3 + 0.7 sin(x - u t) solved per point (before the shock time)."""
    out = np.empty_like(x)
    for k, xx in enumerate(x):
        f = lambda u: u - 0.3 - 0.7 * np.sin(xx - u * t)
        out[k] = brentq(f, -0.5, 1.1)
    return out


def test_burgers_exact_solution_1d():
    """Sec. 5.1.3: u_t + (u^2/2)_x = 0 on [0, 2 pi], u0 = 0.3 + 0.7 sin x, smooth at t = 0.5."""
    import oracle

    T = 0.5
    hs, errs = [], []
    for N in (32, 64, 128):
        L = 2 * np.pi
        mesh = periodic_line(N, 0.0, 0, 0.0, L)
        ubar = fields.line_cell_averages(mesh, lambda x: 0.3 * x - 0.7 * np.cos(x))
        o = oracle.Oracle(1, mesh.verts, mesh.cells, True, p=5, n_lo=7, n_hi=7, flux="burgers")
        h = L / N
        nsteps = int(np.ceil(T / (0.3 * h)))
        u = o.step(ubar, T / nsteps, nsteps)[0]
        # exact cell averages by 8-point Gauss per cell
        g, w = np.polynomial.legendre.leggauss(8)
        a, b = mesh.verts[:-1, 0], mesh.verts[1:, 0]
        pts = (0.5 * (a + b))[:, None] + 0.5 * (b - a)[:, None] * g[None, :]
        ex = _burgers_exact(pts.ravel(), T).reshape(pts.shape) @ (0.5 * w)
        errs.append(np.max(np.abs(u - ex)))
        hs.append(h)
    assert np.all(_slopes(hs, errs) >= 3.0), (errs, _slopes(hs, errs))


@pytest.mark.slow
def test_wave_equation_order_2d_irregular_p3():
    """Sec. 5.2.1: p = 3 on irregular triangles converges at (about) second order."""
    import oracle

    a = np.array([1.0, 1.0])
    T = 0.15
    fn0 = lambda x: np.exp(-((x[:, 0] - 0.4) ** 2 + (x[:, 1] - 0.4) ** 2) / 0.02)
    hs, errs = [], []
    for P in (12, 24, 48):
        mesh = jittered_square(P, 0.3, 500 + P)
        ubar = fields.cell_averages(mesh, fn0)
        o = oracle.Oracle(2, mesh.verts, mesh.cells, p=3, n_lo=12, n_hi=20, velocity=(1.0, 1.0, 0))
        nsteps = int(np.ceil(T / (0.25 * o.mesh.h)))
        u = o.step(ubar, T / nsteps, nsteps)[0]
        exact = fields.cell_averages(mesh, lambda x: fn0(x - a * T))
        errs.append(np.sqrt(np.sum(o.mesh.vol * (u - exact) ** 2)))
        hs.append(o.mesh.h)
    sl = _slopes(hs, errs)
    assert np.all(sl >= 1.6), (errs, sl)


def _overshoot(u):
    return max(0.0, u.max() - 1.0) + max(0.0, -1.0 - u.min())


def test_square_wave_stays_non_oscillatory():
    """Sec. 5.1.2 (piecewise data) on the 200-cell jittered periodic grid: WLS-ENO
    overshoot stays below a tenth of plain least squares' and the total
    variation does not grow by more than 1%."""
    import oracle

    wl = configs.line_advection()
    o = oracle.from_workload(wl)
    o_ls = oracle.from_workload(wl, weight_mode=1)
    dt = 0.5 * np.min(o.mesh.vol)
    u, v = wl.u0.copy(), wl.u0.copy()
    tv0 = np.sum(np.abs(np.diff(np.r_[u, u[0]])))
    worst_ratio = 0.0
    for s in range(10):
        u = o.step(u, dt, 10)[0]
        v = o_ls.step(v, dt, 10)[0]
        ou, ov = _overshoot(u), _overshoot(v)
        assert ov > 0.0
        worst_ratio = max(worst_ratio, ou / ov)
        tv = np.sum(np.abs(np.diff(np.r_[u, u[0]])))
        assert tv <= 1.01 * tv0
    assert worst_ratio <= 0.1
