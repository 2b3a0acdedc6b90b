"""Pins of the oracle's characteristic-wise Euler reconstruction.

The paper reconstructs the Euler system field by field in the eigenvector
basis of the flux Jacobian (Sec. 5.1.4, which prints f'(u) and R(u) for 1-D;
Sec. 5.2.4 uses the same decomposition along facet normals in 2-D).  These
tests tie the oracle's eigenvectors to the printed Jacobian and to central
differences of its own flux, and its per-facet reconstruction to the
component-wise one wherever linear algebra says they must agree.
"""

import numpy as np
import pytest

from workloads import jittered_square, fields

GAMMA = 1.4


def _state(rng, dim):
    rho = rng.uniform(0.2, 2.0)
    vel = rng.uniform(-1.5, 1.5, dim)
    p = rng.uniform(0.1, 3.0)
    E = p / (GAMMA - 1.0) + 0.5 * rho * vel @ vel
    return np.concatenate([[rho], rho * vel, [E]]), rho, vel, p


def _unit(rng, dim):
    if dim == 1:
        return np.array([rng.choice([-1.0, 1.0])])
    t = rng.uniform(0, 2 * np.pi)
    return np.array([np.cos(t), np.sin(t)])


@pytest.mark.parametrize("dim", [1, 2])
def test_left_and_right_eigenvectors_are_inverse(dim):
    import oracle

    rng = np.random.default_rng(11 + dim)
    for _ in range(50):
        U, *_ = _state(rng, dim)
        L, R = oracle.char_basis(dim, GAMMA, U, _unit(rng, dim))
        assert np.max(np.abs(L @ R - np.eye(dim + 2))) < 1e-12 * max(1.0, np.max(np.abs(R)) * np.max(np.abs(L)))


def test_1d_diagonalises_the_printed_jacobian():
    """R^{-1} f'(u) R = diag(v-c, v, v+c) with f'(u) as printed in Sec. 5.1.4."""
    import oracle

    rng = np.random.default_rng(5)
    g = GAMMA
    for _ in range(50):
        U, rho, vel, p = _state(rng, 1)
        v = vel[0]
        H = (U[2] + p) / rho
        c = np.sqrt(g * p / rho)
        J = np.array([[0.0, 1.0, 0.0],
                      [0.5 * (g - 3.0) * v * v, (3.0 - g) * v, g - 1.0],
                      [0.5 * (g - 1.0) * v ** 3 - v * H, H - (g - 1.0) * v * v, g * v]])
        L, R = oracle.char_basis(1, g, U, np.array([1.0]))
        D = L @ J @ R
        lam = np.array([v - c, v, v + c])
        assert np.max(np.abs(D - np.diag(lam))) < 1e-12 * (1 + np.max(np.abs(lam))) * np.max(np.abs(R))


def test_2d_diagonalises_the_flux_jacobian():
    """L A_n R = diag(q_n - c, q_n, q_n, q_n + c) for A_n from central
    differences of the oracle's normal flux F(U).n."""
    import oracle

    rng = np.random.default_rng(6)
    for _ in range(30):
        U, rho, vel, p = _state(rng, 2)
        n = _unit(rng, 2)
        A = np.zeros((4, 4))
        for k in range(4):
            h = 1e-6 * max(1.0, abs(U[k]))
            e = np.zeros(4)
            e[k] = h
            A[:, k] = (oracle.euler_normal_flux(2, GAMMA, U + e, n) - oracle.euler_normal_flux(2, GAMMA, U - e, n)) / (2 * h)
        L, R = oracle.char_basis(2, GAMMA, U, n)
        qn = vel @ n
        c = np.sqrt(GAMMA * p / rho)
        lam = np.array([qn - c, qn, qn, qn + c])
        D = L @ A @ R
        assert np.max(np.abs(D - np.diag(lam))) < 1e-6 * (1 + np.max(np.abs(lam))) * np.max(np.abs(R)) * np.max(np.abs(L))


def test_2d_reduces_to_1d_along_x():
    """With n = (1, 0) and no y-velocity the 2-D decomposition restricted to
    (rho, rho u, E) is the 1-D one of Sec. 5.1.4."""
    import oracle

    rng = np.random.default_rng(7)
    for _ in range(20):
        U1, rho, vel, p = _state(rng, 1)
        U2 = np.array([U1[0], U1[1], 0.0, U1[2]])
        L1, R1 = oracle.char_basis(1, GAMMA, U1, np.array([1.0]))
        L2, R2 = oracle.char_basis(2, GAMMA, U2, np.array([1.0, 0.0]))
        keep_c, keep_f = [0, 1, 3], [0, 1, 3]
        assert np.allclose(R2[np.ix_(keep_c, keep_f)], R1, rtol=1e-14, atol=1e-14)
        assert np.allclose(L2[np.ix_(keep_f, keep_c)], L1, rtol=1e-14, atol=1e-14)


def _euler_fields(mesh, seed):
    """Smooth positive 2-D Euler averages (conserved variables)."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(1, 3, 4)

    def prim(x):
        rho = 1.0 + 0.3 * np.sin(k[0] * x[:, 0] + 0.4) * np.cos(k[1] * x[:, 1])
        u = 0.5 * np.cos(k[2] * x[:, 1])
        v = -0.3 * np.sin(k[3] * x[:, 0])
        p = 1.0 + 0.2 * np.cos(k[0] * x[:, 0] * x[:, 1])
        return rho, u, v, p

    comps = [lambda x: prim(x)[0], lambda x: prim(x)[0] * prim(x)[1], lambda x: prim(x)[0] * prim(x)[2],
             lambda x: prim(x)[3] / (GAMMA - 1) + 0.5 * prim(x)[0] * (prim(x)[1] ** 2 + prim(x)[2] ** 2)]
    return np.stack([fields.cell_averages(mesh, f) for f in comps])


def test_characteristic_equals_components_with_unit_weights():
    """With unit weights the least-squares fit is linear in the data, so
    R (fit of L U) = fit of U: both modes give the same facet values and rhs."""
    import oracle

    mesh = jittered_square(9, 0.3, 71)
    u = _euler_fields(mesh, 3)
    kw = dict(p=3, n_lo=12, n_hi=20, flux="euler", weight_mode=1)
    oc = oracle.Oracle(2, mesh.verts, mesh.cells, characteristic=False, **kw)
    ox = oracle.Oracle(2, mesh.verts, mesh.cells, characteristic=True, **kw)
    fc, fx = oc.reconstruct(u)["fval"], ox.reconstruct(u)["fval"]
    assert np.max(np.abs(fc - fx)) < 1e-12 * np.max(np.abs(fc))
    Lc, ac = oc.rhs(u)
    Lx, ax = ox.rhs(u)
    assert ax == pytest.approx(ac, rel=1e-13)
    assert np.max(np.abs(Lc - Lx)) < 1e-10 * np.max(np.abs(Lc))


def test_characteristic_weights_differ_from_components():
    """With WLS-ENO weights the two modes differ at a discontinuity (the
    weights follow the characteristic fields, not the components)."""
    import oracle

    mesh = jittered_square(9, 0.3, 72)
    cent = oracle.OracleMesh(2, mesh.verts, mesh.cells, False, p=3).cent
    left = cent[:, 0] < 0.5
    u = np.zeros((4, mesh.n_cell))
    u[0] = np.where(left, 1.0, 0.125)
    u[3] = np.where(left, 1.0, 0.1) / (GAMMA - 1)
    kw = dict(p=3, n_lo=12, n_hi=20, flux="euler")
    fc = oracle.Oracle(2, mesh.verts, mesh.cells, characteristic=False, **kw).reconstruct(u)["fval"]
    fx = oracle.Oracle(2, mesh.verts, mesh.cells, characteristic=True, **kw).reconstruct(u)["fval"]
    assert np.max(np.abs(fc - fx)) > 1e-4


@pytest.mark.parametrize("p,n_lo,n_hi", [(3, 12, 20), (4, 18, 24)])
def test_characteristic_reproduces_polynomials(p, n_lo, n_hi):
    """Each projected field L U of polynomial data is a polynomial (L is fixed
    per facet), so it is reconstructed exactly and R maps it back exactly."""
    import oracle

    mesh = jittered_square(10, 0.3, 73)
    o = oracle.Oracle(2, mesh.verts, mesh.cells, p=p, n_lo=n_lo, n_hi=n_hi, flux="euler", characteristic=True)
    fns = [fields.polynomial_field(40 + c, 2, p - 1, scale=0.1) for c in range(4)]
    base = [1.0, 0.2, -0.1, 3.0]
    comps = [(lambda f, b: (lambda x: b + f(x)))(f, b) for f, b in zip(fns, base)]
    u = np.stack([fields.cell_averages(mesh, f) for f in comps])
    fv = o.reconstruct(u)["fval"]
    qx = o.mesh.qx.reshape(-1, 2)
    exact = np.stack([f(qx).reshape(fv.shape[1:]) for f in comps])
    assert np.max(np.abs(fv - exact)) < 1e-11 * np.max(np.abs(exact))


def test_characteristic_uniform_state_is_steady():
    import oracle

    mesh = jittered_square(8, 0.3, 41)
    o = oracle.Oracle(2, mesh.verts, mesh.cells, p=3, n_lo=12, n_hi=20, flux="euler", characteristic=True)
    U = np.array([0.8, 0.8 * 0.3, 0.8 * -0.2, 1.0 / 0.4 + 0.5 * 0.8 * 0.13])
    L, _ = o.rhs(np.repeat(U[:, None], o.nc, axis=1))
    assert np.max(np.abs(L)) < 1e-10


def test_exact_riemann_solver():
    """The exact Riemann solution used to validate shock tubes: Rankine-
    Hugoniot across its shock, isentropic fan, and a symmetric problem with
    u* = 0."""
    import riemann

    g = GAMMA
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = riemann.star_state(L, R, g)
    # right shock: mass and momentum flux continuous in the shock frame
    w = riemann.sample(L, R, np.array([us + 1e-9, 5.0]), g)
    r1, u1, p1 = w[:, 0]
    r2, u2, p2 = w[:, 1]
    s = (r1 * u1 - r2 * u2) / (r1 - r2)
    assert (r1 * (u1 - s) - r2 * (u2 - s)) == pytest.approx(0.0, abs=1e-12)
    assert (r1 * (u1 - s) ** 2 + p1) == pytest.approx(r2 * (u2 - s) ** 2 + p2, rel=1e-12)
    E1 = p1 / (g - 1) + 0.5 * r1 * u1 ** 2
    E2 = p2 / (g - 1) + 0.5 * r2 * u2 ** 2
    assert ((E1 + p1) * u1 - s * E1) == pytest.approx((E2 + p2) * u2 - s * E2, rel=1e-10)
    # left rarefaction: p / rho^gamma constant and u + 2c/(gamma-1) constant through the fan
    xi = np.linspace(-1.18, -0.08, 7)
    r, u, p = riemann.sample(L, R, xi, g)
    assert np.allclose(p / r ** g, 1.0, rtol=1e-12)
    assert np.allclose(u + 2 * np.sqrt(g * p / r) / (g - 1), 2 * np.sqrt(g) / (g - 1), rtol=1e-12)
    # symmetric collision
    ps2, us2 = riemann.star_state((1.0, 0.5, 1.0), (1.0, -0.5, 1.0), g)
    assert us2 == pytest.approx(0.0, abs=1e-14) and ps2 > 1.0
