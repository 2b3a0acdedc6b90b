"""Pin of the oracle's Euler positivity fallback (reading R16: a cell whose
reconstruction has a non-positive density or pressure at any facet point
keeps its cell averages at all of its facet points).

The unlimited component-wise reconstruction of every cell is rebuilt here
from the oracle's cell matrix, weights and least-squares solver and
evaluated at the facet points with eval_taylor; the oracle's fallback set
must be exactly the cells this predicate selects, fallback cells must carry
their averages at every point, and the others the unlimited values."""

import numpy as np
import pytest

from workloads import fields, jittered_square

GAMMA = 1.4


def _near_vacuum(x, gamma=GAMMA):
    r = np.where(np.hypot(x[:, 0] - 0.5, x[:, 1] - 0.5) < 0.25, 1.0, 1e-3)
    u = np.where(x[:, 0] > 0.5, 2.0, -2.0)
    v = 0.5 * np.ones_like(u)
    pr = np.where(x[:, 1] > 0.45, 1.0, 2e-4)
    E = pr / (gamma - 1.0) + 0.5 * r * (u * u + v * v)
    return np.stack([r, r * u, r * v, E], axis=1)


@pytest.mark.parametrize("p,n_lo,n_hi", [(3, 12, 20), (4, 20, 36)])
def test_fallback_set_from_its_definition(p, n_lo, n_hi):
    import oracle

    mesh = jittered_square(10, 0.3, 3102)
    u0 = fields.cell_averages(mesh, _near_vacuum)           # (4, nc)
    o = oracle.Oracle(2, mesh.verts, mesh.cells, p=p, n_lo=n_lo, n_hi=n_hi, flux="euler", gamma=GAMMA)
    ref = o.reconstruct(u0)
    exps = oracle.basis(2, p)
    qx, cent = o.mesh.qx, o.mesh.cent
    nc, F, Q = qx.shape[0], qx.shape[1], qx.shape[2]
    vals = np.zeros((4, nc, F, Q))
    for i in range(nc):
        A = o.cell_matrix(i)
        rows = o.stencil_of(i)
        for v in range(4):
            w = o.cell_weights(i, u0[v])
            coef, _, _, _ = oracle.wls_qrcp_solve(A, w, u0[v][rows], 1e-12)
            for lf in range(F):
                for q in range(Q):
                    vals[v, i, lf, q] = oracle.eval_taylor(2, exps, coef, qx[i, lf, q] - cent[i])
    rho = vals[0]
    pres = (GAMMA - 1.0) * (vals[3] - 0.5 * (vals[1] ** 2 + vals[2] ** 2) / rho)
    bad = np.any(~(rho > 0.0) | ~(pres > 0.0), axis=(1, 2))
    fb = ref["fallback"].astype(bool)
    assert bad.sum() > 3, "the data must make some cells fall back"
    assert np.array_equal(fb, bad)
    assert np.all(ref["fval"][:, fb] == u0[:, fb, None, None])
    keep = ~fb
    assert np.allclose(ref["fval"][:, keep], vals[:, keep], rtol=1e-12, atol=1e-14)
