"""Pin of which cells the oracle's balanced-stencil refit selects (end of
Sec. 3.2: a reconstruction that leaves the range of its stencil's averages
is fitted again on a balanced stencil; here "leaves" means beyond a rounding
band of 1e-10 of the range plus 1e-14 of the largest magnitude).

The first fit of every cell is rebuilt here from the oracle's cell matrix,
weights and least-squares solver and evaluated at the facet points with
eval_taylor; the refitted set must be exactly the cells whose first-fit
facet values leave the banded range, and every other cell keeps its first
fit."""

import numpy as np
import pytest

from workloads import fields, jittered_cube, jittered_square


@pytest.mark.parametrize("dim", [2, 3])
def test_refit_set_from_its_definition(dim):
    import oracle

    if dim == 2:
        mesh = jittered_square(12, 0.3, 3201)
        u0 = fields.cell_averages(mesh, fields.gaussian_bump_with_step_2d)
        kw = dict(p=3, n_lo=12, n_hi=20)
    else:
        mesh = jittered_cube(5, 0.15, 3202)
        u0 = fields.cell_averages(mesh, fields.sine_with_sphere_3d)
        kw = dict(p=3, n_lo=30, n_hi=50)
    u0 = np.asarray(u0, dtype=np.float64).reshape(-1)
    o = oracle.Oracle(dim, mesh.verts, mesh.cells, flux="advection", balance=True, **kw)
    ref = o.reconstruct(u0)
    exps = oracle.basis(dim, kw["p"])
    qx, cent = o.mesh.qx, o.mesh.cent
    nc, F, Q = qx.shape[0], qx.shape[1], qx.shape[2]
    first = np.zeros((nc, F, Q))
    out = np.zeros(nc, dtype=bool)
    for i in range(nc):
        rows = o.stencil_of(i)
        coef, _, _, _ = oracle.wls_qrcp_solve(o.cell_matrix(i), o.cell_weights(i, u0), u0[rows], 1e-12)
        for lf in range(F):
            for q in range(Q):
                first[i, lf, q] = oracle.eval_taylor(dim, exps, coef, qx[i, lf, q] - cent[i])
        mn, mx = u0[rows].min(), u0[rows].max()
        band = 1e-10 * (mx - mn) + 1e-14 * max(abs(mx), abs(mn))
        out[i] = bool(np.any((first[i] > mx + band) | (first[i] < mn - band)))
    reb = ref["rebalanced"].astype(bool)
    assert out.sum() > 3, "the data must make some cells leave their range"
    assert np.array_equal(reb, out)
    keep = ~reb
    assert np.allclose(ref["fval"][0][keep], first[keep], rtol=1e-12, atol=1e-14)
