"""The sub-mesh oracle of the full-size GPU tests (tests/submesh.py) gives, at
the sampled cells, exactly what the whole-mesh oracle gives: the same
stencils, and bit for bit the same facet values, coefficients, ranks and
right-hand sides (CPU; meshes small enough for the whole-mesh oracle, with
the sub-mesh radii of the GPU tests)."""

import numpy as np
import pytest

import oracle
from submesh import SubOracle, mean_edge, sample_cells
from workloads import fields, jittered_cube, jittered_square


@pytest.mark.parametrize("case", ["square-burgers-local-alpha", "square-advection-zero-outside", "cube-advection"])
def test_submesh_oracle_equals_whole_mesh(case):
    if case.startswith("square"):
        mesh = jittered_square(60, 0.3, 9201)
        u0 = fields.cell_averages(mesh, fields.gaussian_bump_with_step_2d)
        R, ns = 4, (8, 4)
        if "burgers" in case:
            kw = dict(p=3, n_lo=12, n_hi=20, flux="burgers", lf_alpha=1)
        else:
            kw = dict(p=3, n_lo=12, n_hi=20, flux="advection", velocity=(1.0, 0.5, 0.0), bc=1)
    else:
        mesh = jittered_cube(14, 0.15, 9202)
        u0 = fields.cell_averages(mesh, fields.sine_with_sphere_3d)
        R, ns = 3, (3, 2)
        kw = dict(p=3, n_lo=30, n_hi=50, flux="advection", velocity=(1.0, 0.5, 0.25))
    sample = sample_cells(mesh, *ns, 9203)
    full = oracle.Oracle(mesh.dim, mesh.verts, mesh.cells, False, **kw)
    assert mean_edge(mesh.verts, mesh.cells) == full.h
    sub = SubOracle(mesh, u0, sample, R, **kw)
    assert len(sub.keep) < mesh.n_cell // 2, "not a proper sub-mesh"
    for i, row in zip(sample, sub.stencil_rows()):
        assert np.array_equal(row, full.stencil_of(i)), f"stencil of cell {i}"
    rf, rs = full.reconstruct(u0), sub.o.reconstruct(sub.u)
    for key in ("fval", "coef", "rank"):
        assert np.array_equal(rs[key][:, sub.loc], rf[key][:, sample]), key
    Lf, _ = full.rhs(u0)
    Ls, _ = sub.o.rhs(sub.u)
    assert np.array_equal(Ls.reshape(-1)[sub.loc], Lf.reshape(-1)[sample])
