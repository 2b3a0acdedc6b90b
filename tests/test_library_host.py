"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every function include/wlseno.h declares;
* a host-only context (device -1) builds stencils that equal the oracle's
  independent builder exactly (sets and row order; integer results);
* error paths return the documented status codes.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from workloads import periodic_line, jittered_square, jittered_square_periodic, jittered_cube, configs


@pytest.fixture(scope="module")
def lib():
    import paper_1602_02694_amd as P

    if not os.path.exists(P.LIB_PATH):
        from paper_1602_02694_amd import build

        build.build()
    from paper_1602_02694_amd import _native

    return _native.load()


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "wlseno.h")).read()
    declared = set(re.findall(r"\b(wlseno_[a-z_]+)\s*\(", hdr))
    from paper_1602_02694_amd import _native

    assert declared == set(_native.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _host_ctx(mesh, **kw):
    from paper_1602_02694_amd import WLSENO

    w = WLSENO(device=-1)
    w.mesh_upload(mesh.dim, mesh.verts, mesh.cells, mesh.periodic)
    w.stencil_build(**kw)
    return w


@pytest.mark.parametrize("case", ["line", "square", "square_p4", "square_p5", "cube", "torus", "torus_p5"])
def test_stencils_equal_oracle(lib, case):
    from oracle.mesh import OracleMesh

    if case == "line":
        mesh, kw = periodic_line(60, 0.1, 1001), dict(p=3, n_lo=5, n_hi=5)
    elif case == "square":
        mesh, kw = jittered_square(24, 0.3, 2001), dict(p=3, n_lo=12, n_hi=20)
    elif case == "square_p4":
        mesh, kw = jittered_square(16, 0.3, 3001), dict(p=4, n_lo=20, n_hi=36)
    elif case == "square_p5":
        mesh, kw = jittered_square(16, 0.3, 3002), dict(p=5, n_lo=24, n_hi=30)
    elif case == "torus":
        mesh, kw = jittered_square_periodic(20, 0.3, 2003), dict(p=3, n_lo=12, n_hi=20)
    elif case == "torus_p5":
        mesh, kw = jittered_square_periodic(14, 0.3, 2004), dict(p=5, n_lo=24, n_hi=30)
    else:
        mesh, kw = jittered_cube(6, 0.15, 4001), dict(p=3, n_lo=30, n_hi=50)
    w = _host_ctx(mesh, **kw)
    rp, col = w.stencil()
    om = OracleMesh(mesh.dim, mesh.verts, mesh.cells, mesh.periodic, p=kw["p"])
    orp, ocol = om.stencils(kw["n_lo"], kw["n_hi"])
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)
    inf = w.info()
    assert inf["h"] == pytest.approx(om.h, rel=1e-13)
    assert inf["min_stencil"] >= min(kw["n_lo"], inf["m"])
    assert inf["max_stencil"] <= kw["n_hi"]


def test_info_sizes(lib):
    w = _host_ctx(jittered_square(10, 0.3, 5), p=3, n_lo=12, n_hi=20)
    inf = w.info()
    assert (inf["dim"], inf["m"], inf["faces_per_cell"], inf["points_per_face"], inf["n_vars"]) == (2, 6, 3, 2, 1)
    w = _host_ctx(periodic_line(30, 0.1, 5), p=5, n_lo=7, n_hi=7)
    inf = w.info()
    assert (inf["dim"], inf["m"], inf["faces_per_cell"], inf["points_per_face"]) == (1, 5, 2, 1)
    assert inf["min_insphere"] == pytest.approx(np.min(np.diff(periodic_line(30, 0.1, 5).verts[:, 0])))


def test_error_paths(lib):
    from paper_1602_02694_amd import WLSENO, WLSENOError

    mesh = jittered_square(6, 0.3, 9)
    # inverted cell
    bad = mesh.cells.copy()
    bad[3, [0, 1]] = bad[3, [1, 0]]
    w = WLSENO(device=-1)
    with pytest.raises(WLSENOError) as e:
        w.mesh_upload(2, mesh.verts, bad)
    assert e.value.status == 1 and "cell 3" in str(e.value)
    # vertex id out of range
    bad = mesh.cells.copy()
    bad[0, 0] = 10 ** 6
    with pytest.raises(WLSENOError) as e:
        w.mesh_upload(2, mesh.verts, bad)
    assert e.value.status == 1
    # empty mesh
    with pytest.raises(WLSENOError) as e:
        w.mesh_upload(2, np.zeros((0, 2)), np.zeros((0, 3), dtype=np.int32))
    assert e.value.status == 1 and "at least one cell" in str(e.value)
    # a square whose opposite sides do not match is no torus
    with pytest.raises(WLSENOError) as e:
        w.mesh_upload(2, mesh.verts, mesh.cells, periodic=True)
    assert "no partner" in str(e.value)
    # periodic flags outside their dimension
    cube = jittered_cube(3, 0.0, 1)
    with pytest.raises(WLSENOError):
        w.mesh_upload(3, cube.verts, cube.cells, periodic=True)
    # stencil before mesh / reversed size rule / too few coefficients
    w2 = WLSENO(device=-1)
    with pytest.raises(WLSENOError) as e:
        w2.stencil_build()
    assert e.value.status == 4
    w.mesh_upload(2, mesh.verts, mesh.cells)
    with pytest.raises(WLSENOError):
        w.stencil_build(p=3, n_lo=20, n_hi=12)
    with pytest.raises(WLSENOError):
        w.stencil_build(p=3, n_lo=4, n_hi=5)        # n_hi < m = 6
    # a 2-cell mesh cannot hold a 6-coefficient stencil
    w3 = WLSENO(device=-1)
    w3.mesh_upload(2, np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]]), np.array([[0, 1, 2], [1, 3, 2]]))
    with pytest.raises(WLSENOError) as e:
        w3.stencil_build(p=3, n_lo=6, n_hi=10)
    assert e.value.status == 1 and "fewer than" in str(e.value)
    # characteristic fields belong to the Euler system
    with pytest.raises(WLSENOError) as e:
        w.stencil_build(p=3, n_lo=12, n_hi=20, flux="burgers", characteristic=True)
    assert e.value.status == 1 and "Euler" in str(e.value)
    w.stencil_build(p=3, n_lo=12, n_hi=20, flux="euler", characteristic=True)
    # and have no per-cell coefficients
    rc = lib.wlseno_reconstruct(w._h, C.c_void_p(16), C.c_void_p(32), None, None)
    assert rc == 1 and b"characteristic" in lib.wlseno_last_error(w._h)
    # boundary options: 0..3, the slip wall for the Euler system only
    with pytest.raises(WLSENOError):
        w.stencil_build(p=3, n_lo=12, n_hi=20, bc=4)
    with pytest.raises(WLSENOError) as e:
        w.stencil_build(p=3, n_lo=12, n_hi=20, flux="burgers", bc=3)
    assert "slip wall" in str(e.value)
    w.stencil_build(p=3, n_lo=12, n_hi=20, flux="euler", bc=3)
    w.stencil_build(p=3, n_lo=12, n_hi=20, flux="euler", bc=2, far_state=(1.0, 0.0, 0.0, 2.5))
    # balanced-stencil refit: scalar fluxes, compiled for p = 3
    with pytest.raises(WLSENOError) as e:
        w.stencil_build(p=3, n_lo=12, n_hi=20, flux="euler", balance=True)
    assert e.value.status == 1
    with pytest.raises(WLSENOError) as e:
        w.stencil_build(p=4, n_lo=18, n_hi=24, flux="burgers", balance=True)
    assert e.value.status == 5
    w.stencil_build(p=3, n_lo=12, n_hi=20, flux="burgers", balance=True)
    # h_mode and lf_alpha take 0 or 1
    with pytest.raises(WLSENOError):
        w.stencil_build(p=3, n_lo=12, n_hi=20, h_mode=2)
    with pytest.raises(WLSENOError):
        w.stencil_build(p=3, n_lo=12, n_hi=20, lf_alpha=2)
    # eps h^2 keeps the WLS-ENO weights finite: eps = 0 only with unit weights
    with pytest.raises(WLSENOError) as e:
        w.stencil_build(p=3, n_lo=12, n_hi=20, eps=0.0)
    assert e.value.status == 1 and "eps > 0" in str(e.value)
    w.stencil_build(p=3, n_lo=12, n_hi=20, eps=0.0, weight_mode=1)
    # device call on a host-only context
    w.stencil_build(p=3, n_lo=12, n_hi=20)
    rc = lib.wlseno_rhs(w._h, C.c_void_p(16), C.c_void_p(32))
    assert rc == 4
    # facet shared by three triangles
    v = np.array([[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.6, 0.9]], dtype=float)
    cells = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]])
    with pytest.raises(WLSENOError) as e:
        w.mesh_upload(2, v, cells)
    assert "more than two" in str(e.value)


def test_numeric_check_option_host():
    """The numeric check is a context option: it can be set on a host-only
    context (whose device calls still return ESTATE), and ENUMERIC has its
    own status code."""
    from paper_1602_02694_amd import WLSENO, WLSENOError, _native

    assert _native.STATUS_NAMES[_native.WLSENO_ENUMERIC] == "ENUMERIC"
    w = WLSENO(device=-1)
    w.set_numeric_check(True)
    w.set_numeric_check(False)
    m = jittered_square(6, 0.3, 3403)
    w.mesh_upload(2, m.verts, m.cells)
    w.stencil_build(p=3, n_lo=12, n_hi=20)
    # device pointers are never touched on a host-only context
    assert w._lib.wlseno_rhs(w._h, C.c_void_p(8), C.c_void_p(16)) == 4
    assert b"host-only" in w._lib.wlseno_last_error(w._h)


def test_null_context_and_create_errors(lib):
    assert lib.wlseno_rhs(None, None, None) == 1
    h = C.c_void_p()
    assert lib.wlseno_create(-5, None, C.byref(h)) == 1
    assert b"device" in lib.wlseno_last_error(None)
    # a host-only context takes no stream
    assert lib.wlseno_create(-1, C.c_void_p(1), C.byref(h)) == 1
    assert b"no stream" in lib.wlseno_last_error(None)
    assert lib.wlseno_destroy(None) == 0


def test_batch_stencils_are_the_meshes_own(lib):
    """A batch's stencils are each mesh's own (oracle builder), with cell ids
    offset by the cells of the meshes before it; n_mesh and each mesh's h."""
    from oracle.mesh import OracleMesh
    from paper_1602_02694_amd import WLSENO, WLSENOError

    meshes = [jittered_square(n, 0.3, 700 + n) for n in (7, 11, 5)]
    w = WLSENO(device=-1)
    for k, m in enumerate(meshes):
        assert w.batch_add_mesh(2, m.verts, m.cells) == k
    w.stencil_build(p=3, n_lo=12, n_hi=20)
    inf = w.info()
    assert inf["n_mesh"] == 3 and inf["n_cell"] == sum(m.n_cell for m in meshes)
    rp, col = w.stencil()
    off = 0
    for m in meshes:
        om = OracleMesh(2, m.verts, m.cells, p=3)
        orp, ocol = om.stencils(12, 20)
        seg = slice(rp[off], rp[off + m.n_cell])
        assert np.array_equal(np.diff(rp[off:off + m.n_cell + 1]), np.diff(orp))
        assert np.array_equal(col[seg], ocol + off)
        off += m.n_cell
    # a mesh of another dimension joins as a group of its own, with its own
    # parameters; stencils stay each mesh's own, in add order
    cube = jittered_cube(4, 0.15, 9)
    assert w.batch_add_mesh(3, cube.verts, cube.cells) == 3
    w.batch_add_mesh(2, meshes[1].verts, meshes[1].cells)
    w.batch_params(3, p=2, n_lo=8, n_hi=16)
    w.stencil_build(p=3, n_lo=12, n_hi=20)
    inf = w.info()
    assert inf["n_mesh"] == 5 and inf["dim"] == 0 and inf["m"] == 0
    assert inf["n_cell"] == sum(m.n_cell for m in meshes) + cube.n_cell + meshes[1].n_cell
    rp, col = w.stencil()
    off = 0
    for m, dim, kw in [(x, 2, (3, 12, 20)) for x in meshes] + [(cube, 3, (2, 8, 16)), (meshes[1], 2, (3, 12, 20))]:
        om = OracleMesh(dim, m.verts, m.cells, p=kw[0])
        orp, ocol = om.stencils(kw[1], kw[2])
        assert np.array_equal(np.diff(rp[off:off + m.n_cell + 1]), np.diff(orp))
        assert np.array_equal(col[rp[off]:rp[off + m.n_cell]], ocol + off)
        off += m.n_cell
    with pytest.raises(WLSENOError) as e:
        w.batch_params(4, p=3)
    assert e.value.status == 1
    # a single upload replaces the batch
    w.mesh_upload(2, meshes[0].verts, meshes[0].cells)
    w.stencil_build(p=3, n_lo=12, n_hi=20)
    assert w.info()["n_mesh"] == 1 and w.info()["n_cell"] == meshes[0].n_cell
