"""GPU parity at the benchmark sizes, checked on sampled cells.

The GPU runs the whole mesh with the automatic lane count and the direct
launches of the reconstruction and update kernels that the benchmark's stages
make.  The oracle cannot build stencils for millions of cells within a test,
so it runs on the sub-mesh of every cell within R vertex rings of a seeded
sample (random cells and cells on the domain boundary; tests/submesh.py).
The sampled cells' stencils are compared as integers, mapped back to
full-mesh numbering, which shows R was enough; their facet values,
polynomials and right-hand sides then meet the parity rule of
tests/parity.py.

A right-hand side with the global Lax-Friedrichs alpha (Burgers, Euler) needs
every cell's facet values.  On the 2 M-triangle mesh it is compared with the
local alpha per facet point, which runs the same reconstruction; the 64-mesh
Euler batch runs at full size and three of its meshes (global alpha per mesh)
are compared against their own whole-mesh oracles: the smallest at every
cell, the median and the largest at sampled cells.
"""

import numpy as np
import pytest

from parity import (assert_parity, assert_poly_parity, cell_conditions, cell_noise, flux_scale, floor_tol,
                    momentum_scale, neighbourhood_max)
from submesh import SubOracle, sample_cells
from workloads import configs, fields, jittered_cube, jittered_square

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)


def _check_sample(w, u_dev, sub, name, rhs=True):
    """Stencils, ranks, facet values, polynomials and (optionally) the
    right-hand side of the sampled cells against the sub-mesh oracle."""
    torch = _torch()
    sample = sub.keep[sub.loc]
    o, ox, loc = sub.o, sub.ox, sub.loc
    rp, col = w.stencil()
    rows = sub.stencil_rows()
    for i, r in zip(sample, rows):
        assert np.array_equal(col[rp[i]:rp[i + 1]], r), f"{name}: stencil of cell {i} differs"
    idx = torch.tensor(sample, device=u_dev.device)
    rec = w.reconstruct(u_dev)
    g_fv = rec["fval"][:, idx].cpu().numpy()
    g_rank = rec["rank"][:, idx].cpu().numpy()
    g_coef = rec["coef"][:, idx].cpu().numpy()
    del rec
    ref, refx = o.reconstruct(sub.u), ox.reconstruct(sub.u)
    assert np.array_equal(g_rank, ref["rank"][:, loc]), f"{name}: numerical ranks differ"
    kappa, kappa_nb = sub.kappas()
    euler = o.flux == "euler"
    fsc = momentum_scale(ref["fval"], o.dim) if euler else None
    # the 1% floor of each field is its magnitude over the whole sub-mesh
    mx = np.max(np.abs(ref["fval"]), axis=(1, 2, 3), keepdims=True)
    sc = np.broadcast_to(1e-2 * mx, ref["fval"].shape)
    if fsc is not None:
        sc = np.maximum(sc, fsc)
    noise = cell_noise(ref["fval"], refx["fval"], scale=sc, cell_axes=2)
    err = assert_parity(g_fv, ref["fval"][:, loc], f"{name} facet values", scale=sc[:, loc],
                        tol_floor=floor_tol(kappa[:, loc, None, None], noise[:, loc]))
    _say(f"[{name}] facet values of {len(sample)} cells: worst {err:.2e}")
    G = np.zeros_like(ref["coef"])
    G[:, loc] = g_coef
    Rf = np.zeros_like(ref["coef"])
    Rf[:, loc] = ref["coef"][:, loc]
    X = np.zeros_like(refx["coef"])
    X[:, loc] = refx["coef"][:, loc]
    assert_poly_parity(G, Rf, o, sub.u, f"{name} polynomials", xcoef=X, tol_floor=floor_tol(kappa))
    if not rhs:
        return
    L = w.rhs(u_dev)
    V = o.nvars
    g_L = L.reshape(V, -1)[:, idx].cpu().numpy()
    Lo, alpha_o = o.rhs(sub.u)
    Lx, _ = ox.rhs(sub.u)
    Lo, Lx = Lo.reshape(V, -1), Lx.reshape(V, -1)
    S = np.asarray(flux_scale(o, ref["fval"], alpha_o)).reshape(V, -1)
    tol = floor_tol(kappa_nb.reshape(V, -1)[:, loc], cell_noise(Lo, Lx, scale=S)[:, loc])
    err = assert_parity(g_L, Lo[:, loc], f"{name} rhs", scale=S[:, loc], tol_floor=tol)
    _say(f"[{name}] rhs of {len(sample)} cells: worst {err:.2e}")


def _gpu(mesh, **kw):
    from paper_1602_02694_amd import WLSENO

    w = WLSENO(device=0)
    w.mesh_upload(mesh.dim, mesh.verts, mesh.cells, mesh.periodic)
    w.stencil_build(**kw)
    return w


def test_square_large_burgers_sampled():
    """2 M triangles (the 1000 x 1000-point benchmark mesh), Burgers p = 3."""
    torch = _torch()
    mesh = jittered_square(1000, 0.3, 2002)
    u0 = fields.cell_averages(mesh, fields.gaussian_bump_with_step_2d)
    _say(f"[case] square-large burgers: n_cell={mesh.n_cell}")
    kw = dict(p=3, n_lo=12, n_hi=20, flux="burgers")
    sample = sample_cells(mesh, 48, 16, 9101)
    u = torch.tensor(u0, device="cuda")
    w = _gpu(mesh, **kw)
    sub = SubOracle(mesh, u0, sample, 4, **kw)
    _check_sample(w, u, sub, "square-large global alpha", rhs=False)
    a = w.last_alpha()
    assert np.isfinite(a) and a > 0
    del w
    w = _gpu(mesh, lf_alpha=1, **kw)
    sub = SubOracle(mesh, u0, sample, 4, lf_alpha=1, **kw)
    _check_sample(w, u, sub, "square-large local alpha")


def test_cube_advection_sampled():
    """409 k tetrahedra (a 40^3 lattice), advection p = 3, 30-50 cell stencils."""
    torch = _torch()
    mesh = jittered_cube(40, 0.15, 4001)
    u0 = fields.cell_averages(mesh, fields.sine_with_sphere_3d)
    _say(f"[case] cube40 advection: n_cell={mesh.n_cell}")
    kw = dict(p=3, n_lo=30, n_hi=50, flux="advection", velocity=(1.0, 0.5, 0.25))
    sample = sample_cells(mesh, 24, 8, 9102)
    u = torch.tensor(u0, device="cuda")
    w = _gpu(mesh, **kw)
    sub = SubOracle(mesh, u0, sample, 3, **kw)
    _check_sample(w, u, sub, "cube40")


def test_cube_full_size_sampled():
    """The 3-D benchmark mesh itself: a Delaunay tetrahedralisation of the
    jittered 74^3 lattice (2,681,294 tetrahedra), advection p = 3, 30-50 cell
    stencils, sine plus sphere data; 32 sampled cells (random and on the
    boundary) against the sub-mesh oracle.  Generating the mesh takes the
    host about two minutes."""
    import time

    torch = _torch()
    t = time.time()
    wl = configs.cube_advection(74, 4001)
    mesh, u0, s = wl.mesh, wl.u0, wl.settings
    _say(f"[case] cube74 advection: n_cell={mesh.n_cell} (mesh and averages in {time.time() - t:.0f}s)")
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux=s["flux"], velocity=s["velocity"])
    sample = sample_cells(mesh, 24, 8, 9105)
    u = torch.tensor(u0, device="cuda")
    w = _gpu(mesh, **kw)
    _say(f"[case] cube74: library set up at {time.time() - t:.0f}s")
    sub = SubOracle(mesh, u0, sample, 3, **kw)
    _check_sample(w, u, sub, "cube74")


def test_adjoint_workload_sampled():
    """The adjoint workload's 200 k triangles (advection p = 3, zero outside
    state): sampled facet values and rhs, and <J(u)^T x, d> with x on the
    sampled cells against central differences of the oracle's rhs."""
    torch = _torch()
    wl = configs.square_advection_adjoint()
    mesh, u0 = wl.mesh, wl.u0
    s = wl.settings
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux=s["flux"], velocity=s["velocity"], bc=s["bc"])
    _say(f"[case] adjoint workload: n_cell={mesh.n_cell}")
    sample = sample_cells(mesh, 48, 16, 9103)
    u = torch.tensor(u0, device="cuda")
    w = _gpu(mesh, **kw)
    sub = SubOracle(mesh, u0, sample, 4, **kw)
    _check_sample(w, u, sub, "adjoint workload")
    rng = np.random.default_rng(9104)
    x = np.zeros(mesh.n_cell)
    x[sample] = rng.standard_normal(len(sample))
    d = rng.standard_normal(mesh.n_cell)
    b = float(np.dot(w.rhs_vjp(u, torch.tensor(x, device="cuda")).cpu().numpy(), d))
    ds, xs = d[sub.keep], x[sub.keep]
    # h small enough that no sampled cell crosses a switch of its smallest
    # facet indicator within +-h (at 4x this h one of them does, and its
    # difference quotient is off by 2e-3)
    h = 2.5e-6 * np.max(np.abs(u0)) / np.max(np.abs(d))

    def D(hh):
        Lp, _ = sub.o.rhs(sub.u[0] + hh * ds)
        Lm, _ = sub.o.rhs(sub.u[0] - hh * ds)
        return xs[sub.loc] * (Lp[0] - Lm[0])[sub.loc] / (2 * hh)

    terms = (4.0 * D(h / 2) - D(h)) / 3.0              # x_i (J d)_i, Richardson-extrapolated
    a = float(np.sum(terms))
    _say(f"[adjoint workload] <J^T x, d> {b:.12e}, oracle differences {a:.12e}")
    assert abs(a - b) <= 1e-6 * float(np.sum(np.abs(terms)))


def test_euler_batch_full_size():
    """All 64 meshes of the Euler batch (1.26 M cells, p = 4) in one set of
    launches; the smallest, the median and the largest mesh compared whole
    against their own oracles (rhs and alpha per mesh)."""
    torch = _torch()
    import oracle
    from paper_1602_02694_amd import WLSENO

    wls = configs.batched_euler()
    sizes = np.array([x.mesh.n_cell for x in wls])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    _say(f"[case] euler batch: {len(wls)} meshes, {offs[-1]} cells")
    kw = dict(p=4, n_lo=20, n_hi=36, flux="euler")
    wb = WLSENO(device=0)
    for x in wls:
        wb.batch_add_mesh(2, x.mesh.verts, x.mesh.cells)
    wb.stencil_build(**kw)
    ub = torch.tensor(np.concatenate([x.u0 for x in wls], axis=1).reshape(-1), device="cuda")
    Lb = wb.rhs(ub).cpu().numpy().reshape(4, -1)
    ab = wb.batch_last_alpha()
    order = np.argsort(sizes, kind="stable")
    for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        whole = k == int(order[0])
        m, u0 = wls[k].mesh, wls[k].u0
        o = oracle.Oracle(2, m.verts, m.cells, False, **kw)
        ox = oracle.Oracle(2, m.verts, m.cells, False, extended=True, stencil=(o.row_ptr, o.col), **kw)
        ref = o.reconstruct(u0)
        Lo, alpha_o = o.rhs(u0)
        Lx, _ = ox.rhs(u0)
        assert ab[k] == pytest.approx(alpha_o, rel=1e-12), f"mesh {k} alpha"
        # the smallest mesh whole; the others at their 64 largest |rhs| cells
        # and a seeded sample (kappa is costly on the CPU)
        rng = np.random.default_rng(9105 + k)
        pick = np.arange(m.n_cell) if whole else np.unique(np.concatenate(
            [np.argsort(-np.abs(Lo).max(axis=0))[:64], rng.choice(m.n_cell, 64, replace=False)]))
        nb = o.mesh.nbr[pick]
        need = np.unique(np.concatenate([pick, nb[nb >= 0]]))
        kap = cell_conditions(o, u0, cells=need)
        kap_nb = np.broadcast_to(neighbourhood_max(o, kap.max(axis=0, keepdims=True)), kap.shape)
        S = np.asarray(flux_scale(o, ref["fval"], alpha_o)).reshape(4, -1)
        g = Lb[:, offs[k]:offs[k + 1]]
        tol = floor_tol(kap_nb[:, pick], cell_noise(Lo, Lx, scale=S)[:, pick])
        err = assert_parity(g[:, pick], Lo[:, pick], f"batch mesh {k} rhs", scale=S[:, pick], tol_floor=tol)
        _say(f"[euler batch] mesh {k} ({m.n_cell} cells): rhs of {len(pick)} cells, worst {err:.2e}")


def test_adjoint_c5_exact_tangent():
    """The 100-step adjoint on the full 200 k-triangle adjoint workload
    against the oracle's exact tangent (its own code on dual numbers).

    The WLS-ENO tangent of this workload grows about 10^12-fold over the 100
    steps (measured on the oracle alone), so two FP64 trajectories from the
    same start drift apart by ~1e-4 and no whole-horizon comparison is
    meaningful.  The check therefore follows the GPU's own trajectory: for
    every step k the oracle's tangent from the GPU's state u_k gives
    <g_{k+1}, J_k d>, which must equal <g_k, d> for the GPU's one-step adjoint
    g_k (8 seeded directions, 1e-6 relative).  The one-step adjoints compose
    bit for bit into the 100-step call with checkpoints every 10 steps."""
    torch = _torch()
    import oracle

    wl = configs.square_advection_adjoint(317, 5001)
    mesh, s = wl.mesh, wl.settings
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux="advection", velocity=s["velocity"], bc=s["bc"])
    w = _gpu(mesh, **kw)
    dt = 0.5 * w.info()["min_insphere"] / float(np.hypot(*s["velocity"][:2]))
    ot = oracle.Oracle(2, mesh.verts, mesh.cells, tangent=True, **kw)
    D = np.random.default_rng(5003).standard_normal((8, mesh.n_cell))
    n = 100
    u = torch.tensor(wl.u0, device="cuda")
    states = [u.clone()]
    for _ in range(n):
        w.step(u, dt, 1)
        states.append(u.clone())
    gT = torch.tensor(states[-1].cpu().numpy() - s["target"], device="cuda")
    g = [None] * (n + 1)
    g[n] = gT
    for k in range(n - 1, -1, -1):
        g[k] = w.step_adjoint(states[k], dt, 1, g[k + 1], 10)
    full = w.step_adjoint(states[0], dt, n, gT, 10)
    torch.cuda.synchronize()
    assert torch.equal(g[0], full)
    worst = 0.0
    for k in range(n):
        _, JD = ot.step_tangent(states[k].cpu().numpy(), D, dt, 1)
        gk, gk1 = g[k].cpu().numpy(), g[k + 1].cpu().numpy()
        for j in range(D.shape[0]):
            a, b = float(gk @ D[j]), float(gk1 @ JD[j])
            worst = max(worst, abs(a - b) / abs(b))
        if k % 10 == 9:
            _say(f"[case] adjoint c5 exact tangent: step {k + 1}, worst {worst:.3e}, "
                 f"|g_k| {float(torch.linalg.norm(g[k])):.3e}")
    assert worst <= 1e-6
