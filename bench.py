"""Benchmark of the WLS-ENO finite-volume path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload square|square-large|cube|batch]

One "step" is one third-order TVD Runge-Kutta step of the whole hot path
(three right-hand sides: reconstruction, Lax-Friedrichs flux, update) over the
whole mesh.  The default workload is the 2-D Burgers problem on a Delaunay
triangulation of a 100x100 jittered lattice (19,602 triangles, p = 3,
12-20 cell stencils, FP64).  Inputs are resident in device memory before the
timed region starts.

Prints one JSON line: throughput in cell-updates/s (cells x steps / s), a
roofline entry for the dominant kernel (the reconstruction, FP64-ALU bound)
and one for the flux/update kernel (HBM bound), both event-timed in this run,
and the FP64 CPU oracle timed on a bounded sample of the same workload on the
host's cores, together with the GPU-vs-oracle parity of that sample.
`--workload square-large` runs the 1000x1000-point companion mesh (~2.0 M
triangles) on which HBM traffic is measured (profiles/traffic.json holds the
calibrated rocprofv3 FETCH_SIZE/WRITE_SIZE per launch, valid while the kernel
source hash matches).  `--workload cube` runs 2.68 M tetrahedra (p = 3,
linear advection); `--workload batch` runs 64 independent 2-D Euler meshes
(p = 4, ~1.25 M cells) as one batch and, for comparison, one context per
mesh (`per_mesh_loop`).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 128 FP64 flop/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s (p=3, 2-D tri, FP64) at 1e-12 vs oracle"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def recon_flops(n, m, dim, F, Q):
    """Algorithmic FP64 operations of one cell reconstruction (an FMA counts 2).

    Row construction from gathered centroid offsets and moments, weights (one
    division each), W A and W u, column norms/scaling, Householder QR with
    exactly recomputed pivot norms (pivot norms 2(n-k)(m-k), reflector
    application to the trailing columns and the right-hand side 4(n-k)(m-k)),
    back substitution, and evaluation at the F*Q facet points."""
    n = np.asarray(n, dtype=np.float64)
    build = n * (dim + 2 * (m - 1))
    weights = 4 * n
    form = n * (m + 1)
    scale = 3 * n * m + 2 * m
    qr = sum(6 * (n - k) * (m - k) + (n - k) + 6 for k in range(m))
    back = m * m + m
    evalf = F * Q * 3 * m
    return build + weights + form + scale + qr + back + evalf


def update_bytes(nc, dim, F, Q, V=1):
    """Compulsory HBM bytes of one flux/update launch: sibling ids (4F),
    area-scaled normals (8 F dim), the cell's own facet values (8 F Q per
    component; the neighbour's copy of a facet value is counted once, as its
    own), 1/|tau|, the state and stage inputs (one array in the first RK
    stage, two in the others: 8 x 4/3 on average) and the output, per
    component."""
    return nc * (4 * F + 8 * F * dim + 8 + V * (8 * F * Q + 8 * 4.0 / 3.0 + 8))


def traffic_record(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters, if the record
    matches the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1602_02694_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        entry = rec.get(workload, {}).get(kernel)
        if entry and entry.get("kernels_sha256") == digest:
            return entry.get("bytes_per_launch")
    except Exception:
        return None
    return None


# name -> (mesh builder, initial data, settings)
WORKLOADS = {
    "square": dict(dim=2, side=100, seed=2001, p=3, n_lo=12, n_hi=20, flux="burgers", velocity=(0, 0, 0),
                   metric=METRIC),
    "square-large": dict(dim=2, side=1000, seed=2002, p=3, n_lo=12, n_hi=20, flux="burgers",
                         velocity=(0, 0, 0), metric=METRIC),
    "cube": dict(dim=3, side=74, seed=4001, p=3, n_lo=30, n_hi=50, flux="advection",
                 velocity=(1.0, 0.5, 0.25), metric="cell-updates/s (p=3, 3-D tet, FP64) at 1e-12 vs oracle"),
}


def make_workload(name, side=0):
    """Mesh and initial cell averages, built in two logged phases (side > 0:
    that many lattice points per side instead of the workload's own)."""
    from workloads import fields, jittered_cube, jittered_square
    from workloads.configs import Workload

    cfg = dict(WORKLOADS[name])
    if side:
        cfg["side"] = int(side)
    t = time.time()
    if cfg["dim"] == 2:
        mesh = jittered_square(cfg["side"], 0.3, cfg["seed"])
    else:
        mesh = jittered_cube(cfg["side"], 0.15, cfg["seed"])
    log(f"[bench] mesh: {mesh.n_cell} cells in {time.time() - t:.1f}s")
    t = time.time()
    fn = fields.gaussian_bump_with_step_2d if cfg["dim"] == 2 else fields.sine_with_sphere_3d
    u0 = fields.cell_averages(mesh, fn)
    kind = "burgers" if cfg["flux"] == "burgers" else "advection"
    shape = "tri" if cfg["dim"] == 2 else "tet"
    log(f"[bench] initial averages in {time.time() - t:.1f}s")
    return Workload(f"{shape}{mesh.n_cell}-{kind}-p{cfg['p']}", mesh, u0, dict(cfg))


def insphere_diameters(mesh):
    """2 dim |tau| / |d tau| per cell (the CFL length), from the vertices."""
    v = mesh.verts[mesh.cells]                                  # (nc, d+1, d)
    d = mesh.dim
    if d == 2:
        e = [v[:, 1] - v[:, 0], v[:, 2] - v[:, 1], v[:, 0] - v[:, 2]]
        area = 0.5 * np.abs(e[0][:, 0] * (-e[2][:, 1]) - e[0][:, 1] * (-e[2][:, 0]))
        per = sum(np.linalg.norm(x, axis=1) for x in e)
        return 4.0 * area / per
    raise ValueError("2-D meshes only")


def run_batch(args, torch, WLSENO):
    """The batched Euler workload: 64 meshes stepped by one set of launches per
    stage, against the same meshes stepped one context at a time."""
    from workloads import configs

    t = time.time()
    wls = configs.batched_euler(64, 3001)
    cells = [w.mesh.n_cell for w in wls]
    log(f"[bench] 64 meshes, {sum(cells)} cells ({min(cells)}-{max(cells)}) in {time.time() - t:.1f}s")
    s0 = wls[0].settings
    kw = dict(p=s0["p"], n_lo=s0["n_lo"], n_hi=s0["n_hi"], flux="euler", gamma=s0["gamma"],
              characteristic=bool(args.characteristic))
    t = time.time()
    wb = WLSENO(device=0)
    for w in wls:
        wb.batch_add_mesh(2, w.mesh.verts, w.mesh.cells)
    wb.stencil_build(**kw)
    info = wb.info()
    log(f"[bench] batch setup {time.time() - t:.1f}s")
    u0 = np.concatenate([w.u0 for w in wls], axis=1)
    u_init = torch.tensor(u0.reshape(-1), device="cuda")
    tune = wb.autotune(u_init)
    log(f"[bench] autotuned reconstruction: {tune['chosen']} lanes per cell "
        f"({', '.join(f'{k}: {v:.1f} us' for k, v in tune['timings_us'].items())})")
    wb.rhs(u_init)
    alphas = wb.batch_last_alpha()
    dts = np.array([0.5 * insphere_diameters(w.mesh).min() / a for w, a in zip(wls, alphas)])
    # batched: warm-up, then K steps timed
    u = u_init.clone()
    wb.batch_step(u, dts, args.warmup)
    torch.cuda.synchronize()
    u = u_init.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    wb.batch_step(u, dts, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    nc = int(info["n_cell"])
    value = nc * args.steps / elapsed
    log(f"[bench] batch: {args.steps} steps in {elapsed * 1e3:.2f} ms -> {value:.4g} cell-updates/s")
    # the same meshes, one context each, stepped one after another
    singles = []
    for w, dt in zip(wls, dts):
        c = WLSENO(device=0)
        c.mesh_upload(2, w.mesh.verts, w.mesh.cells)
        c.stencil_build(**kw)
        ui = torch.tensor(w.u0.reshape(-1), device="cuda")
        c.autotune(ui)
        singles.append((c, ui, dt))
    for c, ui, dt in singles:
        c.step(ui.clone(), dt, args.warmup)
    torch.cuda.synchronize()
    work = [ui.clone() for _, ui, _ in singles]
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for (c, _, dt), ui in zip(singles, work):
        c.step(ui, dt, args.steps)
    torch.cuda.synchronize()
    el_loop = time.perf_counter() - ts
    log(f"[bench] per-mesh loop: {el_loop * 1e3:.2f} ms -> {nc * args.steps / el_loop:.4g} cell-updates/s")
    ub = u.reshape(4, -1)
    off = 0
    same = True
    for ui, w in zip(work, wls):
        n = w.mesh.n_cell
        same = same and bool(torch.equal(ui.reshape(4, -1), ub[:, off:off + n]))
        off += n
    k1 = wb.time_kernel(0, u_init, 3 * args.steps)
    k2 = wb.time_kernel(1, u_init, 3 * args.steps)
    rp, _ = wb.stencil()
    nsz = np.diff(rp)
    F, Q, m = info["faces_per_cell"], info["points_per_face"], info["m"]
    if args.characteristic:
        # per facet and field: one fit evaluated at that facet's points, the
        # projection of the stencil and facet-neighbour averages (4 FMA each),
        # the eigenvectors (~40 flop) and the map back (4 FMA per point)
        per = recon_flops(nsz, m, 2, 1, Q) + 8.0 * (nsz + F + 1) + 40.0 + 8.0 * Q
        flops = 4.0 * F * float(np.sum(per))
    else:
        flops = 4.0 * float(np.sum(recon_flops(nsz, m, 2, F, Q)))
    achieved = flops / (k1 * 1e-3) / 1e12
    log(f"[bench] k_reconstruct avg {k1 * 1e3:.2f} us, k_update avg {k2 * 1e3:.2f} us; "
        f"{flops / nc:.0f} flop/cell")
    wkey = "batch-char" if args.characteristic else "batch"
    ub_bytes = update_bytes(nc, 2, F, Q, V=4)
    ach_u = ub_bytes / (k2 * 1e-3) / 1e9
    return {
        "metric": "cell-updates/s (p=4, 2-D Euler, 64-mesh batch, FP64)" if not args.characteristic else
                  "cell-updates/s (p=4, 2-D Euler in characteristic fields, 64-mesh batch, FP64)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batch64-euler{'-char' if args.characteristic else ''}-p4-{nc}",
            "reconstruction": "characteristic fields per facet" if args.characteristic else "conserved components",
            "mesh": "64 Delaunay triangulations of jittered lattices, 5k-50k cells each (log-uniform, seed 3001)",
            "n_cell": nc,
            "p": 4,
            "stencil_cells": [int(nsz.min()), int(nsz.max())],
            "flux": "2-D Euler (gamma 1.4), per-mesh global Lax-Friedrichs alpha, quadrant Riemann data",
            "time_integrator": "TVD RK3, per-mesh dt, HIP-graph replay",
        },
        "autotune": tune,
        "per_mesh_loop": {"value": nc * args.steps / el_loop, "ms_per_step": el_loop * 1e3 / args.steps,
                          "batch_speedup": el_loop / elapsed, "bitwise_equal_to_batch": same},
        "roofline": {"bound": "alu", "kernel": "k_reconstruct", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic_record(f"k_reconstruct/{tune['chosen']}", wkey), "avg_launch_us": k1 * 1e3,
                     "flops_per_launch": flops},
        "roofline_update": {"bound": "hbm", "kernel": "k_update", "achieved": ach_u, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": ach_u / HBM_PEAK_GBS,
                            "traffic": traffic_record("k_update", wkey), "avg_launch_us": k2 * 1e3,
                            "bytes_per_launch": ub_bytes},
    }


def parity_stats(g, o, tol=1e-12, scale=None):
    """GPU values g against oracle values o: per entry |g - o| / max(|o|,
    1e-2 max|o|) (the floor keeps zeros of a field from making a relative
    error ill-posed; `scale`, if given, raises it further) -- its maximum,
    99.9th percentile and count above tol -- and the norm-wise relative
    error."""
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    o = np.asarray(o, dtype=np.float64).reshape(-1)
    scale0 = np.maximum(np.abs(o), 1e-2 * np.max(np.abs(o)))
    scale = scale0 if scale is None else np.maximum(scale0, np.asarray(scale, dtype=np.float64).reshape(-1))
    r = np.abs(g - o) / scale
    return {"max_rel_err_vs_oracle": float(r.max()), "p99_9_rel_err": float(np.percentile(r, 99.9)),
            "count_above_tolerance": int((r > tol).sum()), "entries": int(r.size),
            "normwise_rel_err": float(np.linalg.norm(g - o) / np.linalg.norm(o)), "tolerance": tol,
            "pass": bool(r.max() <= tol)}


def sampled_parity(torch, w, wl, u_dev, kw, n_random=24, n_boundary=8, R=3, seed=9105):
    """Parity of a mesh too large for the whole-mesh oracle: seeded random and
    boundary cells against the FP64 oracle on the sub-mesh of every cell
    within R vertex rings of them (the oracle helpers of the test suite; on
    small meshes that sub-mesh oracle equals the whole-mesh one bit for bit at
    the sampled cells): stencils, facet values and right-hand sides, and the
    oracle's time for one RK3 step of the sub-mesh."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from submesh import SubOracle, sample_cells
    import oracle

    t0 = time.perf_counter()
    mesh = wl.mesh
    sample = sample_cells(mesh, n_random, n_boundary, seed)
    sub = SubOracle(mesh, wl.u0, sample, R, **kw)
    rp, col = w.stencil()
    same = all(np.array_equal(col[rp[i]:rp[i + 1]], r) for i, r in zip(sample, sub.stencil_rows()))
    idx = torch.tensor(sample, device=u_dev.device)
    fv = w.reconstruct(u_dev)["fval"][:, idx].cpu().numpy()
    L = w.rhs(u_dev)
    L = L.reshape(sub.u.shape[0], -1)[:, idx].cpu().numpy()
    from parity import flux_scale

    rec_o = sub.o.reconstruct(sub.u)
    ref = rec_o["fval"][:, sub.loc]
    Lo, alpha_o = sub.o.rhs(sub.u)
    Lo = Lo.reshape(sub.u.shape[0], -1)[:, sub.loc]
    # L_i differences fluxes: its rounding is relative to the flux sum S_i
    S = np.asarray(flux_scale(sub.o, rec_o["fval"], alpha_o)).reshape(sub.u.shape[0], -1)[:, sub.loc]
    tt = time.perf_counter()
    sub.o.step(sub.u, 1e-4, 1)
    t_step = time.perf_counter() - tt
    rec = {"sampled_cells": int(len(sample)), "submesh_cells": int(len(sub.keep)), "stencils_equal": bool(same),
           "facet_values": parity_stats(fv, ref), "rhs": parity_stats(L, Lo, scale=S),
           "rhs_against_own_magnitude": parity_stats(L, Lo),
           "cpu_baseline": {"value": len(sub.keep) / t_step, "unit": "cell-updates/s",
                            "cores": oracle.core.num_threads(), "kind": "oracle",
                            "sample": f"one TVD RK3 step of the {len(sub.keep)}-cell sub-mesh"},
           "seconds": time.perf_counter() - t0}
    log(f"[bench] sampled parity, {len(sample)} cells (sub-mesh {len(sub.keep)}): stencils equal {same}; facet "
        f"values max {rec['facet_values']['max_rel_err_vs_oracle']:.2e}, rhs max "
        f"{rec['rhs']['max_rel_err_vs_oracle']:.2e} (norm-wise {rec['rhs']['normwise_rel_err']:.2e}); oracle "
        f"{rec['cpu_baseline']['value']:.3g} cell-updates/s")
    return rec


def run_line(torch, WLSENO):
    """1-D periodic line of 200 cells (widths +-20%), p = 3, linear advection
    of the sine + square wave, 100 TVD RK3 steps at CFL 0.5: GPU time, the
    FP64 oracle's time on the same steps, and their parity."""
    import oracle
    from workloads import configs

    wl = configs.line_advection(200, 1001)
    s = wl.settings
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux="advection", velocity=s["velocity"])
    w = WLSENO(device=0)
    w.mesh_upload(1, wl.mesh.verts, wl.mesh.cells, True)
    w.stencil_build(**kw)
    dt = s["cfl"] * w.info()["min_insphere"]
    u0 = torch.tensor(wl.u0, device="cuda")
    u = u0.clone()
    # a few untimed runs: this leg follows seconds of CPU-only oracle work,
    # and the first launch-bound runs after such a pause read up to 3x slower
    for _ in range(3):
        w.step(u, dt, s["steps"])
    torch.cuda.synchronize()
    u = u0.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    w.step(u, dt, s["steps"])
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - ts
    o = oracle.Oracle(1, wl.mesh.verts, wl.mesh.cells, True, **kw)
    ts = time.perf_counter()
    uo = o.step(wl.u0, dt, s["steps"])[0]
    t_cpu = time.perf_counter() - ts
    nc = wl.mesh.n_cell
    rec = {"workload": f"{wl.name}, {s['steps']} steps", "value": nc * s["steps"] / t_gpu,
           "unit": "cell-updates/s", "ms_per_step": t_gpu * 1e3 / s["steps"],
           "cpu_baseline": {"value": nc * s["steps"] / t_cpu, "cores": oracle.core.num_threads(), "kind": "oracle"},
           "parity": parity_stats(u.cpu().numpy(), uo)}
    log(f"[bench] line200: {rec['value']:.3g} cell-updates/s (launch-bound), oracle {rec['cpu_baseline']['value']:.3g}; "
        f"parity after {s['steps']} steps {rec['parity']['max_rel_err_vs_oracle']:.2e}")
    return rec


# compulsory HBM bytes per cell-stage of the 2-D p = 3 scalar path: averages
# in, state and stage buffers, stencil ids, geometry and moments, facet records
B_MIN_2D_P3 = 280.0


def run_square_large(torch, WLSENO, steps=20):
    """The 1000 x 1000-point companion of the benchmark mesh (~2.0 M
    triangles, same data and settings), where the working set far exceeds the
    256 MB last-level cache: throughput, event-timed kernels, their roofline
    fractions and the stage's algorithmic HBM fraction (cell-stages/s x 280 B
    compulsory bytes / 8 TB/s)."""
    t0 = time.time()
    wl = make_workload("square-large")
    cfg, mesh = wl.settings, wl.mesh
    w = WLSENO(device=0)
    w.mesh_upload(2, mesh.verts, mesh.cells)
    w.stencil_build(p=cfg["p"], n_lo=cfg["n_lo"], n_hi=cfg["n_hi"], flux=cfg["flux"])
    info = w.info()
    rp, _ = w.stencil()
    nsz = np.diff(rp)
    dt = 0.5 * info["min_insphere"] / (np.sqrt(2.0) * float(np.max(np.abs(wl.u0))))
    u0 = torch.tensor(wl.u0, device="cuda")
    tune = w.autotune(u0)
    u = u0.clone()
    w.step(u, dt, 4)
    u = u0.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    w.step(u, dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - ts
    nc = mesh.n_cell
    k1 = w.time_kernel(0, u0, 30)
    k2 = w.time_kernel(1, u0, 30)
    F, Q, m = info["faces_per_cell"], info["points_per_face"], info["m"]
    flops = float(np.sum(recon_flops(nsz, m, 2, F, Q)))
    ub = update_bytes(nc, 2, F, Q)
    stage_s = el / steps / 3.0
    alg = nc * B_MIN_2D_P3 / stage_s / 1e9
    rec = {"workload": f"{wl.name}, {steps} steps", "n_cell": nc, "value": nc * steps / el,
           "unit": "cell-updates/s", "ms_per_step": el * 1e3 / steps,
           "autotune": tune,
           "stage_hbm_algorithmic": {"bytes_per_cell_stage": B_MIN_2D_P3, "achieved_GBs": alg,
                                     "peak_GBs": HBM_PEAK_GBS, "frac": alg / HBM_PEAK_GBS},
           "k_reconstruct": {"avg_launch_us": k1 * 1e3, "achieved_TFLOPs": flops / (k1 * 1e-3) / 1e12,
                             "frac_fp64_peak": flops / (k1 * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                             "traffic": traffic_record(f"k_reconstruct/{tune['chosen']}", "square-large")},
           "k_update": {"avg_launch_us": k2 * 1e3, "algorithmic_bytes": ub,
                        "achieved_GBs": ub / (k2 * 1e-3) / 1e9, "frac_hbm_peak": ub / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": traffic_record("k_update", "square-large")},
           "seconds": time.time() - t0}
    log(f"[bench] square-large: {nc} cells, {rec['value']:.4g} cell-updates/s, stage HBM fraction (algorithmic) "
        f"{rec['stage_hbm_algorithmic']['frac']:.3f}; k_reconstruct {k1 * 1e3:.1f} us "
        f"({rec['k_reconstruct']['frac_fp64_peak']:.3f} of FP64), k_update {k2 * 1e3:.1f} us "
        f"({rec['k_update']['frac_hbm_peak']:.3f} of HBM); {rec['seconds']:.0f}s")
    return rec


def exact_tangent_check(torch, w, wl, dt, steps, ckpt, rng, ndir=8):
    """The adjoint against the oracle's exact tangent (its own code on dual
    numbers, exact on the active branch), step by step along the GPU's own
    trajectory: for every step k, <g_k, d> from the GPU's one-step adjoint
    against <g_{k+1}, J_k d> with J_k d the oracle's tangent from the GPU's
    state u_k, for ndir seeded directions.  The one-step adjoints compose bit
    for bit into the full checkpointed call.  Also reported: the growth of the
    gradient along the trajectory and the drift between the GPU's and the
    FP64 oracle's own 100-step trajectories, which that growth causes."""
    import oracle

    mesh, s = wl.mesh, wl.settings
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux="advection", velocity=s["velocity"], bc=s["bc"])
    t0 = time.perf_counter()
    ot = oracle.Oracle(2, mesh.verts, mesh.cells, tangent=True, **kw)
    D = rng.standard_normal((ndir, mesh.n_cell))
    u = torch.tensor(wl.u0, device="cuda")
    states = [u.clone()]
    for _ in range(steps):
        w.step(u, dt, 1)
        states.append(u.clone())
    gT = torch.tensor(states[-1].cpu().numpy() - s["target"], device="cuda")
    g = [None] * (steps + 1)
    g[steps] = gT
    for k in range(steps - 1, -1, -1):
        g[k] = w.step_adjoint(states[k], dt, 1, g[k + 1], ckpt)
    full = w.step_adjoint(states[0], dt, steps, gT, ckpt)
    torch.cuda.synchronize()
    composed = bool(torch.equal(g[0], full))
    rels = []
    for k in range(steps):
        _, JD = ot.step_tangent(states[k].cpu().numpy(), D, dt, 1)
        gk, gk1 = g[k].cpu().numpy(), g[k + 1].cpu().numpy()
        for j in range(ndir):
            a, b = float(gk @ D[j]), float(gk1 @ JD[j])
            rels.append(abs(a - b) / abs(b))
    worst = float(np.max(rels))
    norms = [float(torch.linalg.norm(g[k])) for k in range(steps, -1, -10)]
    o = oracle.Oracle(2, mesh.verts, mesh.cells, **kw)
    tf = time.perf_counter()
    uo = o.step(wl.u0, dt, steps)[0]
    tf = time.perf_counter() - tf
    drift = float(np.max(np.abs(states[-1].cpu().numpy() - uo)) / np.max(np.abs(uo)))
    secs = time.perf_counter() - t0
    log(f"[bench] adjoint vs the oracle's exact tangent, {steps} one-step segments x {ndir} directions: max rel "
        f"err {worst:.3e} (median {float(np.median(rels)):.3e}); composed = full call: {composed}; |g| from step "
        f"{steps} back to 0: {', '.join(f'{x:.2e}' for x in norms)}; GPU vs oracle {steps}-step trajectories "
        f"{drift:.2e} apart ({secs:.0f}s, {oracle.core.num_threads()} oracle threads)")
    return {"steps": steps, "directions": ndir, "reference": "oracle tangent build (dual numbers), per step along "
            "the GPU trajectory", "max_rel_err": worst, "median_rel_err": float(np.median(rels)), "tolerance": 1e-6,
            "pass": worst <= 1e-6 and composed, "one_step_adjoints_compose_to_full_call": composed,
            "gradient_norm_every_10_steps_from_T": norms, "trajectory_drift_gpu_vs_oracle": drift,
            "oracle_forward": {"value": mesh.n_cell * steps / tf, "unit": "cell-updates/s",
                               "cores": oracle.core.num_threads(), "kind": "oracle"},
            "seconds": secs}


def short_tangent_check(torch, w, wl, dt, steps, rng, ndir=8):
    """Over a horizon short enough for the GPU's and the oracle's trajectories
    to stay together, the whole gradient at once: <g_0, d> from the GPU's
    adjoint over `steps` steps against <g_T, J d> with J d the oracle's exact
    tangent of its own trajectory from u_0."""
    import oracle

    mesh, s = wl.mesh, wl.settings
    kw = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux="advection", velocity=s["velocity"], bc=s["bc"])
    ot = oracle.Oracle(2, mesh.verts, mesh.cells, tangent=True, **kw)
    D = rng.standard_normal((ndir, mesh.n_cell))
    uT, JD = ot.step_tangent(wl.u0, D, dt, steps)
    gT = uT[0] - s["target"]
    g0 = w.step_adjoint(torch.tensor(wl.u0, device="cuda"), dt, steps, torch.tensor(gT, device="cuda"), 10)
    g0 = g0.cpu().numpy()
    rels = [abs(float(g0 @ D[j]) - float(gT @ JD[j])) / abs(float(gT @ JD[j])) for j in range(ndir)]
    log(f"[bench] adjoint vs the oracle's exact tangent over {steps} steps from u0: max rel err {max(rels):.3e}")
    return {"steps": steps, "directions": ndir, "max_rel_err": float(max(rels)), "tolerance": 1e-6,
            "pass": max(rels) <= 1e-6}


def run_adjoint(torch, WLSENO, steps=100, ckpt=10, directions=32):
    """Adjoint workload: ~200 k triangles, p = 3, linear advection a = (1, 0.5),
    zero outside state at boundary facets (no inflow),
    loss 1/2 ||u(T) - u_target||^2 after `steps` RK3 steps; the gradient with
    respect to u0 from the checkpointed adjoint and its time against the
    forward run's.  Checks: the oracle's exact tangent step by step along the
    trajectory (exact_tangent_check) and, over the first 10 steps, as a whole
    (short_tangent_check); central differences over all steps in the
    equal-weight limit (unit weights: a linear scheme, so differences are
    exact up to rounding).  Over 100 steps the WLS-ENO map amplifies
    perturbations ~10^12-fold, so no difference quotient resolves it there."""
    from workloads import configs

    t = time.time()
    wl = configs.square_advection_adjoint(317, 5001)
    mesh = wl.mesh
    s = wl.settings
    out = {"workload": f"tri{mesh.n_cell}-advection-p3, {steps} steps, checkpoint every {ckpt}"}
    u0 = torch.tensor(wl.u0, device="cuda")
    tg = torch.tensor(s["target"], device="cuda")
    for weight_mode, tag in ((0, "wls_eno"), (1, "equal_weights")):
        w = WLSENO(device=0)
        w.mesh_upload(2, mesh.verts, mesh.cells)
        w.stencil_build(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux="advection", velocity=s["velocity"],
                        bc=s["bc"], weight_mode=weight_mode)
        dt = 0.5 * w.info()["min_insphere"] / float(np.hypot(*s["velocity"][:2]))

        def forward(x):
            y = x.clone()
            w.step(y, dt, steps)
            return y

        gT = forward(u0) - tg
        g0 = w.step_adjoint(u0, dt, steps, gT, ckpt)          # warm-up (tables, buffers)
        torch.cuda.synchronize()
        if weight_mode == 0:
            log(f"[bench] adjoint workload: {mesh.n_cell} cells, ready in {time.time() - t:.1f}s")
            reps = 3
            ts = time.perf_counter()
            for _ in range(reps):
                forward(u0)
            torch.cuda.synchronize()
            t_fwd = (time.perf_counter() - ts) / reps
            ts = time.perf_counter()
            for _ in range(reps):
                g0 = w.step_adjoint(u0, dt, steps, gT, ckpt)
            torch.cuda.synchronize()
            t_full = (time.perf_counter() - ts) / reps
            # forward with checkpoints, then the reverse sweep alone
            ur = u0.clone()
            w.step_record(ur, dt, steps, ckpt)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(reps):
                g0r = w.step_adjoint_recorded(gT)
            torch.cuda.synchronize()
            t_rev = (time.perf_counter() - ts) / reps
            assert torch.equal(g0r, g0)
            log(f"[bench] forward {t_fwd * 1e3:.2f} ms; adjoint {t_full * 1e3:.2f} ms from u0, "
                f"{t_rev * 1e3:.2f} ms over a recorded forward ({steps} steps)")
            out.update({"forward_ms": t_fwd * 1e3, "adjoint_ms": t_rev * 1e3, "adjoint_over_forward": t_rev / t_fwd,
                        "adjoint_from_u0_ms": t_full * 1e3, "adjoint_from_u0_over_forward": t_full / t_fwd})

        rng = np.random.default_rng(5003)
        if weight_mode == 0:
            out[f"exact_tangent_{steps}_steps"] = exact_tangent_check(torch, w, wl, dt, steps, ckpt, rng)
            out["exact_tangent_10_steps_from_u0"] = short_tangent_check(torch, w, wl, dt, 10, rng)
        else:
            worst = 0.0
            for _ in range(directions):
                d = torch.tensor(rng.standard_normal(mesh.n_cell), device="cuda")
                h = 1e-6 * float(u0.abs().max()) / float(d.abs().max())
                Jd = (forward(u0 + h * d) - forward(u0 - h * d)) / (2 * h)
                fd = float(torch.dot(gT, Jd))
                ad = float(torch.dot(g0, d))
                worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
            log(f"[bench] {tag}: adjoint vs central differences, {directions} directions: max rel err {worst:.3e}, "
                f"max |g0| {float(g0.abs().max()):.3e}")
            out[f"fd_{tag}_{steps}_steps"] = {"steps": steps, "directions": directions, "max_rel_err": worst,
                                              "tolerance": 1e-6, "pass": worst <= 1e-6,
                                              "max_abs_gradient": float(g0.abs().max())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    # the first stepping call captures the library's graphs (every run
    # length, once per context and time step), so any warm-up of 2 or more
    # steps keeps capture out of the timed steps
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="square", choices=sorted(WORKLOADS) + ["batch"])
    ap.add_argument("--balance", action="store_true",
                    help="single-mesh workloads: balanced-stencil refit of out-of-range cells")
    ap.add_argument("--characteristic", action="store_true",
                    help="batch workload: reconstruct characteristic fields per facet")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0 disables the CPU leg)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward measurement of the default workload")
    ap.add_argument("--adjoint-fd", type=int, default=32,
                    help="random directions of the adjoint's finite-difference check")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of the same K steps (median, min, max reported)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per cell of the reconstruction (0: autotune); profiling runs pin it")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2 M-triangle companion record of the default workload")
    ap.add_argument("--side", type=int, default=0,
                    help="single-mesh workloads: lattice points per side instead of the workload's own (a size "
                         "sweep; no stored traffic counters apply then)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs a mesh, or a "
              "batch of meshes, on a single device; sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1602_02694_amd import WLSENO

    if args.workload == "batch":
        print(json.dumps(run_batch(args, torch, WLSENO)), flush=True)
        return
    wl = make_workload(args.workload, args.side)
    cfg = wl.settings
    mesh = wl.mesh
    dim = mesh.dim
    log(f"[bench] workload {wl.name}")
    w = WLSENO(device=0)
    t1 = time.time()
    w.mesh_upload(dim, mesh.verts, mesh.cells)
    w.stencil_build(p=cfg["p"], n_lo=cfg["n_lo"], n_hi=cfg["n_hi"], flux=cfg["flux"], velocity=cfg["velocity"],
                    balance=args.balance, lanes=args.lanes)
    info = w.info()
    rp, _ = w.stencil()
    nsz = np.diff(rp)
    log(f"[bench] setup {time.time() - t1:.2f}s, stencils {nsz.min()}-{nsz.max()} (mean {nsz.mean():.2f})")
    u0 = np.ascontiguousarray(wl.u0, dtype=np.float64)
    if cfg["flux"] == "burgers":
        speed = np.sqrt(float(dim)) * np.max(np.abs(u0))
    else:
        speed = float(np.linalg.norm(cfg["velocity"][:dim]))
    dt = 0.5 * info["min_insphere"] / speed
    u_init = torch.tensor(u0, device="cuda")
    if args.lanes:
        tune = {"chosen": args.lanes, "cached": False, "timings_us": {}, "pinned": True}
    else:
        tune = w.autotune(u_init)
        log(f"[bench] autotuned reconstruction: {tune['chosen']} lanes per cell "
            f"({', '.join(f'{k}: {v:.2f} us' for k, v in tune['timings_us'].items())})")

    # warm-up
    u = u_init.clone()
    w.step(u, dt, args.warmup)
    torch.cuda.synchronize()
    # timed region: exactly K steps
    u = u_init.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    w.step(u, dt, args.steps)
    torch.cuda.synchronize()
    te = time.perf_counter()
    elapsed = te - ts
    nc = mesh.n_cell
    value = nc * args.steps / elapsed
    log(f"[bench] {args.steps} steps in {elapsed * 1e3:.2f} ms -> {value:.4g} cell-updates/s")
    # the same K timed steps again, for the spread
    rep = []
    for _ in range(args.repeats):
        u = u_init.clone()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        w.step(u, dt, args.steps)
        torch.cuda.synchronize()
        rep.append(nc * args.steps / (time.perf_counter() - ts))
    if rep:
        log(f"[bench] {len(rep)} more runs of {args.steps} steps: median {np.median(rep):.4g}, "
            f"min {min(rep):.4g}, max {max(rep):.4g} cell-updates/s")

    # a plain device copy of known size, so that hardware traffic counters of a
    # profiled run can be calibrated (bytes read and written = 2 x 512 MiB)
    cal_src = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    # kernel durations: HIP events on the library's stream around K back-to-back
    # launches of each kernel on the initial state
    k1_n = k2_n = 3 * args.steps
    k1_avg = w.time_kernel(0, u_init, k1_n)
    k2_avg = w.time_kernel(1, u_init, k2_n)
    F, Q, m = info["faces_per_cell"], info["points_per_face"], info["m"]
    flops = float(np.sum(recon_flops(nsz, m, dim, F, Q)))
    achieved = flops / (k1_avg * 1e-3) / 1e12
    log(f"[bench] k_reconstruct avg {k1_avg * 1e3:.2f} us ({k1_n} launches), "
        f"k_update avg {k2_avg * 1e3:.2f} us ({k2_n} launches); {flops / nc:.0f} flop/cell")
    # counters were taken on the workloads' own meshes only
    tkey = None if args.side else args.workload + ("-balance" if args.balance else "")
    traffic = traffic_record(f"k_reconstruct/{tune['chosen']}", tkey)
    roofline = {
        "bound": "alu",
        "kernel": "k_reconstruct",
        "achieved": achieved,
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
        "traffic": traffic,
        "avg_launch_us": k1_avg * 1e3,
        "flops_per_launch": flops,
    }
    ub = update_bytes(nc, dim, F, Q)
    ach_u = ub / (k2_avg * 1e-3) / 1e9
    roofline_update = {
        "bound": "hbm",
        "kernel": "k_update",
        "achieved": ach_u,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": ach_u / HBM_PEAK_GBS,
        "traffic": traffic_record("k_update", tkey),
        "avg_launch_us": k2_avg * 1e3,
        "bytes_per_launch": ub,
    }

    out = {
        "metric": cfg["metric"],
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name + ("-balanced" if args.balance else ""),
            "balanced_refit": bool(args.balance),
            "mesh": (f"Delaunay triangulation of a jittered {cfg['side']}^{dim} lattice on [0,1]^{dim}"
                     f" (seed {cfg['seed']})"),
            "n_cell": nc,
            "p": cfg["p"],
            "stencil_cells": [int(nsz.min()), int(nsz.max())],
            "flux": ("burgers, global Lax-Friedrichs alpha" if cfg["flux"] == "burgers"
                     else f"linear advection, a = {tuple(cfg['velocity'][:dim])}"),
            "time_integrator": "TVD RK3",
            "dt": dt,
        },
        "roofline": roofline,
        "roofline_update": roofline_update,
        "autotune": tune,
    }
    if rep:
        out["repeat_timing"] = {"runs": len(rep), "steps_each": args.steps, "median_value": float(np.median(rep)),
                                "min_value": float(min(rep)), "max_value": float(max(rep))}

    if args.cpu_seconds > 0 and args.workload == "square":
        import oracle

        o = oracle.from_workload(wl, balance=args.balance)
        nthreads = oracle.core.num_threads()
        tt = time.perf_counter()
        o.step(u0, dt, 1)
        one = time.perf_counter() - tt
        S = int(max(2, min(args.steps, args.cpu_seconds / max(one, 1e-6))))
        log(f"[bench] oracle: {one:.3f}s per step on {nthreads} threads; timing {S} steps")
        tt = time.perf_counter()
        uo = o.step(u0, dt, S)[0]
        cpu_t = time.perf_counter() - tt
        ug = u_init.clone()
        w.step(ug, dt, S)
        torch.cuda.synchronize()
        g = ug.cpu().numpy()
        # the same oracle on one thread, over a shorter sample
        S1 = int(max(2, min(S, 0.5 * args.cpu_seconds / max(one * nthreads, 1e-6))))
        prev = oracle.core.set_num_threads(1)
        tt = time.perf_counter()
        o.step(u0, dt, S1)
        cpu1 = time.perf_counter() - tt
        oracle.core.set_num_threads(prev)
        out["cpu_baseline"] = {
            "value": nc * S / cpu_t,
            "unit": "cell-updates/s",
            "cores": nthreads,
            "kind": "oracle",
            "sample": f"{S} TVD RK3 steps of the same workload from the same initial data",
            "one_core": {"value": nc * S1 / cpu1, "cores": 1, "sample": f"{S1} TVD RK3 steps"},
            "host_cpu_count": os.cpu_count(),
        }
        out["parity"] = dict(steps=S, **parity_stats(g, uo))
        log(f"[bench] oracle {nc * S / cpu_t:.4g} cell-updates/s on {nthreads} threads, {nc * S1 / cpu1:.4g} on one; "
            f"GPU vs oracle after {S} steps: max {out['parity']['max_rel_err_vs_oracle']:.3e}, "
            f"99.9% {out['parity']['p99_9_rel_err']:.3e}, norm-wise {out['parity']['normwise_rel_err']:.3e}")
    if args.workload in ("cube", "square-large") and args.cpu_seconds > 0 and not args.balance:
        kwp = dict(p=cfg["p"], n_lo=cfg["n_lo"], n_hi=cfg["n_hi"], flux=cfg["flux"], velocity=cfg["velocity"])
        if cfg["flux"] == "burgers":
            kwp["lf_alpha"] = 1       # the global alpha needs every cell; the local one is checked
            w.stencil_build(**kwp)
        out["sampled_parity"] = sampled_parity(torch, w, wl, u_init, kwp, R=3 if dim == 3 else 4)
    if args.workload == "square" and args.cpu_seconds > 0:
        out["line200"] = run_line(torch, WLSENO)
    if args.workload == "square" and not args.no_large:
        out["square_large"] = run_square_large(torch, WLSENO)
    if args.workload == "square" and not args.no_adjoint:
        out["adjoint"] = run_adjoint(torch, WLSENO, directions=args.adjoint_fd)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
