"""Element-wise parity rule shared by the GPU tests.

A GPU value g matches the oracle value o when
    |g - o| <= rel * max(|o|, floor * max|o|)
per field and component (rel = 1e-12, floor = 1e-2): relative to the value
itself, with a floor at 1% of the field's magnitude so that zeros of a smooth
field do not make the relative error ill-posed.  Right-hand sides are
measured against the magnitude of the fluxes they sum (``flux_scale``).

FP64 floor.  In cells whose weighted system is stiff (weights spanning up to
1/(eps h^2) next to a discontinuity) two correct FP64 solvers can only agree
to about kappa * 2^-53, kappa = cond_2(W A S) of the cell.  The per-cell
tolerance is therefore

    max(rel, K_COND * kappa_i * 2^-53, K_FLOOR * nu_i)

where kappa_i is taken over the cell and its facet neighbours for quantities
that combine several reconstructions (right-hand sides, trajectories), and
nu_i is the FP64 oracle's own relative error in cell i measured against the
same oracle run in x87 extended precision (``Oracle(..., extended=True)``).
With kappa below ~560 (99% of the cells of the 2-D workloads) the tolerance is
rel = 1e-12.  Measured on the 19,602-triangle Burgers workload, GPU and FP64
oracle errors against the extended run stay below 3.2 kappa 2^-53.
"""

import json
import os

import numpy as np

REL = 1e-12
FLOOR = 1e-2
K_FLOOR = 4.0
K_COND = 16.0
U64 = 2.0 ** -53


def rel_errors(g, o, floor=FLOOR, scale=None):
    """|g - o| / max(|o|, floor * max|o|, scale); the max is taken per leading
    index (per field component) for arrays of two or more dimensions."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    if o.size == 0:
        mx = 0.0
    elif o.ndim >= 2:
        mx = np.max(np.abs(o), axis=tuple(range(1, o.ndim)), keepdims=True)
    else:
        mx = np.max(np.abs(o))
    sc = np.maximum(np.abs(o), floor * mx)
    if scale is not None:
        sc = np.maximum(sc, np.asarray(scale, dtype=np.float64).reshape(sc.shape))
    sc = np.where(sc > 0, sc, 1.0)
    return np.abs(g - o) / sc


def momentum_scale(o, dim, floor=FLOOR):
    """Euler arrays (V, ...): a floor for the momentum components at 1% of the
    momentum vector's largest component, the same for every component (a
    rotation of the frame mixes them; a momentum component that vanishes in
    the data, like the transverse momentum of a shock tube, is measured
    against the flow's momentum, not against its own noise).  Zero for the
    other components, which keep their own per-component floor."""
    o = np.asarray(o, dtype=np.float64)
    sc = np.zeros_like(o)
    sc[1:1 + dim] = floor * np.max(np.abs(o[1:1 + dim]))
    return sc


def flux_scale(o, fval, alpha=0.0):
    """Per-cell magnitude of the flux sum that forms the right-hand side:
    S_i = (1/|tau_i|) sum_f |f| sum_q w_q |F(u_q).n_f| from the oracle's own
    facet values.  L_i is a difference of such fluxes divided by |tau_i|, so
    its rounding error is relative to S_i rather than to |L_i|.  For the Euler
    system, per component, with the dissipation term alpha |u_q| added to
    |F(u_q).n_f| (it is of the same size); the result is (V, nc)."""
    m = o.mesh
    if o.flux == "euler":
        fv = np.asarray(fval)                                  # (V, nc, F, Q)
        gamma = o._P.gamma
        rho, mx, my, E = fv[0], fv[1], fv[2], fv[3]
        n = m.normal                                           # (nc, F, 2)
        vn = (mx * n[:, :, 0, None] + my * n[:, :, 1, None]) / rho
        pr = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
        Fn = np.stack([rho * vn, mx * vn + pr * n[:, :, 0, None], my * vn + pr * n[:, :, 1, None],
                       (E + pr) * vn])
        fl = np.abs(Fn) + alpha * np.abs(fv)
        per_face = fl @ m.qw                                   # (V, nc, F)
        return (per_face * m.area[None]).sum(axis=2) / m.vol[None]
    fv = np.asarray(fval)[0]                                   # (nc, F, Q)
    if o.flux == "burgers":
        sn = np.abs(m.normal.sum(axis=2))                      # (nc, F)
        fl = 0.5 * fv ** 2 * sn[:, :, None]
    else:
        vel = np.asarray(o._P.adv[:o.dim])
        an = np.abs(m.normal @ vel)
        fl = np.abs(fv) * an[:, :, None]
    per_face = fl @ m.qw                                       # (nc, F)
    return (per_face * m.area).sum(axis=1) / m.vol


def cell_noise(o, x, floor=FLOOR, scale=None, cell_axes=None):
    """Per-cell FP64 floor nu: the FP64 oracle's relative error against the
    extended-precision oracle, maximised over each cell's entries (the axes
    after ``cell_axes`` leading ones), broadcastable to o."""
    e = rel_errors(o, x, floor, scale)
    if cell_axes is not None and e.ndim > cell_axes:
        e = e.max(axis=tuple(range(cell_axes, e.ndim)), keepdims=True)
    return e


def report(what, err, tol, rel=REL, err_plain=None):
    """Print (and, with WLSENO_PARITY_LOG set, append as a JSON line to that
    file) how the comparison passed: entries, largest error, how many entries
    exceed the plain 1e-12 bar measured against their own magnitude but pass
    through the flux scale S_i, how many pass only through the kappa/nu floor,
    and the largest effective tolerance any entry needed."""
    above = err > rel
    rec = {"what": what, "entries": int(err.size), "max_err": float(err.max()) if err.size else 0.0,
           "floor_only": int(np.sum(above & (err <= tol))),
           "scale_only": int(np.sum((err_plain > rel) & ~above)) if err_plain is not None else 0,
           "largest_tol_needed": float(np.max(tol[above])) if above.any() else rel}
    print(f"[parity] {what}: {rec['entries']} entries, max err {rec['max_err']:.2e}; {rec['scale_only']} pass only "
          f"through the flux scale, {rec['floor_only']} only through the kappa/nu floor (largest tolerance needed "
          f"{rec['largest_tol_needed']:.2e})", flush=True)
    path = os.environ.get("WLSENO_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")
    return rec


def assert_parity(g, o, what="", rel=REL, floor=FLOOR, scale=None, noise=None, tol_floor=None):
    g = np.asarray(g)
    o = np.asarray(o)
    assert g.shape == o.shape, (what, g.shape, o.shape)
    assert np.all(np.isfinite(g)), f"{what}: non-finite GPU values"
    if o.size == 0:
        return 0.0
    err = rel_errors(g, o, floor, scale)
    tol = np.full(err.shape, rel)
    if noise is not None:
        tol = np.maximum(tol, K_FLOOR * np.broadcast_to(np.asarray(noise, dtype=np.float64), err.shape))
    if tol_floor is not None:
        tol = np.maximum(tol, np.broadcast_to(np.asarray(tol_floor, dtype=np.float64), err.shape))
    worst = float(err.max())
    report(what, err, tol, rel, rel_errors(g, o, floor) if scale is not None else None)
    bad = err > tol
    nbad = int(bad.sum())
    if nbad:
        i = int(np.argmax(err - tol))
        idx = np.unravel_index(i, err.shape)
        raise AssertionError(f"{what}: {nbad} of {err.size} entries above tolerance; worst excess at {idx}: "
                             f"err {err.flat[i]:.3e} > tol {tol.flat[i]:.3e} (gpu {g.flat[i]!r}, oracle {o.flat[i]!r})")
    return worst


def poly_dev(gcoef, ocoef, o, u, floor=FLOOR):
    """Taylor coefficient vectors compared through the polynomials they define:
    the bound sum_k |dv_k| rho_i^{|a_k|} / a_k! on their largest difference over
    the ball of radius rho_i (centroid to farthest vertex) that holds cell i,
    relative to the same bound of the reference polynomial itself,
    sum_k |v_k| rho_i^{|a_k|} / a_k! (at least max(|u_i|, floor * max|u|)).

    A backward-stable least-squares solve bounds the error of the whole
    coefficient vector relative to that vector's own size, so a polynomial that
    varies far more across the ball than its mean value (a cell at a steep
    front, u_i near zero) is measured against its own range, as facet values
    are measured against their own magnitude."""
    from math import factorial

    m = o.mesh
    rho = np.sqrt(((m.cv - m.cent[:, None, :]) ** 2).sum(axis=2)).max(axis=1)      # (nc,)
    g = np.asarray(gcoef, dtype=np.float64)
    r = np.asarray(ocoef, dtype=np.float64)
    assert g.shape == r.shape, (g.shape, r.shape)
    assert np.all(np.isfinite(g)), "non-finite GPU coefficients"
    deg = o.exps.sum(axis=1)
    fac = np.array([np.prod([factorial(int(a)) for a in e]) for e in o.exps], dtype=np.float64)
    w = rho[:, None] ** deg[None, :] / fac[None, :]                                # (nc, m)
    dev = (np.abs(g - r) * w[None]).sum(axis=2)                                     # (V, nc)
    size = (np.abs(r) * w[None]).sum(axis=2)
    uu = np.asarray(u, dtype=np.float64).reshape(dev.shape)
    sc = np.maximum(np.maximum(np.abs(uu), size), floor * np.max(np.abs(uu), axis=1, keepdims=True))
    return dev / np.where(sc > 0, sc, 1.0)


def assert_poly_parity(gcoef, ocoef, o, u, what="", rel=REL, floor=FLOOR, xcoef=None, tol_floor=None):
    err = poly_dev(gcoef, ocoef, o, u, floor)
    tol = np.full(err.shape, rel)
    if tol_floor is not None:
        tol = np.maximum(tol, np.broadcast_to(np.asarray(tol_floor, dtype=np.float64), err.shape))
    if xcoef is not None:
        tol = np.maximum(tol, K_FLOOR * poly_dev(ocoef, xcoef, o, u, floor))
    report(what, err, tol, rel)
    bad = err > tol
    if bad.any():
        idx = np.unravel_index(int(np.argmax(err - tol)), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {err.size} cells above tolerance; worst excess at {idx}: "
                             f"err {err[idx]:.3e} > tol {tol[idx]:.3e}")
    return float(err.max())


def cell_conditions(o, u, cells=None):
    """kappa = cond_2(W A S) per (component, cell) from the oracle's own
    per-cell matrix and weights (rows padded with zeros, which leaves the
    singular values unchanged).  With ``cells``, only those cells are
    evaluated; the others are left at zero."""
    u = np.asarray(u, dtype=np.float64).reshape(o.nvars, o.nc)
    cells = np.arange(o.nc) if cells is None else np.asarray(cells, dtype=np.int64)
    nmax = int(np.max(np.diff(o.row_ptr)))
    out = np.zeros((o.nvars, o.nc))
    mats = [o.cell_matrix(int(i)) for i in cells]
    for v in range(o.nvars):
        M = np.zeros((len(cells), nmax, o.m))
        for k, i in enumerate(cells):
            WA = o.cell_weights(int(i), u[v])[:, None] * mats[k]
            nr = np.linalg.norm(WA, axis=0)
            M[k, :len(WA)] = WA / np.where(nr > 0, nr, 1.0)
        sv = np.linalg.svd(M, compute_uv=False)
        out[v, cells] = sv[:, 0] / np.maximum(sv[:, -1], 1e-300)
    return out


def char_cell_conditions(o, u):
    """kappa per (field, cell) for characteristic-wise reconstruction: the
    largest cond_2(W A S) over the cell's facets, with the weights of each
    field projected at that facet's state (2-D Euler)."""
    import oracle

    u = np.asarray(u, dtype=np.float64).reshape(o.nvars, o.nc)
    out = np.zeros((o.nvars, o.nc))
    normal = o.mesh.normal
    for i in range(o.nc):
        A = o.cell_matrix(i)
        for lf in range(o.nf):
            j = o.mesh.nbr[i, lf]
            Ub = 0.5 * (u[:, i] + u[:, j]) if j >= 0 else u[:, i]
            L, _ = oracle.char_basis(o.dim, o._P.gamma, Ub, normal[i, lf])
            wf = L @ u
            for v in range(o.nvars):
                WA = o.cell_weights(i, wf[v])[:, None] * A
                nr = np.linalg.norm(WA, axis=0)
                sv = np.linalg.svd(WA / np.where(nr > 0, nr, 1.0), compute_uv=False)
                out[v, i] = max(out[v, i], sv[0] / max(sv[-1], 1e-300))
    return out


def neighbourhood_max(o, x):
    """max of a per-cell array over each cell and its facet neighbours."""
    x = np.asarray(x)
    nb = o.mesh.nbr
    out = x.copy()
    for lf in range(nb.shape[1]):
        j = nb[:, lf]
        has = j >= 0
        out[..., has] = np.maximum(out[..., has], x[..., j[has]])
    return out


def floor_tol(kappa=None, noise=None):
    """Per-entry tolerance floor K_COND kappa u and/or K_FLOOR nu (see module doc)."""
    t = 0.0
    if kappa is not None:
        t = np.maximum(t, K_COND * np.asarray(kappa) * U64)
    if noise is not None:
        t = np.maximum(t, K_FLOOR * np.asarray(noise))
    return t
