"""Initial data and their cell averages.

Cell averages are computed by numerical quadrature that is independent of
the method: collapsed (Duffy) Gauss-Legendre product rules on each simplex,
with a 4-way midpoint subdivision of triangles.  The 2-D rule (4x4 points per
sub-triangle) is exact for polynomials of degree <= 6 and the 3-D rule (4^3
points) for degree <= 5; 1-D averages of the piecewise data are exact
(antiderivatives).
"""

from __future__ import annotations

import numpy as np

from .meshes import Mesh

_GL_N = 4


def _gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _tri_rule():
    """Points (barycentric) and weights (sum 1) of the collapsed rule on a triangle."""
    g, w = _gauss01(_GL_N)
    lam, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            lam.append((1.0 - a, a * (1.0 - b), a * b))
            wts.append(2.0 * wa * wb * a)
    return np.array(lam), np.array(wts)


def _tet_rule():
    g, w = _gauss01(_GL_N)
    lam, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            for c, wc in zip(g, w):
                lam.append((1.0 - a, a * (1.0 - b), a * b * (1.0 - c), a * b * c))
                wts.append(6.0 * wa * wb * wc * a * a * b)
    return np.array(lam), np.array(wts)


def _subdivided_tri_rule():
    """The collapsed rule applied on the 4 midpoint sub-triangles (weights sum to 1)."""
    lam, wts = _tri_rule()
    e = np.eye(3)
    m01, m12, m20 = (e[0] + e[1]) / 2, (e[1] + e[2]) / 2, (e[2] + e[0]) / 2
    subs = [(e[0], m01, m20), (m01, e[1], m12), (m20, m12, e[2]), (m12, m20, m01)]
    out_l, out_w = [], []
    for a, b, c in subs:
        corners = np.stack([a, b, c])            # 3 x 3 (barycentric of corners)
        out_l.append(lam @ corners)
        out_w.append(wts / 4.0)
    return np.concatenate(out_l), np.concatenate(out_w)


def cell_averages(mesh: Mesh, fn, chunk: int = 1 << 16) -> np.ndarray:
    """Quadrature cell averages of ``fn(x) -> values`` over every simplex.

    ``fn`` receives an ``(npts, dim)`` array and returns ``(npts,)`` or
    ``(npts, V)``; the result is ``(n_cell,)`` or ``(V, n_cell)``.
    """
    if mesh.dim == 1:
        g, w = _gauss01(8)
        lam = np.stack([1.0 - g, g], axis=1)
        wts = w
    elif mesh.dim == 2:
        lam, wts = _subdivided_tri_rule()
    else:
        lam, wts = _tet_rule()
    nc = mesh.n_cell
    out = None
    for s in range(0, nc, chunk):
        cv = mesh.verts[mesh.cells[s:s + chunk]]           # (c, d+1, dim)
        if mesh.dim == 1 and mesh.periodic:
            cv = cv.copy()
        x = np.einsum("qv,cvd->cqd", lam, cv)              # (c, q, dim)
        vals = np.asarray(fn(x.reshape(-1, mesh.dim)))
        if vals.ndim == 1:
            vals = vals.reshape(x.shape[0], x.shape[1])
            avg = vals @ wts
            if out is None:
                out = np.empty(nc)
            out[s:s + chunk] = avg
        else:
            V = vals.shape[1]
            vals = vals.reshape(x.shape[0], x.shape[1], V)
            avg = np.einsum("cqv,q->vc", vals, wts)
            if out is None:
                out = np.empty((V, nc))
            out[:, s:s + chunk] = avg
    return out


def line_cell_averages(mesh: Mesh, antiderivative) -> np.ndarray:
    """Exact 1-D cell averages from an antiderivative ``F`` (vectorised)."""
    a = mesh.verts[mesh.cells[:, 0], 0]
    b = mesh.verts[mesh.cells[:, 1], 0]
    return (antiderivative(b) - antiderivative(a)) / (b - a)


def square_wave_sine_1d(mesh: Mesh) -> np.ndarray:
    """``sin(2 pi x)`` on [0, 0.5), 1 on [0.6, 0.8], 0 elsewhere (exact averages)."""

    def F(x):
        x = np.asarray(x, dtype=np.float64)
        xs = np.clip(x, 0.0, 0.5)
        sine = (1.0 - np.cos(2.0 * np.pi * xs)) / (2.0 * np.pi)
        box = np.clip(x, 0.6, 0.8) - 0.6
        return sine + box

    return line_cell_averages(mesh, F)


def gaussian_bump_with_step_2d(x: np.ndarray) -> np.ndarray:
    r1 = (x[:, 0] - 0.35) ** 2 + (x[:, 1] - 0.35) ** 2
    r2 = np.sqrt((x[:, 0] - 0.65) ** 2 + (x[:, 1] - 0.65) ** 2)
    return 0.25 + np.exp(-r1 / 0.01) + 0.5 * (r2 < 0.15)


def sine_with_sphere_3d(x: np.ndarray) -> np.ndarray:
    s = np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1]) * np.sin(2 * np.pi * x[:, 2])
    r = np.sqrt(((x - 0.5) ** 2).sum(axis=1))
    return s + 1.0 * (r < 0.2)


def gaussian_sum(seed: int, n: int = 8, dim: int = 2):
    """A sum of ``n`` Gaussians with amplitude U[0.5,1], centre U[0.2,0.8]^d, width U[0.05,0.15]."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.0, n)
    cen = rng.uniform(0.2, 0.8, (n, dim))
    sig = rng.uniform(0.05, 0.15, n)

    def fn(x):
        out = np.zeros(x.shape[0])
        for a, c, s in zip(amp, cen, sig):
            out += a * np.exp(-((x - c) ** 2).sum(axis=1) / (2 * s * s))
        return out

    return fn


def euler_quadrants(seed: int, gamma: float = 1.4):
    """Four piecewise-constant Riemann states (conserved variables) about a random split.

    Density and pressure are U[0.1, 1], velocities U[-1, 1]; the split point is
    U[0.3, 0.7]^2.  Returns a function of ``x`` giving ``(npts, 4)`` values
    ``(rho, rho u, rho v, E)``.
    """
    rng = np.random.default_rng(seed)
    split = rng.uniform(0.3, 0.7, 2)
    rho = rng.uniform(0.1, 1.0, 4)
    pr = rng.uniform(0.1, 1.0, 4)
    vel = rng.uniform(-1.0, 1.0, (4, 2))
    E = pr / (gamma - 1.0) + 0.5 * rho * (vel ** 2).sum(axis=1)
    U = np.stack([rho, rho * vel[:, 0], rho * vel[:, 1], E], axis=1)   # (4 quadrants, 4 vars)

    def fn(x):
        q = (x[:, 0] >= split[0]).astype(int) + 2 * (x[:, 1] >= split[1]).astype(int)
        return U[q]

    return fn


def polynomial_field(seed: int, dim: int, degree: int, scale: float = 1.0):
    """A random polynomial of total degree ``<= degree`` (monomials about the origin)."""
    rng = np.random.default_rng(seed)
    exps = []
    for q in range(degree + 1):
        if dim == 1:
            exps.append((q,))
        elif dim == 2:
            for a in range(q, -1, -1):
                exps.append((a, q - a))
        else:
            for a in range(q, -1, -1):
                for b in range(q - a, -1, -1):
                    exps.append((a, b, q - a - b))
    coef = rng.normal(0.0, scale, len(exps))

    def fn(x):
        out = np.zeros(x.shape[0])
        for c, e in zip(coef, exps):
            term = np.full(x.shape[0], c)
            for d in range(dim):
                term = term * x[:, d] ** e[d]
            out += term
        return out

    fn.exps = exps
    fn.coef = coef
    return fn


def isentropic_vortex(t: float = 0.0, beta: float = 5.0, gamma: float = 1.4, centre=(5.0, 5.0), mean=(1.0, 1.0)):
    """Isentropic vortex in a uniform stream (conserved variables), the exact
    solution of the 2-D Euler equations at time ``t`` (Sec. 5.2.3 of the WLS-ENO
    paper: rho, p = 1 at infinity, mean flow (1, 1), strength 5, centred in
    [0,10]^2 at t = 0).  With x' = x - centre - mean t and r^2 = |x'|^2:
    velocity perturbation beta/(2 pi) exp((1 - r^2)/2) (-y', x'), temperature
    T = 1 - (gamma - 1) beta^2 / (8 gamma pi^2) exp(1 - r^2), and no entropy
    perturbation: rho = T^(1/(gamma-1)), p = rho T."""
    cx = centre[0] + mean[0] * t
    cy = centre[1] + mean[1] * t

    def fn(x):
        xb = x[:, 0] - cx
        yb = x[:, 1] - cy
        r2 = xb * xb + yb * yb
        amp = beta / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
        u = mean[0] - amp * yb
        v = mean[1] + amp * xb
        T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
        return np.stack([rho, rho * u, rho * v, E], axis=1)

    return fn


def sod_x(x0: float = 0.5, gamma: float = 1.4):
    """Sod's shock-tube states (Sec. 5.1.4 of the WLS-ENO paper) along x, at
    rest: (rho, p) = (1, 1) for x < x0 and (0.125, 0.1) beyond (conserved
    variables of the 2-D system)."""

    def fn(x):
        left = x[:, 0] < x0
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        z = np.zeros_like(rho)
        return np.stack([rho, z, z, p / (gamma - 1.0)], axis=1)

    return fn
