"""Seeded simplex meshes shaped like the paper's test meshes.

The paper's meshes are shown only as figures (non-uniform 1-D grids,
unstructured triangle meshes of a square, tetrahedral meshes of a cube;
Numerical Results, 1-D/2-D/3-D subsections), so these generators stand in for
them: jittered lattices triangulated by Delaunay (scipy/qhull).

Conventions shared by every consumer:

* ``verts`` is ``float64[n_vert, dim]``; ``cells`` is ``int32[n_cell, dim+1]``.
* 2-D triangles are counter-clockwise, 3-D tetrahedra positively oriented.
* A periodic 1-D mesh lists ``n_cell + 1`` nodes ``x_0 < ... < x_N``; the
  first and last node are the same point of the circle, the period is
  ``x_N - x_0``, and cell ``k`` is ``(k, k+1)``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    verts: np.ndarray
    cells: np.ndarray
    periodic: bool = False
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_cell(self) -> int:
        return int(self.cells.shape[0])

    @property
    def period(self) -> float:
        """1-D: the circle's length; 2-D: the period along x."""
        if not self.periodic:
            return 0.0
        if self.dim == 2:
            return float(self.meta["periods"][0])
        return float(self.verts[-1, 0] - self.verts[0, 0])


def periodic_line(n_cells: int, jitter: float = 0.1, seed: int = 1001,
                  x0: float = 0.0, length: float = 1.0) -> Mesh:
    """Periodic 1-D grid with node offsets ``U(-jitter, jitter)`` cell widths.

    Nodes are ``x_k = x0 + (k + delta_k) * length / n`` with ``delta_0 =
    delta_n = 0``; a jitter of 0.1 keeps every width within +-20% of uniform.
    """
    rng = np.random.default_rng(seed)
    k = np.arange(n_cells + 1, dtype=np.float64)
    delta = rng.uniform(-jitter, jitter, n_cells + 1)
    delta[0] = 0.0
    delta[-1] = 0.0
    x = x0 + (k + delta) * (length / n_cells)
    x[-1] = x0 + length
    cells = np.stack([np.arange(n_cells), np.arange(1, n_cells + 1)], axis=1).astype(np.int32)
    return Mesh(1, x[:, None].copy(), cells, periodic=True,
                name=f"line{n_cells}_j{jitter}_s{seed}")


def uniform_periodic_line(n_cells: int, x0: float = 0.0, length: float = 1.0) -> Mesh:
    x = x0 + np.arange(n_cells + 1, dtype=np.float64) * (length / n_cells)
    x[-1] = x0 + length
    cells = np.stack([np.arange(n_cells), np.arange(1, n_cells + 1)], axis=1).astype(np.int32)
    return Mesh(1, x[:, None].copy(), cells, periodic=True, name=f"uline{n_cells}")


def _orient(verts: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """Reorder vertices so every simplex has positive signed measure."""
    dim = verts.shape[1]
    v0 = verts[cells[:, 0]]
    edges = np.stack([verts[cells[:, k + 1]] - v0 for k in range(dim)], axis=1)
    det = np.linalg.det(edges)
    cells = cells.copy()
    neg = det < 0
    cells[neg, 0], cells[neg, 1] = cells[neg, 1].copy(), cells[neg, 0].copy()
    keep = np.abs(det) > 1e-14 * np.max(np.abs(det))
    return cells[keep].astype(np.int32)


def _lattice_points(n_per_side: int, dim: int, jitter: float, rng, lo: float, hi: float) -> np.ndarray:
    s = (hi - lo) / (n_per_side - 1)
    g = lo + np.arange(n_per_side) * s
    grids = np.meshgrid(*([g] * dim), indexing="ij")
    pts = np.stack([q.ravel() for q in grids], axis=1)
    on_lo = np.isclose(pts, lo)
    on_hi = np.isclose(pts, hi)
    free = ~(on_lo | on_hi)          # coordinates allowed to move
    noise = rng.uniform(-jitter * s, jitter * s, size=pts.shape)
    pts = pts + noise * free
    # Re-snap the boundary coordinates exactly (they were not moved).
    pts[on_lo] = lo
    pts[on_hi] = hi
    return pts


def jittered_square(n_per_side: int, jitter: float = 0.3, seed: int = 2001,
                    lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Delaunay triangulation of an ``n x n`` jittered lattice on ``[lo,hi]^2``.

    Interior points move by ``U(+-jitter*s)`` per axis, boundary points slide
    along their edge, corners stay fixed.  100x100 points give 19,602
    triangles.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = _lattice_points(n_per_side, 2, jitter, rng, lo, hi)
    tri = Delaunay(pts)
    cells = _orient(pts, tri.simplices.astype(np.int64))
    return Mesh(2, pts, cells, name=f"square{n_per_side}_j{jitter}_s{seed}")


def jittered_square_periodic(n_per_side: int, jitter: float = 0.3, seed: int = 2001,
                             lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Delaunay triangulation of an ``n x n`` jittered lattice on ``[lo,hi]^2``
    whose opposite boundaries carry identical points (a boundary point slides
    along its edge by the same amount as its partner across the square), so
    the mesh closes into a doubly periodic one.  ``meta["periods"]`` holds
    ``(hi - lo, hi - lo)``."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    n = n_per_side
    s = (hi - lo) / (n - 1)
    g = lo + np.arange(n) * s
    X, Y = np.meshgrid(g, g, indexing="ij")
    noise = rng.uniform(-jitter * s, jitter * s, size=(n, n, 2))
    noise[n - 1, :, 1] = noise[0, :, 1]       # x = hi copies the slide of x = lo
    noise[:, n - 1, 0] = noise[:, 0, 0]       # y = hi copies the slide of y = lo
    noise[0, :, 0] = noise[n - 1, :, 0] = 0.0
    noise[:, 0, 1] = noise[:, n - 1, 1] = 0.0
    X = X + noise[:, :, 0]
    Y = Y + noise[:, :, 1]
    X[0, :], X[n - 1, :] = lo, hi
    Y[:, 0], Y[:, n - 1] = lo, hi
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    tri = Delaunay(pts)
    cells = _orient(pts, tri.simplices.astype(np.int64))
    return Mesh(2, pts, cells, periodic=True, name=f"torus{n_per_side}_j{jitter}_s{seed}",
                meta={"periods": (hi - lo, hi - lo)})


def jittered_cube(n_per_side: int, jitter: float = 0.15, seed: int = 4001,
                  lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Delaunay tetrahedralisation of an ``n^3`` jittered lattice on ``[lo,hi]^3``."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = _lattice_points(n_per_side, 3, jitter, rng, lo, hi)
    tri = Delaunay(pts)
    cells = _orient(pts, tri.simplices.astype(np.int64))
    return Mesh(3, pts, cells, name=f"cube{n_per_side}_j{jitter}_s{seed}")
