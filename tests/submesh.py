"""Oracles on a sub-mesh around sampled cells, for parity checks at sizes
where the oracle cannot build every cell's stencil.

The sub-mesh holds every cell within R vertex rings of the sampled cells,
kept in the full mesh's order (ties between equally distant cells break the
same way) and given the full mesh's mean edge length h for eps h^2.  Once R
covers a sampled cell's k-ring stencil, its facet neighbours and their
stencils, the oracle's stencil, reconstruction and right-hand side of that
cell are those of the whole mesh (tests/test_submesh.py checks this on meshes
small enough for the whole-mesh oracle).
"""

import numpy as np

from parity import cell_conditions, neighbourhood_max


def _say(msg):
    print(msg, flush=True)


def rings(cells, nv, start, R):
    """Cells within R vertex rings of the cells ``start`` (sorted ids)."""
    mask = np.zeros(len(cells), dtype=bool)
    mask[start] = True
    for _ in range(R):
        vm = np.zeros(nv, dtype=bool)
        vm[cells[mask]] = True
        mask = vm[cells].any(axis=1)
    return np.flatnonzero(mask)


def mean_edge(verts, cells):
    """Mean length over the mesh's distinct edges."""
    nv = len(verts)
    k = cells.shape[1]
    pairs = np.concatenate([np.sort(cells[:, [a, b]].astype(np.int64), axis=1)
                            for a in range(k) for b in range(a + 1, k)])
    key = np.unique(pairs[:, 0] * nv + pairs[:, 1])
    a, b = key // nv, key % nv
    return float(np.mean(np.linalg.norm(verts[a] - verts[b], axis=1)))


def sample_cells(mesh, n_random, n_boundary, seed):
    """Seeded random cells plus cells with a vertex on the domain boundary."""
    rng = np.random.default_rng(seed)
    lo, hi = mesh.verts.min(axis=0), mesh.verts.max(axis=0)
    on_bnd = (np.isclose(mesh.verts, lo) | np.isclose(mesh.verts, hi)).any(axis=1)
    bcells = np.flatnonzero(on_bnd[mesh.cells].any(axis=1))
    pick = np.concatenate([rng.choice(mesh.n_cell, n_random, replace=False),
                           rng.choice(bcells, n_boundary, replace=False)])
    return np.unique(pick)


class SubOracle:
    """FP64 and extended-precision oracles on the sub-mesh around ``sample``."""

    def __init__(self, mesh, u0, sample, R, **kw):
        import oracle

        self.keep = rings(mesh.cells, len(mesh.verts), sample, R)
        vids, inv = np.unique(mesh.cells[self.keep], return_inverse=True)
        sub_cells = inv.reshape(len(self.keep), -1).astype(np.int32)
        sub_verts = mesh.verts[vids]
        self.loc = np.searchsorted(self.keep, sample)
        assert np.array_equal(self.keep[self.loc], sample)
        h = mean_edge(mesh.verts, mesh.cells)
        V = 4 if kw.get("flux") == "euler" else 1
        self.u = np.ascontiguousarray(np.asarray(u0).reshape(V, -1)[:, self.keep])
        self.o = oracle.Oracle(mesh.dim, sub_verts, sub_cells, False, h=h, **kw)
        self.ox = oracle.Oracle(mesh.dim, sub_verts, sub_cells, False, h=h, extended=True,
                                stencil=(self.o.row_ptr, self.o.col), **kw)
        _say(f"[oracle] sub-mesh of {len(self.keep)} cells around {len(sample)} sampled cells (R = {R})")

    def stencil_rows(self):
        o = self.o
        return [self.keep[o.col[o.row_ptr[i]:o.row_ptr[i + 1]]] for i in self.loc]

    def kappas(self):
        """kappa at the sampled cells, and its max over each sampled cell's facet neighbours."""
        o = self.o
        nb = o.mesh.nbr[self.loc]
        need = np.unique(np.concatenate([self.loc, nb[nb >= 0]]))
        k = cell_conditions(o, self.u, cells=need)
        return k, neighbourhood_max(o, k.max(axis=0, keepdims=True))
