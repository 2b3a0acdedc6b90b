"""The named synthetic workloads (mesh + initial cell averages + run settings).

Each builder returns a ``Workload``; nothing here computes any part of the
reconstruction.  ``settings`` carries the physics and stencil settings that the
library and the oracle are both configured with.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import Mesh, periodic_line, jittered_square, jittered_cube
from . import fields


@dataclass
class Workload:
    name: str
    mesh: Mesh
    u0: np.ndarray                 # (n_cell,) or (V, n_cell)
    settings: dict = field(default_factory=dict)


def line_advection(n_cells: int = 200, seed: int = 1001) -> Workload:
    """1-D periodic, +-20% widths, p=3, 5-cell stencil, u_t+u_x=0, sine + square wave."""
    mesh = periodic_line(n_cells, 0.1, seed)
    u0 = fields.square_wave_sine_1d(mesh)
    return Workload(f"line{n_cells}-advection-p3", mesh, u0,
                    dict(p=3, n_lo=5, n_hi=5, flux="advection", velocity=(1.0, 0.0, 0.0),
                         steps=100, cfl=0.5))


def square_burgers(n_per_side: int = 100, seed: int = 2001) -> Workload:
    """2-D Delaunay triangles of the unit square, p=3, 12-20 cell stencils, Burgers."""
    mesh = jittered_square(n_per_side, 0.3, seed)
    u0 = fields.cell_averages(mesh, fields.gaussian_bump_with_step_2d)
    return Workload(f"tri{mesh.n_cell}-burgers-p3", mesh, u0,
                    dict(p=3, n_lo=12, n_hi=20, flux="burgers", velocity=(0.0, 0.0, 0.0),
                         steps=200, cfl=0.5))


def square_advection_adjoint(n_per_side: int = 317, seed: int = 5001) -> Workload:
    """2-D triangles (~200k for 317^2 points), p=3, linear advection a=(1,0.5)."""
    mesh = jittered_square(n_per_side, 0.3, seed)
    u0 = fields.cell_averages(mesh, fields.gaussian_sum(seed, 8, 2))
    target = fields.cell_averages(mesh, fields.gaussian_sum(seed + 1, 8, 2))
    # zero outside state at boundary facets (no inflow): with the inside
    # state there, inflow facets make the operator grow without bound
    return Workload(f"tri{mesh.n_cell}-advection-p3", mesh, u0,
                    dict(p=3, n_lo=12, n_hi=20, flux="advection", velocity=(1.0, 0.5, 0.0),
                         steps=100, cfl=0.5, target=target, ckpt_every=10, bc=1))


def cube_advection(n_per_side: int = 74, seed: int = 4001) -> Workload:
    """3-D Delaunay tetrahedra of the unit cube, p=3, 30-50 cell stencils, a=(1,.5,.25)."""
    mesh = jittered_cube(n_per_side, 0.15, seed)
    u0 = fields.cell_averages(mesh, fields.sine_with_sphere_3d)
    return Workload(f"tet{mesh.n_cell}-advection-p3", mesh, u0,
                    dict(p=3, n_lo=30, n_hi=50, flux="advection", velocity=(1.0, 0.5, 0.25),
                         steps=50, cfl=0.5))


def batched_euler(n_meshes: int = 64, seed: int = 3001, lo_cells: float = 5e3,
                  hi_cells: float = 5e4) -> list[Workload]:
    """Many independent triangle meshes with log-uniform sizes, p=4, 2-D Euler."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(lo_cells), np.log(hi_cells), n_meshes))).astype(int)
    out = []
    for k, nc in enumerate(sizes):
        side = max(3, int(round(np.sqrt(nc / 2.0))) + 1)
        mesh = jittered_square(side, 0.3, seed + 1 + k)
        u0 = fields.cell_averages(mesh, fields.euler_quadrants(seed + 1000 + k))
        out.append(Workload(f"euler{k}-tri{mesh.n_cell}", mesh, u0,
                            dict(p=4, n_lo=20, n_hi=36, flux="euler", gamma=1.4,
                                 velocity=(0.0, 0.0, 0.0), steps=1, cfl=0.5)))
    return out
