"""Seeded synthetic inputs: simplex meshes and initial cell averages.

This package is shared by the oracle tests, the GPU parity tests and the
benchmark.  It only produces *inputs* (vertex coordinates, cell
connectivity, cell averages of prescribed initial data); it contains none of
the reconstruction, flux or time-stepping arithmetic of the method.

Every generator is deterministic for a given seed (numpy PCG64 via
``numpy.random.default_rng``).
"""

from .meshes import Mesh, periodic_line, uniform_periodic_line, jittered_square, jittered_square_periodic, jittered_cube
from .fields import (
    cell_averages,
    line_cell_averages,
    square_wave_sine_1d,
    gaussian_bump_with_step_2d,
    sine_with_sphere_3d,
    gaussian_sum,
    euler_quadrants,
    polynomial_field,
)
from . import configs

__all__ = [
    "Mesh",
    "periodic_line",
    "uniform_periodic_line",
    "jittered_square",
    "jittered_square_periodic",
    "jittered_cube",
    "cell_averages",
    "line_cell_averages",
    "square_wave_sine_1d",
    "gaussian_bump_with_step_2d",
    "sine_with_sphere_3d",
    "gaussian_sum",
    "euler_quadrants",
    "polynomial_field",
    "configs",
]
