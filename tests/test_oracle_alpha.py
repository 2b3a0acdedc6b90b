"""Pins of the oracle's global Lax-Friedrichs alpha.

The flux equation of Sec. 1 takes alpha as a constant bound of the normal
Jacobian's eigenvalues, and Sec. 4.2.1 uses alpha = max |f'(u)| over the
states the flux sees.  The oracle's global alpha is the largest normal
spectral radius over every cell's own facet-point values.  Each case below
computes the expected value by hand from the mesh vertices and closed forms,
and is chosen so that a plausible mistake gives a different number: alpha
from cell averages instead of facet values, from the area-scaled instead of
the unit normal, or from one side of the facets only.
"""

import numpy as np

from workloads import jittered_square, uniform_periodic_line


def _unit_edge_normals(mesh):
    """Outward unit normals and lengths of every edge of every (counter-
    clockwise) triangle, straight from the vertex coordinates."""
    v = mesh.verts[mesh.cells]                       # (nc, 3, 2)
    normals, lengths = [], []
    for a in range(3):
        p, q = v[:, a], v[:, (a + 1) % 3]
        d = q - p
        ln = np.hypot(d[:, 0], d[:, 1])
        # rotating a counter-clockwise edge by -90 degrees points outwards
        normals.append(np.stack([d[:, 1], -d[:, 0]], axis=1) / ln[:, None])
        lengths.append(ln)
    return np.concatenate(normals), np.concatenate(lengths)


def test_alpha_uniform_burgers_state(oracle_lib):
    """Burgers, u = c everywhere: every facet value is c, and the normal speed
    u (n_x + n_y) bounds alpha = |c| max over facets |n_x + n_y| (unit n)."""
    mesh = jittered_square(12, 0.3, 2101)
    n, ln = _unit_edge_normals(mesh)
    for c in (0.7, -1.3):
        o = oracle_lib.Oracle(2, mesh.verts, mesh.cells, p=3, n_lo=12, n_hi=20, flux="burgers")
        u = np.full(mesh.n_cell, c)
        _, alpha = o.rhs(u)
        expect = abs(c) * np.max(np.abs(n[:, 0] + n[:, 1]))
        assert abs(alpha - expect) <= 1e-13 * expect, (alpha, expect)
        # the area-scaled normal would give a clearly different bound
        scaled = abs(c) * np.max(np.abs(n[:, 0] + n[:, 1]) * ln)
        assert abs(scaled - expect) > 0.1 * expect


def test_alpha_uniform_euler_state(oracle_lib):
    """Euler, one uniform state: alpha = max over facets |v.n| + sqrt(gamma p / rho)."""
    mesh = jittered_square(10, 0.3, 2102)
    n, _ = _unit_edge_normals(mesh)
    gamma = 1.4
    rho, vx, vy, pr = 1.2, 0.3, -0.5, 0.8
    E = pr / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    o = oracle_lib.Oracle(2, mesh.verts, mesh.cells, p=3, n_lo=12, n_hi=20, flux="euler", gamma=gamma)
    u = np.stack([np.full(mesh.n_cell, s) for s in (rho, rho * vx, rho * vy, E)])
    _, alpha = o.rhs(u)
    expect = np.max(np.abs(vx * n[:, 0] + vy * n[:, 1])) + np.sqrt(gamma * pr / rho)
    assert abs(alpha - expect) <= 1e-13 * expect, (alpha, expect)


def test_alpha_comes_from_facet_values(oracle_lib):
    """1-D Burgers on a uniform periodic grid, plain least squares (unit
    weights) of a quadratic on the 5-cell window i-2..i+2, piecewise-constant
    data 0 / 1 / 0.5.  The fit's facet values, computed here from the closed
    cell averages of 1, (x - x_i) and (x - x_i)^2 / 2 on a uniform grid,
    overshoot the largest cell average 1; alpha is the largest |value| over
    both facets of every cell.  The left and right facets reach different
    maxima, so a one-sided sweep would differ too."""
    N = 20
    mesh = uniform_periodic_line(N)
    h = 1.0 / N
    u = np.zeros(N)
    u[5:10] = 1.0
    u[10:14] = 0.5
    o = oracle_lib.Oracle(1, mesh.verts, mesh.cells, True, p=3, n_lo=5, n_hi=5, flux="burgers", weight_mode=1)
    _, alpha = o.rhs(u)
    # cell averages over cell i + j of 1, x - x_i, (x - x_i)^2 / 2
    A = np.array([[1.0, j * h, 0.5 * (j * j * h * h + h * h / 12.0)] for j in range(-2, 3)])
    right, left = [], []
    for i in range(N):
        b = np.array([u[(i + j) % N] for j in range(-2, 3)])
        v = np.linalg.lstsq(A, b, rcond=None)[0]
        right.append(v[0] + v[1] * (h / 2) + v[2] * (h * h / 8))
        left.append(v[0] - v[1] * (h / 2) + v[2] * (h * h / 8))
    expect = max(np.max(np.abs(right)), np.max(np.abs(left)))
    assert abs(alpha - expect) <= 1e-12 * expect, (alpha, expect)
    assert expect > np.max(np.abs(u)) + 0.1          # averages alone would give 1
    assert abs(np.max(np.abs(right)) - np.max(np.abs(left))) > 0.05
