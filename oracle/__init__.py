"""WLS-ENO oracle: a plain, slow FP64 CPU reference of the finite-volume path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything in
this package.  The GPU library never uses it, and it shares no code, header,
table or helper with the GPU library; both sides only read the same seeded
inputs from ``workloads``.

Layout:

* ``wlseno_oracle.c`` -- per-cell numerics in plain C (Taylor/cell-average
  matrix by exact simplex integration, weights, column-scaled Householder QR
  with column pivoting, evaluation, Lax-Friedrichs flux, right-hand side,
  third-order TVD Runge-Kutta);
* ``mesh.py`` -- topology, geometry, facet quadrature and k-ring stencils
  (numpy and Python sets);
* ``core.py`` -- the ctypes harness (``Oracle``).

Every function cites the passage of the paper it follows.  Pins that tie the
oracle to the paper and to mathematics (not to itself) live in
``tests/test_oracle_*.py``.  Functions without such a pin are marked
"parity unpinned" where they are defined; at present that is the k-ring
stencil *sets* beyond the cases the tests enumerate by hand and cells of real
meshes whose numerical rank is truncated (the truncation rule is pinned on
constructed matrices).  Which cells the Euler positivity fallback and the
balanced refit select is pinned through their definitions only: the first
(unlimited) fit rebuilt from this oracle's own cell matrices, weights and
solver.
"""

from .core import (Oracle, build, basis, num_coeffs, wls_qrcp_solve, simplex_avg_monomial, eval_taylor, from_workload,
                   char_basis, euler_normal_flux)
from .mesh import OracleMesh

__all__ = ["Oracle", "OracleMesh", "build", "basis", "num_coeffs", "wls_qrcp_solve",
           "simplex_avg_monomial", "eval_taylor", "from_workload"]
