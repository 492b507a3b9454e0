"""FP64 CPU oracle for the mesh-registration hot path -- TEST INFRASTRUCTURE.

Plain, slow NumPy/SciPy code written from the paper (Baghaie, Yu, D'souza,
"Fast Mesh-Based Medical Image Registration", arXiv:1411.2141) to check the
HIP library against.  It shares no code with the library: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The library never calls it and never falls back to it.

Modules:

* ``bspline``      -- cubic B-spline prefilter and evaluation (abstract: spline
  interpolation of both images at the nodes).
* ``mesh``         -- tables T1-T6 (Algorithm 1 pre-computation), P1 element
  gradients (eq. 9), stiffness, mass and lumped mass (eq. 10, Section 2.3).
* ``registration`` -- the iteration (eq. 3-8, Algorithm 1), warp and MSD, and
  the loop to convergence (a relative-MSD stopping rule).
* ``adjoint``      -- reverse-mode gradient of the final MSD.

Pins (see ``tests/test_oracle_*.py``): spline interpolation and quadratic
reproduction, scipy's cubic spline as an independent evaluator, closed-form
element matrices, symmetry and zero row sums of the stiffness, eq. 9 against
exact gradients of linear functions, dense solves on tiny meshes, fixed
points, translation recovery, integer-shift warps, brute-force pixel
location, adjoint dot-product identities and central finite differences.
"""
from . import adjoint, bspline, mesh, registration

__all__ = ["adjoint", "bspline", "mesh", "registration"]
