"""Plain FP64 CPU oracle for the parametrix remainder-operator apply and solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the HIP path.

What it computes (Goodwill & O'Neil, "A parametrix method for elliptic surface
PDEs"), for div_G(a grad_G u) = f on a closed surface (c = 0, b = 0):

* ``geometry``  node normals, area elements, quadrature weights, mean curvature
  (Section 2.2 and the Nystrom rule of Section 6.1), patch centroids and radii
  and the near criterion (Section 6.1.2).
* ``kernels``   the parametrix K = G(|x - x'|; a(x')) and its remainder R written
  as in eq:explicit_remainder with c = 0 (Theorem 4.x), and R_LB
  (eq:explicit_remainderLB).
* ``rules``     the singular (self) rule in polar coordinates about the target
  pre-image (Section 6.1.1, eq:radial_int) and the nearly singular rule by
  subdivision of the parameter square (Section 6.1.2), both on quad patches.
* ``operator``  the Nystrom system sigma + R[sigma] + int sigma = f (eq:IE with
  the rank-one term of Section 3), its dense solve, and the representation
  u = K[sigma] made mean zero (eq:representation).
* ``cfar``      the same smooth-rule (far) sums in plain C with OpenMP (``far.c``,
  compiled by ``cfar.build``), for whole-operator applies at large N.
* ``gmres``     GMRES with classical Gram-Schmidt twice, for systems beyond dense LU.
* ``system``    the whole operator at large N (blocks from worker processes, C far
  sums, a sparse matrix of the blocks), its GMRES solve and representation, and
  sampled rows of the operator.

Pinned by ``tests/test_oracle_pins.py`` (closed forms, invariants, the
diagonal limit eq:limiting_behaviour, exact integrals of the rules, and
brute-force agreement) and ``tests/test_oracle_large.py`` (C sums against the
NumPy rows and the unit-sphere closed form, GMRES against dense LU, the whole
system against the dense operator).  No function here is "parity unpinned".
"""
