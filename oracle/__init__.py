"""Plain FP64 CPU oracle for the PRADMM sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  The product (the HIP library and its
Python binding) never imports it, and this package never imports the
product: the two share no code, no constants, no pre- or post-processing.
The only thing both sides consume is the seeded input generator in
``pgo_synth``, which holds none of the method's arithmetic.

Layout
  quat.py    quaternion algebra of App. A.2 (product, conjugate, M, W, D,
             rotation by sandwiching)
  prep.py    boundary preparation: SO(3) projection by SVD, rotation matrix to
             unit quaternion by the symmetric 4x4 eigenvector method, vertex
             sign rule, edge sign alignment against the initial poses
  pradmm.py  the iteration (eq. 3a-3f, Alg. 1) with every subproblem written in
             the G-matrix form of App. B, cost of model (1), augmented
             Lagrangian, residuals of App. E.1, and a reference adjoint by
             automatic differentiation through the unrolled FP64 sweeps
  gn.py      brute-force local optimisation of model (1) (library least
             squares) for tiny graphs

Parity status of each function is stated in its docstring; none is
"parity unpinned" except where noted.
"""
