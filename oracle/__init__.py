"""CPU FP64 oracle for the learned finite-temperature Fermi-operator expansion.

TEST INFRASTRUCTURE ONLY. This package is the independent checker of the GPU
path. Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import or run it; the product path never does, and it shares
no code, tables or helpers with the HIP library.

Two layers:

* ``oracle.fermi`` -- the plain definitions the method approximates:
  the Fermi-Dirac density matrix D = V f(Lambda) V^T and the electronic
  entropy S = sum_i s(lambda_i), computed by a dense FP64 eigendecomposition
  (Sec. II.A, Eq. FD_Func; Sec. III.B, Eqs. entropy-matrix and entropy).
* ``oracle.recursion`` -- the paper's algorithm written step by step in FP64:
  Gershgorin bounds, the affine rescale with flip and region-of-validity clamp
  (Sec. IV.1, Eqs. H', mu', beta', H0, conditions, flip), the MLSP2 layers
  (Eq. mlsp2, Alg. 1) and the entropy expansion (Eq. entropy expansion),
  composed as in Alg. 2. It separates model error (recursion vs definition)
  from arithmetic error (GPU vs recursion at the same coefficients).
* ``oracle.variants`` -- Skip-SP2 and Max-SP2 (Sec. III.A), scalar and matrix forms, the
  embeddings MLSP2 -> Skip-SP2 -> Max-SP2 (App. C) and their complex-step Jacobians.
* ``oracle.training`` -- the scalar recursion's Jacobian with respect to the
  coefficients (forward-mode sensitivities in FP64), the targets of Sec. III.C
  and the sampling densities, used to check the GPU trainer's kernels.

Parity status: every function here is pinned by a test in ``tests/`` against
closed forms, values printed in the paper, brute force or finite differences,
except where a docstring says "parity unpinned".
"""
from . import fermi, recursion, training, variants  # noqa: F401
