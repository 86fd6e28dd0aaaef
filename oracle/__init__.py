"""Plain CPU oracle for the structured-sketching hot path (test infrastructure).

This package is the reference that the GPU library is checked against. It is
slow on purpose: every function follows the paper's definitions or algorithm
steps directly, in float64 NumPy/SciPy, with no blocking, fusion or
reordering beyond what the definition states.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it. The GPU library never imports, links or calls
anything in here, and this package imports nothing from the GPU library.

Paper: Camano, Epperly, Meyer, Tropp, "Faster Linear Algebra Algorithms with
Structured Random Matrices" (arXiv 2508.21189).

Modules
  philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11),
             the random source for every sketch (readings: see each function).
  sketches   SparseStack (Def. 1.5), CountSketch (eq. B.1), SRTT (eq. 1.1),
             SparseRTT (Def. 1.7, SparseCol of Def. 4.1),
             Gaussian test matrix (Def. 1.4): dense construction and
             application S @ A, A @ S^T, S^T @ Y.
  lstsq      sketch-and-solve (Alg. 3), exact least squares by Householder
             TSQR, sketch-and-precondition with LSQR (Sec. 1.4 remark).
  lowrank    randomized SVD (Alg. 1) and the spectral-error estimate.
  metrics    subspace-embedding distortion (Prop. 1.9, Defs. 1.1-1.2),
             coherence, isotropy statistics.

Parity status of each function is recorded in its docstring; functions with
no independent pin say "parity unpinned".
"""
