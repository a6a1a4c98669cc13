"""FP64 CPU oracle for abstract rendering of Gaussian-splat scenes.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__.py and the
CPU-baseline leg of bench.py may import or run anything in this package.  The
product path (the HIP library and its Python binding) never imports it; the two
share no code.

Modules:
  lf      linear forms over the normalised pose box and their relaxations
  pose    the camera sets (CAMERA6 box, ORBIT cell) as linear forms
  matinv  MatrixInv (Sec. 3.1) on 2x2 linear forms, and the adjugate inverse it is compared with
  crown   MatrixInv with its linear bounds propagated backward (CROWN-style)
  render  concrete renderer (Alg. GaussianSplat, BlendSort, BlendInd), FP64
  splat   AbstractSplat (Sec. 3.3): lower/upper images over a pose box
  refine  adaptive refinement of a pose box where MatrixInv fails (Sec. 3.1, 4.2)

Parity status: every function is pinned by the CPU tests (tests/test_oracle_*.py)
against closed forms, the paper's printed examples, brute force on small inputs,
or the soundness theorem.  No function is "parity unpinned".
"""
