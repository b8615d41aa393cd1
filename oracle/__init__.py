"""FP64 CPU oracle for one Levenberg-Marquardt iteration of holistic bundle adjustment.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does,
and it shares no code with the HIP library.

What it computes, and where each part comes from in the paper:

* residuals of every family - point reprojection (Sec. 3.1 Eq. 1), line
  endpoint reprojection with 4-vector endpoint perpendicular vectors
  (Sec. 3.2 Eq. 4), VP angular residual (Sec. 3.3 Eq. 6 / App. B), group-
  induced point and line reprojection (Sec. 3.3 Eqs. 7-8, plane-line
  projection of App. B), cross-feature point->line and line->point distances
  (Sec. 3.4 Eqs. 11-12) - in ``oracle.model``;
* expansion of associations into residual records with the visibility rules
  of Sec. 3.3 and 3.4 - in ``oracle.records``;
* Jacobians by complex-step differentiation of those residuals (exact to
  rounding), robust IRLS weighting, the normal equations of Sec. 3.1 Eq. 2 /
  Sec. 3.2 Eq. 5, the Schur complement of Eq. 3 formed densely, a Cholesky
  solve, back-substitution, the gain ratio and Marquardt/Nielsen damping,
  and the pixel-only relative-cost termination of Sec. 3.5 - in ``oracle.lm``;
* the learned block-Jacobi correction network in FP64 - in ``oracle.gnn``.

Readings where the paper is silent are listed in the design notes and in
each function's docstring.
"""
