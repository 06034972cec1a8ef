"""Plain FP64 CPU oracle for the Nystrom-accelerated primal LS-SVM ODE solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP library.  Every function is a direct,
unblocked transcription of the definitions in arXiv 2510.04094 (section and
equation cited in each docstring), written for a reader to check by eye
against the paper, in float64 with NumPy / SciPy primitives (eigh, solve,
lstsq) as single steps.

Modules
  rbf       RBF kernel and its derivatives (Sec. 3, eq. for nabla^a_c K)
  nystrom   landmarks, K_mm eigendecomposition, explicit feature map (App. A.2)
  linear    Lemma 1 primal KKT system for p-th order linear ODEs (Sec. 3.1, App. A.3/A.4)
  newton    Lemma 2 Newton iteration for first-order nonlinear ODEs (Sec. 3.2, App. A.5)
  adjoint   gradient of a loss on y_hat through the Lemma 1 solve (no paper
            section: derived from the Lemma 1 Lagrangian, see module docstring)
  dual      dual LS-SVM for linear ODEs with an arbitrary kernel (Sec. 2 / App. A.1),
            used as an independent cross-check of the primal solve
"""
from . import rbf, nystrom, linear, newton, adjoint, dual  # noqa: F401
