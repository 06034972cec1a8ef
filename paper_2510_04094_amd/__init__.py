"""nyls: Nystrom-accelerated primal LS-SVM ODE solver for AMD MI355X (gfx950).

The compute path is the HIP library `libnyls.so` (C ABI declared in
include/nyls.h); `paper_2510_04094_amd.nyls` is its thin Python binding.
Importing the package loads nothing: the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["nyls", "workloads"]
