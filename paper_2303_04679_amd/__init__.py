"""Multiresolution ODIL (mODIL) on AMD MI355X (gfx950).

The mODIL iteration of Karnakov, Litvinov & Koumoutsakos (arXiv 2303.04679):
multigrid decomposition of the unknown fields (Section 2.2), the discrete
ODIL loss (Section 2.1) with the residual operators of Section 3, its exact
adjoint and Adam on every level -- as hand-written HIP kernels behind the C
ABI in include/modil.h (libmodil.so), with this package as a thin binding.
"""
from .modil import Context, ProblemSpec, layout  # noqa: F401

__all__ = ["Context", "ProblemSpec", "layout"]
