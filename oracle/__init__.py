"""Plain FP64 CPU oracle for the mODIL iteration (test infrastructure only).

This package is the independent reference that the HIP path is checked
against.  It is written from the paper (Karnakov, Litvinov & Koumoutsakos,
"Flow reconstruction by multiresolution optimization of a discrete loss with
automatic differentiation", arXiv 2303.04679) and shares no code with the
product package: it imports nothing from it, and the product never imports
this package.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may use it.

Everything is double precision on the CPU.  Loss terms are written with
explicit array slicing; gradients are obtained by reverse-mode automatic
differentiation (torch.autograd), which is how the paper itself obtains the
gradient of the discrete loss (Section 2.1 and the end of Section 2.2).

Modules
  multigrid  interpolation operators T (cell and node based), the multigrid
             decomposition M_L in Horner and direct form, and its transpose
  operators  discrete residuals and loss terms of each PDE problem
  adam       the Adam update (Kingma & Ba)
  reference  forward solvers that produce reference fields / measurements
  cnn        the warm-start convolutional network (forward, loss)
"""
