"""Plain FP64 CPU oracle for the tensor B-spline implicit heat step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call or execute this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, tables or constants with the GPU path: every number here is
derived from the B-spline definitions of the paper (Shulga et al., "Tensor
B-Spline Numerical Methods for PDEs", arXiv:1904.03057).

Modules
  bspline   centred B-splines, Galerkin taps, Fourier symbols   (Sec. 2.3, Table 1)
  operator  1-D Toeplitz matrices, separable apply, dense Kronecker, RHS
                                                               (Sec. 2.4, tensor form F(c)=t and
                                                                the separable kernel decomposition)
  exact     exact implicit step: FFT (periodic), fast diagonalisation (Dirichlet)
  solvers   Hestenes-Stiefel CG (Sec. 2.5, step 3) and mixed-precision refinement
  cnn       FP64 reference of the learned initial-guess network (not in the paper)
  rounding  bf16 round-to-nearest-even, done bit-exactly on float32 bit patterns

Parity pins (tests/test_oracle_*.py): exact rational taps and the textbook n=1
FEM matrices, Table tblFlop1d (values printed in the paper), dense Kronecker
assembly at <= 8^3, the closed-form B-spline symbol from Poisson summation,
dense Cholesky at <= 16^3, polynomial reproduction, torch.nn.functional.conv3d,
central finite differences and the closed-form first Adam step.
The learned-guess *gain* is empirical: "parity unpinned" (only the fallback
invariant is pinned).
"""
