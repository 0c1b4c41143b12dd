"""CPU oracle for the RMTR phase-field fracture hot path (TEST INFRASTRUCTURE).

Plain, slow, FP64 numpy/scipy code written from the paper's statement of the
method (Sec. 2 energy, Sec. 3 RMTR, Algorithms 1-3).  It shares no code with
the HIP library: only tests, the smoke check and the benchmark's CPU-baseline
leg may import it.  The product path never calls into this package.

Modules
  fem       discrete functional f, gradient, Hessian (assembled), Hv
  fields    nodal inclusion initialisation of c and the pressure field
  transfer  prolongation I, restriction R = I^T, projection P, box restriction
  qp        projected Gauss-Seidel and MPRGP for the box-constrained TR QP
  rmtr      trust-region steps (Alg. 2, 3) and the RMTR V-cycle (Alg. 1)
  cnn       3D convolutional network forward/backward in FP64 (learned proposal)
"""
