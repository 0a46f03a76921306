"""CPU FP64 oracle for the tensor-product multigrid (TPMG) preconditioned
flexible-CG solve of the anisotropic pressure-correction equation.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP library.

Everything follows Dedner, Mueller & Scheichl, "Efficient Multigrid
Preconditioners for Atmospheric Flow Simulations at High Aspect Ratio":
  mesh.py      icosahedral hierarchy and spherical geometry (Sections 4.1, 4.2,
               Appendix A)
  operator.py  finite-volume tensor-stencil operator (Appendix A, eqs.
               hatFunctionsNonFac / hatFunctionsFac; eq. ColumnEquation)
  tpmg.py      line smoother with the Thomas solve (eq. BlockJacobi),
               restriction/prolongation (Section 5), the TPMG V-cycle
               (Algorithm 1), flexible CG, Richardson rate, direct solve
  mlp.py       per-column MLP reference (forward, manual backward, Adam)

Parity status per function is stated in each module header; functions with
no independent pin say "parity unpinned".
"""
