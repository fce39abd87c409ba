"""CPU FP64 oracle for the inexact low-rank Sylvester ADI path.

Test infrastructure only: tests/, the smoke check and the CPU-baseline leg of
the benchmark may import it; the library and its Python binding never do, and
this package imports nothing from them.  Everything here is plain NumPy/SciPy
in FP64, written from the paper (Algorithm 1, eqs. (lradi_basic),
(adi_res_inexact), (ADI_relax1_prak), (ADI_relax2_prak), (simple_tols),
(one_side), (upd_resgap); Sec. 4 for the test matrices), with sparse-direct
inner solves, so that it can be checked by eye against the text.

Modules:
  convdiff    CSR of the upwind convection-diffusion coefficient matrices
  fadi        LR-ADI with direct solves, residual and difference norms,
              dense Bartels-Stewart reference
  controller  dynamic inner tolerances of Sec. 3.2
  lyap        Lyapunov special case (B = A^T, C = M^T, g = f), one solve
              per step, written in its own residual-factor form
  gmres_ref   a plain block GMRES used to pin block-Krylov test cases
              (optionally right-preconditioned)
  precond     red-black ILU(0) of A + s I with Jacobi sweeps on the Schur
              complement, the inner solver's right preconditioner
"""
