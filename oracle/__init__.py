"""CPU oracle for y = sign(H_w(mu)) b (Bloch, Wettig, Frommer, Lang).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls, links or imports it, and it shares no code with the GPU library: the
two meet only at the seeded inputs of ``lattice_inputs``.

Everything is plain numpy / scipy in float64 / complex128:

* ``dirac``      -- explicit D_w(mu) and H_w(mu) = gamma_5 D_w(mu)   (Eq. 1-2)
* ``sign_dense`` -- sign(A) by the spectral definition and by Newton  (Eq. 4-6)
* ``free_field`` -- closed form of sign(H) b at U = 1 (derived from Eq. 2)
* ``krylov``     -- Arnoldi + LR deflation, step by step            (Eq. 7, 11, 20-22)
* ``eigen``      -- critical left/right eigenpairs                  (Eq. 20)
* ``overlap``    -- D_ov = 1 + gamma_5 sign(H_w) and sign(H)^dag      (Eq. 1)
* ``schur``      -- Arnoldi with Schur deflation, Sylvester coupling    (Eq. 13-19)
* ``block_krylov`` -- block Arnoldi for several sources (not the paper's; Eq. 11, 22 per block)
"""
from .dirac import (gamma_matrices, kappa_of, wilson_dirac_sparse, hermitian_wilson_sparse,
                    hermitian_wilson_dense, gamma5_diag)
from .sign_dense import sign_eig, sign_eig_apply, sign_newton, sgn
from .free_field import (free_field_sign_apply, free_field_h_apply, free_field_spectrum,
                         free_field_h_of_p)
from .krylov import arnoldi_cgs2, lr_arnoldi_sign, small_sign_e1, Deflation
from .eigen import critical_dense, critical_sparse, critical_order, eig_residuals
from .overlap import overlap_apply, sign_adjoint_apply
from .schur import schur_basis, schur_arnoldi, schur_arnoldi_sign, coupling_y
from .block_krylov import block_arnoldi, block_lr_sign

__all__ = [n for n in dir() if not n.startswith("_")]
