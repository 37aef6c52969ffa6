"""The overlap operator and the adjoint sign, dense (test infrastructure only).

* ``overlap_apply``       -- D_ov b = b + gamma_5 sign(H_w) b            (Eq. 1)
* ``sign_adjoint_apply``  -- sign(H)^dag b = sign(H^dag) b; for the Wilson
  operator H_w(mu)^dag = H_w(-mu), so the left eigenpairs of H_w(mu) serve as
  the right ones of the adjoint problem (the results section's remark on
  sign(H) and sign(H)^dag)
"""
import numpy as np

from .dirac import gamma5_diag
from .sign_dense import sign_eig_apply


def overlap_apply(h: np.ndarray, b: np.ndarray) -> np.ndarray:
    """D_ov b = b + gamma_5 sign(H_w) b (Eq. 1) for the dense H_w = h."""
    g5 = gamma5_diag(h.shape[0] // 12)
    s = sign_eig_apply(h, b)
    return b + (g5[:, None] * s if s.ndim == 2 else g5 * s)


def sign_adjoint_apply(h: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sign(H)^dag b, computed as sign(H^dag) b from the spectral definition."""
    return sign_eig_apply(h.conj().T, b)
