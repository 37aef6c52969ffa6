"""Oracle: critical eigenpairs of H_w(mu) for LR deflation (Eq. 20).

TEST INFRASTRUCTURE ONLY.

"Critical" eigenvalues are those close to the imaginary axis, where sgn is
discontinuous (Results section).  They are ordered here by |Re lambda|, ties
broken by |lambda| and then Im lambda.

Left eigenvectors: L^dag A = Lambda L^dag.  Because gamma_5 is Hermitian and
the backward hops carry the adjoint links and e^{-mu}, H_w(mu)^dag = H_w(-mu),
so the left eigenvectors of H_w(mu) are the right eigenvectors of H_w(-mu)
with the conjugate eigenvalues.  The dense route reads them off U^{-1}
instead, which fixes L^dag R = I directly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def critical_order(lam):
    lam = np.asarray(lam)
    return np.lexsort((lam.imag, np.abs(lam), np.abs(lam.real)))


def critical_dense(h: np.ndarray, m: int):
    """(R, L, lambda) of the m critical eigenpairs from a full eigendecomposition.

    Columns of R are right eigenvectors normalised to |r_i| = 1; L is chosen so
    that L^dag R = I (rows of U^{-1} for the selected eigenvalues)."""
    lam, u = np.linalg.eig(h)
    order = critical_order(lam)[:m]
    uinv = np.linalg.inv(u)
    r = u[:, order]
    l = uinv[order, :].conj().T
    nrm = np.linalg.norm(r, axis=0)
    r = r / nrm
    l = l * nrm
    return r, l, lam[order]


def critical_sparse(h_mu, h_minus_mu, m: int, extra: int = None, tol: float = 1e-13):
    """(R, L, lambda) via ARPACK shift-invert about 0 on H(mu) and H(-mu).

    Requests m + extra eigenvalues of smallest modulus from each, keeps the m of
    smallest |Re lambda| of H(mu) and pairs every right vector with the left one
    whose eigenvalue is the conjugate; then scales so that diag(L^dag R) = 1."""
    extra = max(4, m // 2) if extra is None else extra
    nev = m + extra
    lam_r, vr = spla.eigs(h_mu.tocsc(), k=nev, sigma=0.0, tol=tol)
    lam_l, vl = spla.eigs(h_minus_mu.tocsc(), k=nev, sigma=0.0, tol=tol)
    order = critical_order(lam_r)[:m]
    r = vr[:, order]
    lam = lam_r[order]
    l = np.zeros_like(r)
    for i, li in enumerate(lam):
        j = int(np.argmin(np.abs(lam_l - np.conj(li))))
        l[:, i] = vl[:, j]
    d = np.einsum("ni,ni->i", l.conj(), r)
    r = r / np.linalg.norm(r, axis=0)
    d = np.einsum("ni,ni->i", l.conj(), r)
    l = l / d.conj()
    return r, l, lam


def eig_residuals(h, r, l, lam):
    """max_i |H r_i - lam_i r_i| / |r_i| and the same for the left vectors."""
    rr = h @ r - r * lam
    ll = (h.conj().T @ l) - l * lam.conj()
    return (float(np.max(np.linalg.norm(rr, axis=0) / np.linalg.norm(r, axis=0))),
            float(np.max(np.linalg.norm(ll, axis=0) / np.linalg.norm(l, axis=0))))
