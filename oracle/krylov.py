"""Oracle: Arnoldi approximation of f(A)x with LR deflation, step by step.

TEST INFRASTRUCTURE ONLY.

* Arnoldi recurrence (Eq. 7): A V_k = V_k H_k + beta_k v_{k+1} e_k^T with
  v_1 = x/|x|; orthonormal V_k, upper Hessenberg H_k.  The paper does not say
  how the long recurrence is orthogonalised; this uses classical Gram-Schmidt
  applied twice per step (CGS2), with h_{j+1,j} = |w| real and positive.
  A happy breakdown (h_{j+1,j} <= 1e-14 |H_j|_F) ends the recurrence early:
  the Krylov space is then invariant and the approximation exact.
* Arnoldi approximation (Eq. 11): f(A)x ~ beta V_k f(H_k) e_1.
* LR deflation (Eq. 20-22): with right/left eigenvectors A R = R Lambda,
  L^dag A = Lambda L^dag, x = x_par + x_ominus, x_par = R G^{-1} L^dag x with
  G = L^dag R (G = I under the paper's normalisation l_i^dag r_i = 1, and
  G^{-1} keeps the projector oblique and exact when it is not), and
    f(A) x ~ R f(Lambda) G^{-1} L^dag x + beta V_k f(H_k) e_1,
  the Arnoldi part built on x_ominus.  Optionally every new Arnoldi vector is
  re-projected with (1 - R G^{-1} L^dag), which is the identity in exact
  arithmetic (the Krylov space of x_ominus does not mix with Omega_m).
* Convergence estimate (the paper gives no stopping rule): every `check`
  steps s_j = f(H_j) e_1 is recomputed and
    est_j = beta |s_j - [s_{j'}; 0]| / |b|
  with j' the previous checkpoint; the run stops once est_j <= tol.
"""
from __future__ import annotations

import numpy as np

from .sign_dense import sign_eig, sign_newton, sgn


def arnoldi_cgs2(matvec, x, k, project=None, breakdown_rel=1e-14):
    """k Arnoldi steps with CGS2.  Returns V (N, k+1), H ((k+1), k), beta, k_done."""
    n = x.shape[0]
    beta = float(np.linalg.norm(x))
    vmat = np.zeros((n, k + 1), dtype=np.complex128)
    hmat = np.zeros((k + 1, k), dtype=np.complex128)
    vmat[:, 0] = x / beta
    for j in range(k):
        w = matvec(vmat[:, j])
        if project is not None:
            w = project(w)
        basis = vmat[:, : j + 1]
        h = basis.conj().T @ w
        w = w - basis @ h
        h2 = basis.conj().T @ w
        w = w - basis @ h2
        h = h + h2
        hmat[: j + 1, j] = h
        hn = float(np.linalg.norm(w))
        hmat[j + 1, j] = hn
        if hn <= breakdown_rel * np.linalg.norm(hmat[: j + 2, : j + 1]):
            return vmat[:, : j + 2], hmat[: j + 2, : j + 1], beta, j + 1
        vmat[:, j + 1] = w / hn
    return vmat, hmat, beta, k


def small_sign_e1(hk, route="newton"):
    """First column of sign(H_k) for the small square Hessenberg H_k."""
    if route == "newton":
        return sign_newton(hk)[:, 0]
    if route == "eig":
        return sign_eig(hk)[:, 0]
    raise ValueError(route)


class Deflation:
    """Critical eigen-data (R, L, lambda) and the oblique projector of Eq. 20-21."""

    def __init__(self, r, l, lam):
        self.r = np.asarray(r, dtype=np.complex128)
        self.l = np.asarray(l, dtype=np.complex128)
        self.lam = np.asarray(lam, dtype=np.complex128)
        self.g = self.l.conj().T @ self.r if self.r.shape[1] else np.zeros((0, 0))

    @property
    def m(self):
        return self.r.shape[1]

    def coeffs(self, x):
        """c = G^{-1} L^dag x."""
        if self.m == 0:
            return np.zeros(0, dtype=np.complex128)
        return np.linalg.solve(self.g, self.l.conj().T @ x)

    def split(self, x):
        """(c, x_ominus) with x_par = R c and x_ominus = x - x_par (Eq. 21)."""
        c = self.coeffs(x)
        return c, (x - self.r @ c if self.m else x.copy())

    def project_out(self, w):
        return w - self.r @ self.coeffs(w) if self.m else w

    def exact_part(self, c):
        """R f(Lambda) c with f = sgn (Eq. 21, first term)."""
        if self.m == 0:
            return 0.0
        return self.r @ (sgn(self.lam) * c)


def lr_arnoldi_sign(matvec, b, defl: Deflation | None, k, reproject=True,
                    route="newton", check=None, tol=None):
    """sign(A) b by Eq. 22.  Returns (y, info).

    With check/tol set, the recurrence stops at the first checkpoint whose
    estimate is <= tol (at most k steps); otherwise exactly k steps are taken.
    """
    defl = defl if defl is not None else Deflation(np.zeros((b.size, 0)),
                                                   np.zeros((b.size, 0)), np.zeros(0))
    c, xo = defl.split(b)
    proj = defl.project_out if (reproject and defl.m) else None
    vmat, hmat, beta, kd = arnoldi_cgs2(matvec, xo, k, project=proj)
    est = np.nan
    k_used = kd
    if check and tol is not None:
        prev = None
        bn = float(np.linalg.norm(b))
        for j in list(range(check, kd + 1, check)) + ([kd] if kd % check else []):
            s = small_sign_e1(hmat[:j, :j], route)
            if prev is not None:
                d = s.copy()
                d[: prev.size] -= prev
                est = beta * float(np.linalg.norm(d)) / bn
                if est <= tol:
                    k_used = j
                    break
            prev = s
            k_used = j
    s = small_sign_e1(hmat[:k_used, :k_used], route)
    y = defl.exact_part(c) + beta * (vmat[:, :k_used] @ s)
    return y, dict(k_used=k_used, beta=beta, est=est, hk=hmat[: k_used + 1, :k_used],
                   c=c, s=s)
