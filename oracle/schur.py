"""Oracle: Arnoldi approximation of f(A)x with Schur deflation (Eq. 13-19).

TEST INFRASTRUCTURE ONLY.

* Schur basis (Eq. 13): S_m is an orthonormal basis of the span of the m
  critical right eigenvectors, and A S_m = S_m T_m with T_m = S_m^dag A S_m.
  S_m comes from a QR factorisation of the eigenvector matrix, R = S_m U, so
  T_m = U Lambda U^{-1} is upper triangular with the eigenvalues, in R's column
  order, on its diagonal.
* Modified Arnoldi (Eq. 14): v_1 = x_perp / beta with x_perp = (1 - S S^dag) x
  and beta = |x_perp|; beta <= 1e-14 |x| counts as x in Omega_m (no Krylov
  part).  Each new vector A v_j is orthogonalised against the
  composite basis (S_m, V_j), by classical Gram-Schmidt applied twice.  Its
  S_m coefficients are column j of X = S_m^dag A V_k, its V_j coefficients and
  its norm column j of H_k.
* Eq. 15-17: H = [[T_m, X], [0, H_k]] and f(H) = [[f(T_m), Y], [0, f(H_k)]],
  with Y the solution of the Sylvester equation of Eq. 18.  The paper cites a
  dedicated triangular/Hessenberg solver without giving it; here scipy's
  Bartels-Stewart routine solves it.
* Eq. 19: f(A) x ~ S_m f(T_m) S_m^dag x + (S_m Y + V_k f(H_k)) beta e_1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .sign_dense import sign_newton


def schur_basis(r: np.ndarray, a_apply) -> tuple[np.ndarray, np.ndarray]:
    """(S_m, T_m) of Eq. 13 from right eigenvectors r (N x m); a_apply(X) = A X."""
    if r.shape[1] == 0:
        return np.zeros((r.shape[0], 0), dtype=np.complex128), np.zeros((0, 0), np.complex128)
    s, _ = np.linalg.qr(r)
    t = s.conj().T @ a_apply(s)
    return s, t


def schur_arnoldi(matvec, x, s, k, breakdown_rel=1e-14):
    """k steps of the modified Arnoldi process of Eq. 14.

    Returns (V (N, k_done+1), H_k ((k_done+1), k_done), X (m, k_done), beta,
    coefficients S^dag x, k_done)."""
    n, m = x.shape[0], s.shape[1]
    c0 = s.conj().T @ x
    xp = x - s @ c0
    beta = float(np.linalg.norm(xp))
    vmat = np.zeros((n, k + 1), dtype=np.complex128)
    hmat = np.zeros((k + 1, k), dtype=np.complex128)
    xmat = np.zeros((m, k), dtype=np.complex128)
    if beta <= 1e-14 * float(np.linalg.norm(x)):   # x lies in Omega_m (to rounding)
        return vmat[:, :0], hmat[:0, :0], xmat[:, :0], 0.0, c0, 0
    vmat[:, 0] = xp / beta
    for j in range(k):
        w = matvec(vmat[:, j])
        q = np.concatenate([s, vmat[:, : j + 1]], axis=1)
        h = q.conj().T @ w
        w = w - q @ h
        h2 = q.conj().T @ w
        w = w - q @ h2
        h = h + h2
        xmat[:, j] = h[:m]
        hmat[: j + 1, j] = h[m:]
        hn = float(np.linalg.norm(w))
        hmat[j + 1, j] = hn
        if hn <= breakdown_rel * np.linalg.norm(hmat[: j + 2, : j + 1]):
            kd = j + 1
            return vmat[:, : kd + 1], hmat[: kd + 1, :kd], xmat[:, :kd], beta, c0, kd
        vmat[:, j + 1] = w / hn
    return vmat, hmat, xmat, beta, c0, k


def coupling_y(t, fT, hk, fH, xmat):
    """Y of Eq. 18: T Y - Y H_k = f(T) X - X f(H_k)."""
    return scipy.linalg.solve_sylvester(t, -hk, fT @ xmat - xmat @ fH)


def schur_arnoldi_sign(matvec, b, s, t, k):
    """sign(A) b by Eq. 19 after exactly k modified Arnoldi steps (fewer on a
    happy breakdown).  Returns (y, info)."""
    m = s.shape[1]
    vmat, hmat, xmat, beta, c0, kd = schur_arnoldi(matvec, b, s, k)
    fT = sign_newton(t) if m else np.zeros((0, 0), np.complex128)
    y = s @ (fT @ c0) if m else np.zeros_like(b)
    if kd == 0:
        return y, dict(k_used=0, beta=beta, x=xmat, hk=hmat, y_coupling=None)
    hk = hmat[:kd, :kd]
    fH = sign_newton(hk)
    if m:
        ycp = coupling_y(t, fT, hk, fH, xmat)
        y = y + beta * (s @ ycp[:, 0])
    else:
        ycp = np.zeros((0, kd), np.complex128)
    y = y + beta * (vmat[:, :kd] @ fH[:, 0])
    return y, dict(k_used=kd, beta=beta, x=xmat, hk=hmat, y_coupling=ycp, fT=fT, fH=fH)
