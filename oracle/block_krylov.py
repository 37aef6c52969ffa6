"""Oracle: block Krylov approximation of sign(A) B for several sources at once.

TEST INFRASTRUCTURE ONLY.

Not the paper's method: a multi-source variant of its Eq. 11 and Eq. 22.  One
Krylov space is built from all s sources together.  These are the block full
orthogonalisation (block FOM) approximations of f(A) B, written from their
definition:

* Block Arnoldi: B_ominus = V_1 R_0 (thin QR, V_1 N x s), then for each block
  step A V_j is orthogonalised against all previous blocks by classical
  Gram-Schmidt applied twice, and its QR factorisation gives V_{j+1} and the
  subdiagonal block H_{j+1,j}.  Then A V_K = V_K H_K + V_{K+1} H_{K+1,K} E_K^T,
  with H_K block upper Hessenberg (K s x K s).
* Approximation: f(A) B ~ V_K f(H_K) E_1 R_0.  With s = 1 this is Eq. 11.
* LR deflation as in Eq. 21-22: B = R G^{-1} L^dag B + B_ominus, the block
  recurrence runs on B_ominus (re-projected every step), and
  sign(A) B ~ R sgn(Lambda) G^{-1} L^dag B + V_K sign(H_K) E_1 R_0.
* A block is rank deficient when an R diagonal entry falls below 1e-12 of the
  block's largest column norm; the recurrence then stops there (the space is
  then invariant up to that tolerance for the block, the block analogue of a
  happy breakdown).
"""
from __future__ import annotations

import numpy as np

from .krylov import Deflation
from .sign_dense import sign_newton, sgn


def block_arnoldi(matvec_block, b0, kblocks, project=None, rank_rel=1e-12):
    """Block Arnoldi with block CGS2.  b0: N x s.

    Returns (V (N, (K+1) s), H ((K+1) s, K s), R0 (s x s), K_done)."""
    n, s = b0.shape
    v1, r0 = np.linalg.qr(b0)
    vmat = np.zeros((n, (kblocks + 1) * s), dtype=np.complex128)
    hmat = np.zeros(((kblocks + 1) * s, kblocks * s), dtype=np.complex128)
    vmat[:, :s] = v1
    for j in range(kblocks):
        w = matvec_block(vmat[:, j * s:(j + 1) * s])
        if project is not None:
            w = project(w)
        q = vmat[:, : (j + 1) * s]
        h = q.conj().T @ w
        w = w - q @ h
        h2 = q.conj().T @ w
        w = w - q @ h2
        hmat[: (j + 1) * s, j * s:(j + 1) * s] = h + h2
        vn, hs = np.linalg.qr(w)
        hmat[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = hs
        d = np.abs(np.diag(hs))
        if d.min() <= rank_rel * max(np.linalg.norm(w, axis=0).max(), np.abs(hmat).max()):
            return vmat[:, : (j + 2) * s], hmat[: (j + 2) * s, : (j + 1) * s], r0, j + 1
        vmat[:, (j + 1) * s:(j + 2) * s] = vn
    return vmat, hmat, r0, kblocks


def block_lr_sign(matvec, b, defl: Deflation | None, kblocks):
    """sign(A) B for the N x s block B after K block steps.  Returns (Y, info)."""
    n, s = b.shape
    mvb = lambda x: np.stack([matvec(x[:, i]) for i in range(x.shape[1])], axis=1)  # noqa: E731
    if defl is not None and defl.m:
        c = np.linalg.solve(defl.g, defl.l.conj().T @ b)
        bo = b - defl.r @ c
        proj = lambda w: w - defl.r @ np.linalg.solve(defl.g, defl.l.conj().T @ w)  # noqa: E731
        y = defl.r @ (sgn(defl.lam)[:, None] * c)
    else:
        bo, proj, y = b, None, np.zeros_like(b)
    vmat, hmat, r0, kd = block_arnoldi(mvb, bo, kblocks, project=proj)
    fh = sign_newton(hmat[: kd * s, : kd * s])
    y = y + vmat[:, : kd * s] @ (fh[:, :s] @ r0)
    return y, dict(k_used=kd, hk=hmat, r0=r0, dim=kd * s)
