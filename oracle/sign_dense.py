"""Oracle: the matrix sign function of a dense matrix, two independent routes.

TEST INFRASTRUCTURE ONLY.

Route E (spectral definition, Eq. 4-6): with A = U diag(lambda_i) U^{-1},
  sign(A) = U diag(sgn(Re lambda_i)) U^{-1},
using sgn(z) = z / sqrt(z^2) = sgn(Re z) with the square-root cut on the
negative real axis (Eq. 5).  Undefined when some Re lambda_i = 0.

Route N (the matrix iterations the paper refers to in the Arnoldi section,
Higham's survey): Roberts' Newton iteration X <- (X + X^{-1}) / 2 from
X_0 = A, which converges quadratically to sign(A).  Determinantal scaling
(Byers): X <- (mu X + (mu X)^{-1}) / 2 with mu = |det X|^{-1/n} while the
iteration is far from convergence.  Stopping is stagnation-aware: once the
relative change is small, stop as soon as it no longer shrinks.
"""
from __future__ import annotations

import numpy as np


def sgn(z):
    """sgn(z) = sgn(Re z) (Eq. 5)."""
    return np.where(np.real(z) > 0, 1.0, -1.0)


def sign_eig(a: np.ndarray, return_info: bool = False):
    """Route E: U diag(sgn Re lambda) U^{-1}."""
    lam, u = np.linalg.eig(a)
    s = u @ np.diag(sgn(lam).astype(a.dtype)) @ np.linalg.inv(u)
    if return_info:
        return s, dict(lam=lam, cond_u=np.linalg.cond(u),
                       min_abs_re=float(np.min(np.abs(lam.real))))
    return s


def sign_eig_apply(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Route E applied to a vector (or block): U (sgn(Re lambda) * U^{-1} b)."""
    lam, u = np.linalg.eig(a)
    c = np.linalg.solve(u, b)
    f = sgn(lam)
    return u @ (f[:, None] * c if c.ndim == 2 else f * c)


def sign_newton(a: np.ndarray, max_iter: int = 100, scale_until: float = 1e-2,
                return_info: bool = False):
    """Route N: scaled Newton iteration for sign(A)."""
    x = np.array(a, dtype=np.complex128, copy=True)
    n = x.shape[0]
    prev = np.inf
    it = 0
    change = np.inf
    scaled = True
    for it in range(1, max_iter + 1):
        if scaled:
            _, logdet = np.linalg.slogdet(x)
            mu = np.exp(-logdet / n)
        else:
            mu = 1.0
        xs = mu * x
        xn = 0.5 * (xs + np.linalg.inv(xs))
        change = np.linalg.norm(xn - x) / np.linalg.norm(xn)
        x = xn
        if change < scale_until:
            scaled = False
        if change < 1e-14:
            break
        if change < 1e-8 and change > 0.5 * prev:   # stagnation at rounding level
            break
        prev = change
    if return_info:
        return x, dict(iters=it, last_change=change,
                       x2_minus_i=float(np.linalg.norm(x @ x - np.eye(n)) / np.sqrt(n)))
    return x
