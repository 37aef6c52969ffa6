"""Oracle: the Wilson-Dirac operator at chemical potential, assembled explicitly.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this.

Follows the paper's definition section (Eq. 2 and the text below it):

  [D_w(mu)]_{nm} = delta_{nm}
      - kappa sum_{j=1..3} (1+gamma_j) U_{n,j} delta_{n+j,m}
      - kappa sum_{j=1..3} (1-gamma_j) U^dag_{n-j,j} delta_{n-j,m}
      - kappa (1+gamma_4) e^{+mu} U_{n,4} delta_{n+4,m}
      - kappa (1-gamma_4) e^{-mu} U^dag_{n-4,4} delta_{n-4,m}

  kappa = 1 / (8 + 2 m_w),  m_w in (-2, 0);   H_w(mu) = gamma_5 D_w(mu)   (Eq. 1).

Readings where the paper is silent:
  * gamma basis: chiral, gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 =
    [[0, 1], [1, 0]], so gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 =
    diag(1, 1, -1, -1).
  * boundary conditions periodic; optional antiperiodic time direction
    (a factor -1 on temporal hops that wrap around).
  * index 3 (0-based) is the temporal direction carrying e^{+-mu}.
  * on a lattice of extent 2 the forward and backward neighbours coincide;
    both hop terms are added into the same block.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_PAULI = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def gamma_matrices():
    """(gamma_1, gamma_2, gamma_3, gamma_4, gamma_5) in the chiral basis."""
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in _PAULI]
    g.append(np.block([[z, one], [one, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g + [g5]


def kappa_of(m_w: float) -> float:
    """kappa = 1/(8 + 2 m_w) (definition section, below Eq. 2)."""
    return 1.0 / (8.0 + 2.0 * m_w)


def site_coords(dims):
    lx, ly, lz, lt = (int(v) for v in dims)
    s = np.arange(lx * ly * lz * lt)
    return np.stack([s % lx, (s // lx) % ly, (s // (lx * ly)) % lz,
                     s // (lx * ly * lz)], axis=1)


def site_index(coords, dims):
    lx, ly, lz, _ = (int(v) for v in dims)
    c = coords
    return c[:, 0] + lx * (c[:, 1] + ly * (c[:, 2] + lz * c[:, 3]))


def neighbour(dims, nu: int, step: int):
    """Site index of n + step*nu_hat for every n, and a flag for wrapping."""
    d = np.asarray(dims)
    c = site_coords(dims)
    moved = c.copy()
    moved[:, nu] = c[:, nu] + step
    wrapped = (moved[:, nu] < 0) | (moved[:, nu] >= d[nu])
    moved[:, nu] %= d[nu]
    return site_index(moved, dims), wrapped


def _backward_link(links, bwd, nu):
    """U^dag_{n-nu,nu} for every site n (bwd[n] = n - nu_hat)."""
    return np.conj(np.transpose(links[bwd, nu], (0, 2, 1)))


def wilson_dirac_sparse(links, dims, mu: float, m_w: float,
                        antiperiodic_t: bool = False) -> sp.csr_matrix:
    """D_w(mu) of Eq. 2 as an N x N CSR matrix, N = 12 V."""
    links = np.asarray(links, dtype=np.complex128)
    g = gamma_matrices()
    kap = kappa_of(m_w)
    v = links.shape[0]
    i12 = np.arange(12)
    rows, cols, vals = [], [], []
    # diagonal term delta_{nm}
    rows.append(np.arange(12 * v))
    cols.append(np.arange(12 * v))
    vals.append(np.ones(12 * v, dtype=np.complex128))
    eye4 = np.eye(4, dtype=np.complex128)
    for nu in range(4):
        fwd, fwd_wrap = neighbour(dims, nu, +1)
        bwd, bwd_wrap = neighbour(dims, nu, -1)
        ph_f = np.exp(mu) if nu == 3 else 1.0
        ph_b = np.exp(-mu) if nu == 3 else 1.0
        bc_f = np.ones(v)
        bc_b = np.ones(v)
        if nu == 3 and antiperiodic_t:
            bc_f = np.where(fwd_wrap, -1.0, 1.0)
            bc_b = np.where(bwd_wrap, -1.0, 1.0)
        # forward hop: -kappa (1+gamma_nu) e^{+mu delta_{nu,4}} U_{n,nu}, column block n+nu
        u_f = links[:, nu]                                   # U_{n,nu}
        blk_f = -kap * ph_f * bc_f[:, None, None] * np.einsum(
            "st,nab->nsatb", eye4 + g[nu], u_f).reshape(v, 12, 12)
        # backward hop: -kappa (1-gamma_nu) e^{-mu delta_{nu,4}} U^dag_{n-nu,nu}, column block n-nu
        u_b = _backward_link(links, bwd, nu)                    # U^dag_{n-nu,nu}
        blk_b = -kap * ph_b * bc_b[:, None, None] * np.einsum(
            "st,nab->nsatb", eye4 - g[nu], u_b).reshape(v, 12, 12)
        for blk, nb in ((blk_f, fwd), (blk_b, bwd)):
            r = (np.arange(v)[:, None, None] * 12 + i12[None, :, None])
            c = (nb[:, None, None] * 12 + i12[None, None, :])
            rows.append(np.broadcast_to(r, (v, 12, 12)).ravel())
            cols.append(np.broadcast_to(c, (v, 12, 12)).ravel())
            vals.append(blk.ravel())
    mat = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(12 * v, 12 * v))
    return mat.tocsr()  # duplicates (extent-2 directions) are summed


def gamma5_diag(v: int) -> np.ndarray:
    """Diagonal of gamma_5 (x) 1_color on the full vector space."""
    g5 = np.real(np.diag(gamma_matrices()[4]))
    return np.tile(np.repeat(g5, 3), v)


def hermitian_wilson_sparse(links, dims, mu, m_w, antiperiodic_t=False) -> sp.csr_matrix:
    """H_w(mu) = gamma_5 D_w(mu) (Eq. 1) as CSR."""
    d = wilson_dirac_sparse(links, dims, mu, m_w, antiperiodic_t)
    v = d.shape[0] // 12
    return (sp.diags(gamma5_diag(v)) @ d).tocsr()


def hermitian_wilson_dense(links, dims, mu, m_w, antiperiodic_t=False) -> np.ndarray:
    return hermitian_wilson_sparse(links, dims, mu, m_w, antiperiodic_t).toarray()
