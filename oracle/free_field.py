"""Oracle: closed form of sign(H_w(mu)) b on the free field (all links U = 1).

TEST INFRASTRUCTURE ONLY.

Derived from Eq. 2.  A plane wave psi_n = e^{i p.n} chi is mapped by D_w(mu)
with U = 1 to D(p) chi, where (using (1+g)e^{ip} + (1-g)e^{-ip} = 2 cos p +
2 i g sin p for the spatial hops and the same with p_4 -> p_4 - i mu for the
temporal one)

  D(p) = a(p) - 2 i kappa sum_j gamma_j sin p_j - 2 kappa gamma_4 sinh(mu + i p_4),
  a(p) = 1 - 2 kappa (sum_j cos p_j + cosh(mu + i p_4)).

Since gamma_5 anticommutes with every gamma_nu and the gamma_nu obey the
Clifford algebra, H(p) = gamma_5 D(p) satisfies H(p)^2 = s(p) 1 with

  s(p) = a^2 + 4 kappa^2 sum_j sin^2 p_j - 4 kappa^2 sinh^2(mu + i p_4).

The eigenvalues of H(p) are +-sqrt(s), so by Eq. 5 sign(H(p)) = H(p)/sqrt(s(p))
with the principal square root.  Momenta p_nu = 2 pi n_nu / L_nu, shifted by
pi / L_t in time for antiperiodic boundary conditions.  The colour structure
is the identity.
"""
from __future__ import annotations

import numpy as np

from .dirac import gamma_matrices, kappa_of


def _momenta(dims, antiperiodic_t):
    lx, ly, lz, lt = (int(v) for v in dims)
    px = 2 * np.pi * np.fft.fftfreq(lx) * 1.0
    py = 2 * np.pi * np.fft.fftfreq(ly)
    pz = 2 * np.pi * np.fft.fftfreq(lz)
    pt = 2 * np.pi * np.fft.fftfreq(lt) + (np.pi / lt if antiperiodic_t else 0.0)
    # array axes are ordered (t, z, y, x) because site = x + Lx(y + Ly(z + Lz t))
    P = np.meshgrid(pt, pz, py, px, indexing="ij")
    return P[3], P[2], P[1], P[0]


def free_field_h_of_p(dims, mu, m_w, antiperiodic_t=False):
    """H(p) for every momentum, shape (Lt, Lz, Ly, Lx, 4, 4), and s(p)."""
    g = gamma_matrices()
    kap = kappa_of(m_w)
    px, py, pz, pt = _momenta(dims, antiperiodic_t)
    zt = mu + 1j * pt
    a = 1 - 2 * kap * (np.cos(px) + np.cos(py) + np.cos(pz) + np.cosh(zt))
    d = (a[..., None, None] * np.eye(4)
         - 2j * kap * (np.sin(px)[..., None, None] * g[0]
                       + np.sin(py)[..., None, None] * g[1]
                       + np.sin(pz)[..., None, None] * g[2])
         - 2 * kap * np.sinh(zt)[..., None, None] * g[3])
    h = np.einsum("ij,...jk->...ik", g[4], d)
    s = a ** 2 + 4 * kap ** 2 * (np.sin(px) ** 2 + np.sin(py) ** 2 + np.sin(pz) ** 2) \
        - 4 * kap ** 2 * np.sinh(zt) ** 2
    return h, s


def free_field_spectrum(dims, mu, m_w, antiperiodic_t=False):
    """All 12 V eigenvalues of H_w(mu) at U = 1: +-sqrt(s(p)), each 6-fold."""
    _, s = free_field_h_of_p(dims, mu, m_w, antiperiodic_t)
    r = np.sqrt(s.astype(np.complex128)).ravel()
    return np.concatenate([np.repeat(r, 6), np.repeat(-r, 6)])


def free_field_apply(fn, dims, mu, m_w, b, antiperiodic_t=False):
    """y = f(H) b on the free field for f(H(p)) given per momentum by fn(h, s)."""
    lx, ly, lz, lt = (int(v) for v in dims)
    x = np.asarray(b, dtype=np.complex128).reshape(lt, lz, ly, lx, 4, 3)
    tw = None
    if antiperiodic_t:
        tw = np.exp(1j * np.pi * np.arange(lt) / lt)[:, None, None, None, None, None]
        x = x / tw
    xh = np.fft.fftn(x, axes=(0, 1, 2, 3))
    h, s = free_field_h_of_p(dims, mu, m_w, antiperiodic_t)
    f = fn(h, s)
    yh = np.einsum("...ij,...jc->...ic", f, xh)
    y = np.fft.ifftn(yh, axes=(0, 1, 2, 3))
    if antiperiodic_t:
        y = y * tw
    return y.reshape(-1)


def free_field_sign_apply(dims, mu, m_w, b, antiperiodic_t=False):
    """sign(H_w(mu)) b at U = 1 via H(p)/sqrt(s(p))."""
    return free_field_apply(lambda h, s: h / np.sqrt(s.astype(np.complex128))[..., None, None],
                            dims, mu, m_w, b, antiperiodic_t)


def free_field_h_apply(dims, mu, m_w, b, antiperiodic_t=False):
    """H_w(mu) b at U = 1 (momentum space), an independent check of the stencil."""
    return free_field_apply(lambda h, s: h, dims, mu, m_w, b, antiperiodic_t)
