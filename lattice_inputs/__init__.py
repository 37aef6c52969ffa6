"""Seeded synthetic inputs for sign(H_w(mu)) b: gauge links, sources, workloads.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It holds only input generation (random numbers, SU(3) sampling,
layouts); none of the method's arithmetic lives here.

The paper measures on two unspecified gauge configurations (a 4^4 and a 6^4
lattice, Results section); none is available, so every input is a seeded
synthetic stand-in:

* Haar-random SU(3) links: QR of a complex Ginibre matrix with the phases of
  diag(R) moved into Q (Mezzadri's recipe), then divided by the principal cube
  root of det(Q) so that det = 1.
* Disordered links U = exp(i eps H), H = sum_a h_a lambda_a / 2 over the eight
  Gell-Mann matrices with h_a ~ N(0, 1) (eps -> 0 is the free field U = 1).
* Sources: Gaussian complex (re, im iid N(0,1), then unit norm), point
  sources e_{site,spin,color}, or the paper's all-ones vector (normalised).

Layouts (the library boundary uses the same):
  site  = x + Lx*(y + Ly*(z + Lz*t))
  vector index i = (site*4 + spin)*3 + color         (complex128)
  links  U[site, nu, a, b],  nu = 0,1,2 spatial (x,y,z), nu = 3 temporal.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 710341

# Stream ids inside one (workload, instance) seed.
STREAM_LINKS = 0
STREAM_SOURCE = 1
STREAM_PARAMS = 2
STREAM_DEFL = 3


def rng_for(cfg: int, inst: int, stream: int) -> np.random.Generator:
    """PCG64 generator seeded by SeedSequence([710341, cfg, inst, stream])."""
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, inst, stream])))


def volume(dims) -> int:
    d = [int(v) for v in dims]
    return d[0] * d[1] * d[2] * d[3]


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, shape (n, 3, 3) complex128."""
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


def disordered_su3(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """n matrices exp(i eps H), H Gaussian traceless Hermitian (see module doc)."""
    h = rng.standard_normal((n, 8))
    herm = np.einsum("na,aij->nij", h, _gell_mann()) * 0.5
    w, vecs = np.linalg.eigh(herm)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", vecs, ph, vecs.conj())


def make_links(dims, kind: str = "haar", eps: float = 0.0, rng=None,
               cfg: int = 0, inst: int = 0) -> np.ndarray:
    """Links in boundary layout, shape (V, 4, 3, 3) complex128.

    kind: "haar" (Haar SU(3)), "disordered" (exp(i eps H)) or "unit" (U = 1).
    """
    v = volume(dims)
    if kind == "unit":
        out = np.zeros((v, 4, 3, 3), dtype=np.complex128)
        out[:, :, 0, 0] = out[:, :, 1, 1] = out[:, :, 2, 2] = 1.0
        return out
    if rng is None:
        rng = rng_for(cfg, inst, STREAM_LINKS)
    if kind == "haar":
        u = haar_su3(rng, 4 * v)
    elif kind == "disordered":
        u = disordered_su3(rng, 4 * v, eps)
    else:
        raise ValueError(f"unknown link kind {kind!r}")
    return np.ascontiguousarray(u.reshape(v, 4, 3, 3))


def round_links_fp32(links: np.ndarray) -> np.ndarray:
    """Round links once to complex64 and promote back exactly.

    For the mixed-precision workloads the rounded links *are* the instance:
    the FP64 oracle and the FP32-link GPU path then see the same operator.
    """
    return links.astype(np.complex64).astype(np.complex128)


def gaussian_source(dims, rng=None, cfg: int = 0, inst: int = 0) -> np.ndarray:
    n = 12 * volume(dims)
    if rng is None:
        rng = rng_for(cfg, inst, STREAM_SOURCE)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return b / np.linalg.norm(b)


def point_source(dims, site: int = 0, spin: int = 0, color: int = 0) -> np.ndarray:
    b = np.zeros(12 * volume(dims), dtype=np.complex128)
    b[(site * 4 + spin) * 3 + color] = 1.0
    return b


def ones_source(dims) -> np.ndarray:
    n = 12 * volume(dims)
    return np.full(n, 1.0 / np.sqrt(n), dtype=np.complex128)


def placeholder_deflation(n: int, m: int, cfg: int = 0, inst: int = 0):
    """(R, L, lambda) of the shapes of m deflation pairs for vectors of length n:
    unit Gaussian columns and values with |Re| in [0.05, 0.5].  They are not
    eigenpairs; they only give a timing run the memory traffic and arithmetic
    of an m-pair deflation."""
    rng = rng_for(cfg, inst, STREAM_DEFL)
    r = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    l = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    r /= np.linalg.norm(r, axis=0)
    l /= np.linalg.norm(l, axis=0)
    re = rng.uniform(0.05, 0.5, m) * rng.choice([-1.0, 1.0], m)
    lam = re + 1j * rng.uniform(-0.1, 0.1, m)
    return r, l, lam


# ---------------------------------------------------------------------------
# Workloads.  Index 0 is the small case the dense oracle handles in seconds;
# index 3 (16^4, 12 point sources, batched) is the headline single-GPU
# workload; 1, 2 and 4 are the other measured configurations.
# ---------------------------------------------------------------------------
WORKLOADS = [
    dict(name="haar4_mu0.3_m10", dims=(4, 4, 4, 4), kind="haar", eps=0.0,
         m_w=-1.5, mu=0.3, k_max=300, n_defl=10, tol=1e-8, link_prec="fp64",
         source="gaussian"),
    dict(name="dis8_eps0.6", dims=(8, 8, 8, 8), kind="disordered", eps=0.6,
         m_w=-1.5, mu=(0.1, 0.5), k_max=600, n_defl=(20, 40), tol=1e-10,
         link_prec="fp64", source="gaussian"),
    dict(name="haar12_fp32links", dims=(12, 12, 12, 12), kind="haar", eps=0.0,
         m_w=-1.8, mu=0.3, k_max=800, n_defl=30, tol=1e-8, link_prec="fp32",
         source="gaussian"),
    dict(name="dis16_12pt", dims=(16, 16, 16, 16), kind="disordered", eps=0.5,
         m_w=-1.5, mu=0.2, k_max=500, n_defl=40, tol=1e-8, link_prec="fp32",
         source="point12"),
    dict(name="uneven64", dims=None, kind="disordered", eps=None, m_w=None,
         mu=None, k_max=600, n_defl=None, tol=1e-8, link_prec="fp64",
         source="gaussian"),
]


def uneven_batch_params(n: int = 64, cfg: int = 4):
    """Instance parameters of the uneven batch: L in {6,8,10}, mu ~ U[0.05,0.5],
    m_w ~ U[-1.9,-1.2], eps ~ U[0.3,1.0], n_defl ~ U{8..32}."""
    rng = rng_for(cfg, 0, STREAM_PARAMS)
    out = []
    for i in range(n):
        L = int(rng.choice([6, 8, 10]))
        out.append(dict(inst=i, dims=(L, L, L, L), mu=float(rng.uniform(0.05, 0.5)),
                        m_w=float(rng.uniform(-1.9, -1.2)), eps=float(rng.uniform(0.3, 1.0)),
                        n_defl=int(rng.integers(8, 33))))
    return out
