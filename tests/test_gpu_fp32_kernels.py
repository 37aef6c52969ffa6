"""GPU parity of the FP32 kernel instantiations (the FP32 eigensearch's
stencil, Gram-Schmidt and normalisation kernels), through the C ABI, against
the oracle in FP64 on the same FP32-rounded inputs.

Bounds.  The FP32 stencil sums about 30 rounded terms per output entry (eight
spin-projected hops of a 3x3 complex product each, plus the diagonal), so its
entries differ from the exact operator by at most about 30 u sum|terms| with
u = 2^-24 = 6e-8: 2e-6 of the entry scale.  The tests take 1e-5 of the largest
entry.  An Arnoldi run in FP32 arithmetic keeps orthonormality and the Arnoldi
relation to a few u, and the FP64 oracle's Hessenberg entries for these
operators and k <= 16 are reproduced to ~4e-8 of their largest entry by an
FP32 simulation of the oracle; the tests take 1e-5.  FP64 runs are held to
1e-12.
"""
import sys

import numpy as np
import pytest

import lattice_inputs as LI
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def osa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_0710_0341_amd as osa_mod
    osa_mod.lib()
    return osa_mod


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


STENCIL32_CASES = [
    ((4, 4, 4, 4), "haar", 0.3, False, True),
    ((3, 4, 5, 6), "disordered", 0.5, True, True),    # ragged, antiperiodic
    ((4, 4, 4, 4), "haar", -0.2, False, False),       # FP64-stored links, rounded once
]


@pytest.mark.parametrize("dims,kind,mu,ap,links_fp32", STENCIL32_CASES)
def test_fp32_stencil_matches_oracle(osa, dims, kind, mu, ap, links_fp32):
    say(f"fp32 stencil dims={dims} kind={kind} mu={mu} ap={ap} links_fp32={links_fp32}")
    links = LI.make_links(dims, kind, eps=0.6, cfg=9, inst=4)
    l32 = LI.round_links_fp32(links)
    tl = dev(l32.astype(np.complex64) if links_fp32 else links)
    b = np.stack([LI.gaussian_source(dims, cfg=9, inst=10 + i) for i in range(3)])
    b32 = b.astype(np.complex64)
    ctx = osa.Context(tl, dims, mu, -1.5, antiperiodic_t=ap)
    y = host(ctx.apply_hw32(dev(b32)))
    assert y.dtype == np.complex64
    h = O.hermitian_wilson_sparse(l32, dims, mu, -1.5, ap)
    for i in range(3):
        ref = h @ b32[i].astype(np.complex128)
        err = np.abs(y[i].astype(np.complex128) - ref)
        assert err.max() <= 1e-5 * np.abs(ref).max()
    ctx.close()


KRYLOV_CASES = [   # prec: 1 = FP32, 0 = FP64
    (1, False, 16, (4, 4, 4, 4), 0.3),
    (1, True, 12, (3, 4, 5, 6), 0.5),
    (0, False, 16, (4, 4, 4, 4), 0.3),
    (0, True, 16, (3, 4, 5, 6), 0.5),
]


@pytest.mark.parametrize("prec,adjoint,k,dims,mu", KRYLOV_CASES)
def test_krylov_h2_matches_oracle(osa, prec, adjoint, k, dims, mu):
    """The eigensearch's Arnoldi expansion on H(+-mu)^2 against the oracle's
    CGS2 Arnoldi (Eq. 7) on the same FP32-stored links, and the defining
    properties of the decomposition (v_1 = x/|x|, orthonormal V, upper
    Hessenberg S with real positive subdiagonal, A V_k = V_{k+1} S with the
    oracle's operator)."""
    say(f"krylov_h2 prec={prec} adjoint={adjoint} k={k} dims={dims} mu={mu}")
    tol = 1e-5 if prec == osa.FP32 else 1e-12
    l32 = LI.round_links_fp32(LI.make_links(dims, "haar", cfg=9, inst=5))
    x = LI.gaussian_source(dims, cfg=9, inst=20)
    ctx = osa.Context(dev(l32.astype(np.complex64)), dims, mu, -1.5)
    vt, st = ctx.krylov_h2(dev(x), k, prec=prec, adjoint=adjoint)
    V = host(vt).T                      # (N, k+1)
    S = host(st)                        # (k+1, k)
    h = O.hermitian_wilson_sparse(l32, dims, -mu if adjoint else mu, -1.5)

    def a_op(v):
        return h @ (h @ v)

    smax = np.abs(S).max()
    assert np.linalg.norm(V[:, 0] - x / np.linalg.norm(x)) <= tol
    assert np.abs(V.conj().T @ V - np.eye(k + 1)).max() <= tol
    assert np.all(np.tril(S, -2) == 0)
    sub = np.diag(S, -1)
    assert np.all(sub.imag == 0) and np.all(sub.real > 0)
    av = np.stack([a_op(V[:, j]) for j in range(k)], axis=1)
    assert np.linalg.norm(av - V @ S) <= tol * np.linalg.norm(S)
    Vo, Ho, beta, kd = O.arnoldi_cgs2(a_op, x, k)
    assert kd == k
    assert np.abs(S - Ho).max() <= tol * smax
    assert np.abs(V - Vo).max() <= tol
    ctx.close()


def test_krylov_h2_rejects_bad_arguments(osa):
    dims = (2, 2, 2, 2)
    links = LI.make_links(dims, "haar", cfg=9, inst=6)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5)
    x = dev(LI.gaussian_source(dims, cfg=9, inst=21))
    for k in (0, 65):
        with pytest.raises(osa.OsaError):
            ctx.krylov_h2(x, k)
    with pytest.raises(osa.OsaError):
        ctx.krylov_h2(x, 4, prec=7)
    ctx.close()
