"""GPU checks through the C ABI: the matrix-core GEMM of the small sign, the
adjoint with left vectors in any order, link replacement, the Hermitian and
antiperiodic cases, and every error status forced from the host.

References: numpy's complex128 matmul for the GEMM; the dense oracle
(spectral definition, Eq. 4-6) for the solves.
"""
import sys

import numpy as np
import pytest

import lattice_inputs as LI
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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


# ------------------------------------------------------ matrix-core GEMM
@pytest.mark.parametrize("n,nb", [(1, 1), (5, 2), (16, 1), (32, 1), (33, 3), (100, 2),
                                  (257, 1), (700, 2)])
def test_small_gemm_matches_numpy(osa, n, nb):
    """C = A B on the FP64 matrix cores against numpy (one and several problems,
    sizes below, at and across the 32-wide tile, ragged tails)."""
    say(f"small gemm n={n} nb={nb}")
    rng = np.random.default_rng(1000 * n + nb)
    A = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    B = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    C = host(osa.small_gemm(dev(A), dev(B)))
    ref = A @ B
    for b in range(nb):
        # FP64 products of length n: error of a few ulp times sqrt(n) per entry
        assert rel(C[b], ref[b]) < 1e-14 * max(1.0, np.sqrt(n))
    # a single problem through the 2-D form
    C1 = host(osa.small_gemm(dev(A[0]), dev(B[0])))
    assert np.array_equal(C1, C[0])


def test_small_gemm_rejects_overlap(osa):
    A = torch.zeros((4, 4), dtype=torch.complex128, device="cuda:0")
    L = osa.lib()
    import ctypes
    st = L.osa_small_gemm(4, 1, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                          ctypes.c_void_p(A.data_ptr()), None)
    assert st == -1


# --------------------------------------------- adjoint, left vectors in any order
@pytest.fixture(scope="module")
def haar4():
    w = LI.WORKLOADS[0]
    dims = w["dims"]
    links = LI.make_links(dims, "haar", cfg=0, inst=0)
    b = LI.gaussian_source(dims, cfg=0, inst=0)
    h = O.hermitian_wilson_dense(links, dims, w["mu"], w["m_w"])
    return dims, links, b, h


def test_adjoint_with_permuted_and_scaled_left_vectors(osa, haar4):
    """Only the projector R (L^dag R)^{-1} L^dag is canonical: the columns of L
    may come in any order and with any scale.  sign(H) b and sign(H)^dag a must
    not change (the deflated part of the adjoint is L G^{-H} sgn(Lambda) R^dag a)."""
    dims, links, b, h = haar4
    r, l, lam = O.critical_dense(h, 10)
    rng = np.random.default_rng(5)
    perm = rng.permutation(10)
    ph = np.exp(2j * np.pi * rng.random(10)) * (0.1 + 3 * rng.random(10))
    lp = l[:, perm] * ph
    a = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    a /= np.linalg.norm(a)
    say("adjoint with permuted, rescaled left vectors")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=500, check_every=25)
    ctx.set_deflation(dev(r.T.copy()), dev(lp.T.copy()), lam)
    ya, _, st = ctx.apply_adjoint(dev(a), tol=1e-11)
    assert st == osa.OSA_OK
    assert rel(host(ya), O.sign_adjoint_apply(h, a)) < 1e-9
    y, _, st = ctx.apply(dev(b), tol=1e-11)
    assert st == osa.OSA_OK
    assert rel(host(y), O.sign_eig_apply(h, b)) < 1e-9
    ctx.close()


def test_deflate_pairs_left_with_right(osa, haar4):
    """osa_deflate returns L in R's order: G = L^dag R is nearly diagonal."""
    dims, links, b, h = haar4
    say("deflate: left vectors paired with the right ones")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5)
    ctx.deflate(12)
    R, L, lam = ctx.get_deflation()
    R, L = host(R).T, host(L).T
    g = L.conj().T @ R
    off = g - np.diag(np.diag(g))
    assert np.abs(off).max() < 1e-8 * np.abs(np.diag(g)).min()
    # and the left vectors are left eigenvectors for the conjugate pairing
    assert max(O.eig_residuals(h, R, L, lam)) < 1e-10
    ctx.close()


# ------------------------------------------------------------- link replacement
def test_set_links_matches_fresh_context(osa):
    """osa_set_links replaces the operator: deflating and solving afterwards
    gives bitwise what a new context on the new links gives."""
    dims = (3, 4, 3, 4)
    l1 = LI.make_links(dims, "haar", cfg=9, inst=30)
    l2 = LI.make_links(dims, "disordered", eps=0.7, cfg=9, inst=31)
    b = dev(LI.gaussian_source(dims, cfg=9, inst=30))
    say("set_links against a fresh context")
    ctx = osa.Context(dev(l1), dims, 0.4, -1.4, k_max=900, check_every=20)
    ctx.deflate(8)
    y1, _, _ = ctx.apply(b, tol=1e-10)
    ctx.set_links(dev(l2))
    ctx.deflate(8)
    y2, _, st2 = ctx.apply(b, tol=1e-10)
    fresh = osa.Context(dev(l2), dims, 0.4, -1.4, k_max=900, check_every=20)
    fresh.deflate(8)
    y2f, _, st2f = fresh.apply(b, tol=1e-10)
    assert st2 == st2f == osa.OSA_OK
    assert torch.equal(y2, y2f)
    h2 = O.hermitian_wilson_dense(l2, dims, 0.4, -1.4)
    assert rel(host(y2), O.sign_eig_apply(h2, host(b))) < 1e-9
    assert not torch.equal(y1, y2)
    ctx.close()
    fresh.close()


# ------------------------------------------------ Hermitian and antiperiodic cases
def test_hermitian_mu0_solve(osa):
    """mu = 0: H is Hermitian, sign(H) = W sgn(Lambda) W^dag (eigh) is Hermitian and
    unitary, so |sign(H) b| = |b|; the deflation reduces to Eq. 12 (L spans R)."""
    dims = (4, 4, 4, 4)
    links = LI.make_links(dims, "haar", cfg=9, inst=32)
    b = LI.gaussian_source(dims, cfg=9, inst=32)
    h = O.hermitian_wilson_dense(links, dims, 0.0, -1.5)
    assert np.abs(h - h.conj().T).max() < 1e-14
    w, v = np.linalg.eigh(h)
    yref = v @ (np.sign(w) * (v.conj().T @ b))
    say("mu = 0 solve")
    ctx = osa.Context(dev(links), dims, 0.0, -1.5, k_max=900, check_every=25)
    ctx.deflate(10)
    R, L, lam = ctx.get_deflation()
    assert np.abs(np.asarray(lam).imag).max() < 1e-10
    y, _, st = ctx.apply(dev(b), tol=1e-11)
    y = host(y)
    assert st == osa.OSA_OK
    assert rel(y, yref) < 1e-9
    assert abs(np.linalg.norm(y) - 1.0) < 1e-9
    ctx.close()


def test_antiperiodic_solve_matches_dense(osa):
    dims = (4, 4, 2, 6)
    links = LI.make_links(dims, "disordered", eps=0.8, cfg=9, inst=33)
    b = LI.gaussian_source(dims, cfg=9, inst=33)
    h = O.hermitian_wilson_dense(links, dims, 0.25, -1.6, antiperiodic_t=True)
    say("antiperiodic solve")
    ctx = osa.Context(dev(links), dims, 0.25, -1.6, antiperiodic_t=True, k_max=1200,
                      check_every=25)
    ctx.deflate(8)
    y, _, st = ctx.apply(dev(b), tol=1e-11)
    assert st == osa.OSA_OK
    assert rel(host(y), O.sign_eig_apply(h, b)) < 1e-9
    ctx.close()


# ------------------------------------------------------ statuses forced from the host
def test_imag_axis_leaves_no_deflation_active(osa, haar4):
    """Importing an eigenvalue on the imaginary axis returns OSA_ERR_IMAG_AXIS and
    leaves the context without deflation: the next solve is the undeflated one."""
    dims, links, b, h = haar4
    r, l, lam = O.critical_dense(h, 6)
    bad = lam.copy()
    bad[2] = 1j * bad[2].imag
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=600, check_every=25)
    with pytest.raises(osa.OsaError) as e:
        ctx.set_deflation(dev(r.T.copy()), dev(l.T.copy()), bad)
    assert e.value.status == -5
    y, infos, st = ctx.apply(dev(b), tol=1e-10)
    assert st == osa.OSA_OK and infos[0]["n_defl"] == 0
    assert rel(host(y), O.sign_eig_apply(h, b)) < 1e-8
    ctx.close()


def test_eig_noconv_with_one_restart(osa, haar4):
    dims, links, b, h = haar4
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, eig_max_restarts=1)
    with pytest.raises(osa.OsaError) as e:
        ctx.deflate(10)
    assert e.value.status == -6
    # the context stays usable without deflation
    y, infos, st = ctx.apply(dev(b), tol=1e-6)
    assert st == osa.OSA_OK and infos[0]["n_defl"] == 0
    ctx.close()


def test_newton_noconv_on_imaginary_eigenvalue(osa):
    """sgn is undefined on the imaginary axis: the small sign of a matrix with an
    eigenvalue there does not converge (OSA_ERR_NEWTON_NOCONV)."""
    a = np.diag([1.0, 0.7j, -2.0]).astype(np.complex128)
    a[0, 1] = 0.3
    with pytest.raises(osa.OsaError) as e:
        osa.small_sign(dev(a))
    assert e.value.status == -7


def test_oom_from_allocator_hook(osa):
    """An allocator hook that returns NULL makes the call fail with OSA_ERR_OOM."""
    dims = (2, 2, 2, 2)
    links = dev(LI.make_links(dims, "haar", cfg=9, inst=34))
    L = osa.lib()
    pair = (osa.ALLOC_FN(lambda n, s, u: None), osa.DEALLOC_FN(lambda p, s, u: None))
    osa._hooks.append(pair)
    assert L.osa_set_allocator(pair[0], pair[1], None) == 0
    try:
        with pytest.raises(osa.OsaError) as e:
            osa.Context(links, dims, 0.3, -1.5)
        assert e.value.status == -3
    finally:
        osa.use_torch_allocator(False)
    c = osa.Context(links, dims, 0.3, -1.5)   # hipMalloc again
    c.close()


# --------------------------------------------- graph replay and the autotuner
def test_graph_replay_bitwise_and_autotune_table(osa, haar4):
    """Arnoldi segments recorded as HIP graphs and replayed give bitwise the
    results of direct launches (one source and a lockstep batch, repeated solves
    with new sources); the dot-kernel autotuner has recorded its choices."""
    dims, links, b, h = haar4
    rng = np.random.default_rng(9)
    srcs = rng.standard_normal((4, b.size)) + 1j * rng.standard_normal((4, b.size))
    srcs /= np.linalg.norm(srcs, axis=1, keepdims=True)
    say("graph replay vs direct launches")
    outs = {}
    for ng in (True, False):
        ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=400, check_every=25, max_batch=3,
                          no_graphs=ng)
        ctx.deflate(10)
        ys = []
        for rep in range(3):                       # the third solve replays recorded graphs
            y1, _, st1 = ctx.apply(dev(srcs[rep]), tol=1e-10)
            y3, _, st3 = ctx.apply(dev(srcs[1:4]), tol=1e-10)
            assert st1 == st3 == osa.OSA_OK
            ys.append((host(y1), host(y3)))
        cap, lau = ctx.graph_stats()
        if ng:
            assert cap == 0 and lau == 0
        else:
            assert cap > 0 and lau > cap
        outs[ng] = ys
        ctx.close()
    for (a1, a3), (b1, b3) in zip(outs[True], outs[False]):
        assert np.array_equal(a1, b1) and np.array_equal(a3, b3)
    assert rel(outs[False][2][0], O.sign_eig_apply(h, srcs[2])) < 1e-9
    table = osa.autotune_table()
    assert table and all(1 <= w <= 64 for _, _, w in table)
