"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP64 mode): operator application to rounding (1e-13 relative);
the full method at fixed (k, deflation data) to 1e-10 relative, the bar set
for FP64 results; the converged result against the exact sign(H) b within the
requested tolerance (times a small safety factor, since the stopping test is
an estimate).
"""
import sys

import numpy as np
import scipy.linalg
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


# ------------------------------------------------------------------ stencil
STENCIL_CASES = [
    ((2, 2, 2, 2), "haar", 0.3, False, False),
    ((4, 4, 4, 4), "haar", 0.3, False, False),
    ((3, 4, 5, 6), "haar", 0.5, True, False),      # ragged: no padding-free tile
    ((2, 3, 2, 5), "disordered", -0.2, False, False),
    ((4, 4, 4, 4), "haar", 0.3, False, True),       # FP32-stored links
    ((6, 2, 3, 4), "haar", 0.1, True, True),
]


@pytest.mark.parametrize("dims,kind,mu,ap,fp32", STENCIL_CASES)
def test_stencil_matches_oracle(osa, dims, kind, mu, ap, fp32):
    say(f"stencil dims={dims} kind={kind} mu={mu} ap={ap} fp32={fp32}")
    links = LI.make_links(dims, kind, eps=0.6, cfg=9, inst=1)
    if fp32:
        links = LI.round_links_fp32(links)
    tl = dev(links.astype(np.complex64) if fp32 else links)
    b = np.stack([LI.gaussian_source(dims, cfg=9, inst=i) for i in range(3)])
    ctx = osa.Context(tl, dims, mu, -1.5, antiperiodic_t=ap)
    y = host(ctx.apply_hw(dev(b)))
    h = O.hermitian_wilson_sparse(links, dims, mu, -1.5, ap)
    for i in range(3):
        assert rel(y[i], h @ b[i]) < 1e-14
    ctx.close()


def test_stencil_free_field_8(osa):
    """At 8^4 (the headline lattice) against the momentum-space closed form."""
    dims = (8, 8, 8, 8)
    say("stencil free field 8^4")
    u = LI.make_links(dims, "unit")
    b = LI.gaussian_source(dims, cfg=9, inst=5)
    ctx = osa.Context(dev(u), dims, 0.5, -1.5)
    y = host(ctx.apply_hw(dev(b)))
    assert rel(y, O.free_field_h_apply(dims, 0.5, -1.5, b)) < 1e-13
    ctx.close()


# ---------------------------------------------------------------- small sign
@pytest.mark.parametrize("k", [1, 7, 64, 130, 257])
def test_small_sign_matches_oracle(osa, k):
    say(f"small sign k={k}")
    dims = (3, 3, 3, 3)
    links = LI.make_links(dims, "haar", cfg=9, inst=2)
    h = O.hermitian_wilson_sparse(links, dims, 0.3, -1.5)
    b = LI.gaussian_source(dims, cfg=9, inst=2)
    _, hm, _, _ = O.arnoldi_cgs2(lambda x: h @ x, b, k)
    hk = hm[:k, :k]
    s, its = osa.small_sign(dev(hk))
    ref = O.small_sign_e1(hk, "newton")
    assert rel(host(s), ref) < 1e-12
    assert rel(ref, O.small_sign_e1(hk, "eig")) < 1e-9


@pytest.mark.parametrize("k", [700, 2100])
def test_small_sign_large(osa, k):
    """Krylov sizes beyond the solve's default cap (k = 700) and far beyond it
    (k = 2100, 4 x 2100 Gauss-Jordan column blocks per pivot launch)."""
    say(f"small sign k={k}")
    dims = (4, 4, 4, 4)
    links = LI.make_links(dims, "haar", cfg=9, inst=2)
    h = O.hermitian_wilson_sparse(links, dims, 0.3, -1.5)
    b = LI.gaussian_source(dims, cfg=9, inst=2)
    _, hm, _, _ = O.arnoldi_cgs2(lambda x: h @ x, b, k)
    hk = hm[:k, :k]
    s, its = osa.small_sign(dev(hk))
    assert rel(host(s), O.small_sign_e1(hk, "newton")) < 1e-11


def test_small_sign_dense_nonhessenberg(osa):
    """A dense matrix with a known spectrum off the imaginary axis."""
    rng = np.random.default_rng(3)
    n = 50
    lam = np.concatenate([rng.uniform(0.1, 2, 25), -rng.uniform(0.1, 2, 25)]) + 0.3j * rng.standard_normal(50)
    q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = q @ np.diag(lam) @ np.linalg.inv(q)
    s, _ = osa.small_sign(dev(a))
    ref = (q @ np.diag(np.sign(lam.real)) @ np.linalg.inv(q))[:, 0]
    assert rel(host(s), ref) < 1e-9


# ---------------------------------------------------------- small Schur
def _ks_like(p, rng, keep):
    """Triangular leading block + spike row + Hessenberg tail, as after a restart."""
    a = np.triu(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)), -1)
    a[:keep, :keep] = np.triu(a[:keep, :keep])
    a[keep, :keep] = rng.standard_normal(keep) + 1j * rng.standard_normal(keep)
    return a


def _split_hessenberg(p, rng):
    """Upper Hessenberg with zero subdiagonal entries: QR sweeps on active blocks
    that start and end inside the matrix."""
    a = np.triu(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)), -1)
    for i in range(3, p, 7):
        a[i, i - 1] = 0
    return a


@pytest.mark.parametrize("p,kind,mode", [(2, "dense", 0), (3, "dense", 1), (4, "dense", 0),
                                         (5, "dense", 0), (17, "ks", 1), (33, "dense", 1),
                                         (48, "split", 0), (64, "ks", 0), (64, "split", 1),
                                         (65, "dense", 0), (80, "ks", 1), (96, "ks", 0),
                                         (96, "dense", 1)])
def test_small_schur_properties(osa, p, kind, mode):
    say(f"small schur p={p} kind={kind} mode={mode}")
    rng = np.random.default_rng(p + 7 * mode)
    if kind == "dense":
        a = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    elif kind == "split":
        a = _split_hessenberg(p, rng)
    else:
        a = _ks_like(p, rng, p // 2)
    T, Z, w = osa.small_schur(dev(a), mode)
    T, Z, w = host(T), host(Z), host(w)
    nrm = np.linalg.norm(a)
    assert np.linalg.norm(Z @ T @ Z.conj().T - a) < 1e-12 * nrm
    assert np.abs(Z.conj().T @ Z - np.eye(p)).max() < 1e-12
    assert np.abs(np.tril(T, -1)).max() < 1e-13 * nrm
    key = np.abs(w) if mode == 0 else np.abs(w.real)
    assert np.all(np.diff(key) >= -1e-12 * nrm)
    # a backward stable Schur form fixes each eigenvalue only to its condition
    # number (1/|y^H x| for unit left/right eigenvectors) times the backward error
    ev, vl, vr = scipy.linalg.eig(a, left=True, right=True)
    cond = np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0) / np.abs(np.sum(vl.conj() * vr, axis=0))
    tol = np.maximum(1e-9, 1e-12 * cond) * nrm
    for x in w:
        assert np.any(np.abs(ev - x) < tol)


# ------------------------------------------------- full method, fixed k
def _fixed_k_case(osa, dims, kind, mu, m, k, inst, reproject=True, eps=0.6, orth=0):
    links = LI.make_links(dims, kind, eps=eps, cfg=9, inst=inst)
    b = LI.gaussian_source(dims, cfg=9, inst=inst)
    h = O.hermitian_wilson_sparse(links, dims, mu, -1.5)
    ctx = osa.Context(dev(links), dims, mu, -1.5, k_max=k, check_every=-1,
                      no_reproject=not reproject, orth=orth)
    defl = None
    if m:
        r, l, lam = O.critical_dense(h.toarray(), m)
        defl = O.Deflation(r, l, lam)
        ctx.set_deflation(dev(r.T.copy()), dev(l.T.copy()), lam)
    y, infos, st = ctx.apply(dev(b), tol=1e-30)
    yo, info = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=k, reproject=reproject)
    ctx.close()
    return host(y), yo, infos[0], info


@pytest.mark.parametrize("dims,kind,mu,m,k", [
    ((2, 2, 2, 2), "haar", 0.3, 0, 40),
    ((3, 4, 3, 4), "disordered", 0.5, 0, 90),
    ((3, 4, 3, 4), "disordered", 0.5, 8, 90),
    ((4, 4, 4, 4), "haar", 0.3, 10, 150),
])
def test_fixed_k_matches_oracle(osa, dims, kind, mu, m, k):
    say(f"fixed k dims={dims} m={m} k={k}")
    y, yo, info, oinfo = _fixed_k_case(osa, dims, kind, mu, m, k, inst=3)
    assert info["k_used"] == oinfo["k_used"] == k
    assert rel(y, yo) < 1e-10


@pytest.mark.parametrize("reproject", [True, False])
def test_fixed_k_delayed_and_plain_cgs2_agree(osa, reproject):
    """The solve's two orthogonalisations (second Gram-Schmidt pass delayed by
    one step, default; both passes in the same step) give the same Krylov
    approximation up to rounding, and both match the oracle's CGS2."""
    say(f"fixed k, delayed vs plain CGS2, re-projection {reproject}")
    y0, yo, i0, _ = _fixed_k_case(osa, (4, 4, 4, 4), "haar", 0.3, 10, 150, inst=5,
                                  reproject=reproject, orth=0)
    y1, _, i1, _ = _fixed_k_case(osa, (4, 4, 4, 4), "haar", 0.3, 10, 150, inst=5,
                                 reproject=reproject, orth=1)
    assert i0["k_used"] == i1["k_used"] == 150
    assert rel(y0, yo) < 1e-10 and rel(y1, yo) < 1e-10
    assert rel(y0, y1) < 1e-12


def test_fixed_k_without_reprojection(osa):
    say("fixed k, re-projection off")
    y, yo, info, _ = _fixed_k_case(osa, (3, 4, 3, 4), "disordered", 0.5, 8, 60, inst=4,
                                   reproject=False)
    assert rel(y, yo) < 1e-10


# --------------------------------------------------- converged vs exact
@pytest.fixture(scope="module")
def haar4_dense():
    """The small workload: 4^4 Haar links, m_w = -1.5, mu = 0.3, Gaussian source."""
    w = LI.WORKLOADS[0]
    dims = w["dims"]
    links = LI.make_links(dims, "haar", cfg=0, inst=0)
    b = LI.gaussian_source(dims, cfg=0, inst=0)
    h = O.hermitian_wilson_dense(links, dims, w["mu"], w["m_w"])
    say("dense oracle 4^4 (route E) ...")
    y = O.sign_eig_apply(h, b)
    return dims, links, b, h, y


def test_converged_matches_dense_haar4(osa, haar4_dense):
    dims, links, b, h, yref = haar4_dense
    say("haar4 full method: GPU deflation + adaptive Krylov")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=500, check_every=25)
    dinfo = ctx.deflate(10)
    assert dinfo["max_eig_resid"] < 1e-10
    y, infos, st = ctx.apply(dev(b), tol=1e-11)
    err = rel(host(y), yref)
    say(f"  k_used={infos[0]['k_used']} est={infos[0]['resid_est']:.2e} err={err:.2e}")
    assert st == osa.OSA_OK
    assert err < 1e-10
    # the configured tolerance 1e-8 with k_max = 300 (the small workload as specified)
    ctx.set_opts(k_max=300, check_every=25)
    y8, infos8, st8 = ctx.apply(dev(b), tol=1e-8)
    assert rel(host(y8), yref) < 1e-7
    ctx.close()


@pytest.mark.parametrize("ncv,filt,prec", [(96, 0, 0), (32, 0, 0), (0, 128, 0), (32, 40, 0),
                                           (0, 0, 1)])
def test_deflation_matches_oracle_eigenpairs(osa, haar4_dense, ncv, filt, prec):
    """Krylov-Schur (filt 0) with both Schur kernels: the LDS one (active block
    <= 64) and the logged one (<= 96); the Chebyshev-filtered subspace iteration
    (degree filt) with its default block and with a 32-vector block; an FP32
    Krylov-Schur search (prec 1) whose subspace is refined in FP64."""
    dims, links, b, h, _ = haar4_dense
    say(f"haar4 eigenpairs vs dense oracle, block {ncv}, filter {filt}, prec {prec}")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, eig_ncv=ncv, eig_filter=filt, eig_prec=prec)
    ctx.deflate(10)
    R, L, lam = ctx.get_deflation()
    R, L = host(R).T, host(L).T
    r0, l0, lam0 = O.critical_dense(h, 10)
    assert np.abs(np.sort_complex(lam) - np.sort_complex(lam0)).max() < 1e-10
    # the oblique projector R G^{-1} L^dag is canonical
    p_gpu = O.Deflation(R, L, lam)
    p_ref = O.Deflation(r0, l0, lam0)
    assert rel(p_gpu.r @ p_gpu.coeffs(b), p_ref.r @ p_ref.coeffs(b)) < 1e-9
    assert max(O.eig_residuals(h, R, L, lam)) < 1e-10
    ctx.close()


def test_one_shot_entry_point(osa):
    dims = (2, 2, 3, 4)
    links = LI.make_links(dims, "haar", cfg=9, inst=6)
    b = LI.gaussian_source(dims, cfg=9, inst=6)
    say("one-shot overlap_sign_apply")
    y, est, st = osa.overlap_sign_apply(dev(links), dims, 0.3, -1.5, dev(b), 1e-10, 6)
    h = O.hermitian_wilson_dense(links, dims, 0.3, -1.5)
    assert rel(host(y), O.sign_eig_apply(h, b)) < 1e-9


# --------------------------------------------------------------- edge cases
def test_breakdown_plane_wave_is_exact(osa):
    dims = (2, 2, 2, 4)
    say("breakdown: free plane wave")
    u = LI.make_links(dims, "unit")
    t = np.arange(dims[3])
    wave = np.exp(2j * np.pi * t / dims[3])[:, None, None, None, None, None] * np.ones((1, 2, 2, 2, 4, 3))
    chi = np.zeros((4, 3), dtype=complex)
    chi[0, 0] = 1.0
    b = (wave * chi).reshape(-1)
    b /= np.linalg.norm(b)
    ctx = osa.Context(dev(u), dims, 0.3, -1.5, k_max=50, check_every=5)
    y, infos, st = ctx.apply(dev(b), tol=1e-12)
    assert infos[0]["breakdown"] == 1 and infos[0]["k_used"] <= 4
    assert rel(host(y), O.free_field_sign_apply(dims, 0.3, -1.5, b)) < 1e-12
    ctx.close()


def test_not_converged_status_and_nonfinite(osa):
    dims = (3, 3, 3, 3)
    links = LI.make_links(dims, "haar", cfg=9, inst=7)
    b = LI.gaussian_source(dims, cfg=9, inst=7)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=20, check_every=10)
    say("not converged at k_max = 20")
    y, infos, st = ctx.apply(dev(b), tol=1e-14)
    assert st == osa.OSA_NOT_CONVERGED and infos[0]["k_used"] == 20
    say("NaN source")
    bad = b.copy()
    bad[5] = np.nan
    with pytest.raises(osa.OsaError) as e:
        ctx.apply(dev(bad), tol=1e-8)
    assert e.value.status == -4
    ctx.close()


def test_source_inside_deflation_space(osa):
    """b in span(R): x_ominus = 0 and the result is the exact first term of Eq. 21."""
    dims = (2, 2, 3, 3)
    links = LI.make_links(dims, "haar", cfg=9, inst=8)
    h = O.hermitian_wilson_dense(links, dims, 0.3, -1.5)
    r, l, lam = O.critical_dense(h, 6)
    b = r @ (np.arange(6) + 1.0)
    b /= np.linalg.norm(b)
    say("source in span(R)")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=30, check_every=10)
    ctx.set_deflation(dev(r.T.copy()), dev(l.T.copy()), lam)
    y, infos, st = ctx.apply(dev(b), tol=1e-10)
    assert infos[0]["k_used"] == 0
    assert rel(host(y), O.sign_eig_apply(h, b)) < 1e-11
    ctx.close()


def test_multi_rhs_and_determinism(osa):
    dims = (3, 3, 3, 4)
    links = LI.make_links(dims, "disordered", eps=0.6, cfg=9, inst=9)
    B = np.stack([LI.gaussian_source(dims, cfg=9, inst=10 + i) for i in range(3)])
    say("multi-rhs + determinism")
    ctx = osa.Context(dev(links), dims, 0.2, -1.5, k_max=400, check_every=20)
    ctx.deflate(8)
    Y1, inf1, st1 = ctx.apply(dev(B), tol=1e-10)
    assert st1 == osa.OSA_OK
    Y2, inf2, _ = ctx.apply(dev(B), tol=1e-10)
    Y1, Y2 = host(Y1), host(Y2)
    assert np.array_equal(Y1, Y2)
    for i in range(3):
        yi, _, _ = ctx.apply(dev(B[i]), tol=1e-10)
        assert np.array_equal(host(yi), Y1[i])
    h = O.hermitian_wilson_dense(links, dims, 0.2, -1.5)
    for i in range(3):
        assert rel(Y1[i], O.sign_eig_apply(h, B[i])) < 1e-9
    ctx.close()


# ------------------------------------------------------------ batched solve
@pytest.fixture(scope="module")
def haar4_sign(haar4_dense):
    _, _, _, h, _ = haar4_dense
    say("dense sign matrix 4^4 ...")
    return O.sign_eig(h)


def test_batched_point_sources_match_single_and_dense(osa, haar4_dense, haar4_sign):
    """12 spin-colour point sources at one site in one lockstep batch: every
    result matches the dense sign and is bitwise the single-source result."""
    dims, links, _, _, _ = haar4_dense
    V = int(np.prod(dims))
    site = 37
    B = np.zeros((12, 12 * V), dtype=complex)
    for sc in range(12):
        B[sc, site * 12 + sc] = 1.0
    say("batch of 12 point sources, haar 4^4, m = 10")
    # the oracle's error at k = 400 is 1.7e-11, so the estimate crosses 1e-10 just after
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=500, check_every=25, max_batch=12)
    ctx.deflate(10)
    Yb, infb, st = ctx.apply(dev(B), tol=1e-10)
    assert st == osa.OSA_OK and all(i["batch"] == 12 for i in infb)
    Yb = host(Yb)
    ref = (haar4_sign @ B.T).T
    for sc in range(12):
        assert rel(Yb[sc], ref[sc]) < 1e-9, sc
    ctx.set_opts(k_max=500, check_every=25, max_batch=1)
    for sc in (0, 5, 11):
        y1, inf1, _ = ctx.apply(dev(B[sc]), tol=1e-10)
        assert inf1[0]["batch"] == 1 and inf1[0]["k_used"] == infb[sc]["k_used"]
        assert np.array_equal(host(y1), Yb[sc])
    ctx.close()


def test_batch_mixed_sources_and_split(osa, haar4_dense, haar4_sign):
    """One batch with sources that stop at different Krylov sizes (one inside
    span(R), k = 0; one almost inside it; Gaussian and point sources) and one
    NaN source, whose error stays its own.  Splitting the batch (max_batch 2)
    gives bitwise the same results."""
    dims, links, b, h, _ = haar4_dense
    N = 12 * int(np.prod(dims))
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=400, check_every=20, max_batch=8)
    ctx.deflate(10)
    R, _, _ = ctx.get_deflation()
    r = host(R)
    in_span = (np.arange(10) + 1.0) @ r
    in_span /= np.linalg.norm(in_span)
    near = in_span + 1e-7 * LI.gaussian_source(dims, cfg=9, inst=22)
    point = np.zeros(N, dtype=complex)
    point[12 * 200 + 7] = 1.0
    nan = LI.gaussian_source(dims, cfg=9, inst=23)
    nan[3] = np.nan
    B = np.stack([b, in_span, nan, near, point, LI.gaussian_source(dims, cfg=9, inst=21)])
    say("mixed batch of 6 (k = 0, near span(R), NaN, point, 2 Gaussian)")
    Y, inf, st = ctx.apply(dev(B), tol=1e-10, check=False)
    assert st == -4
    stat = [i["status"] for i in inf]
    assert stat == [0, 0, -4, 0, 0, 0], stat
    assert inf[1]["k_used"] == 0
    ks = [inf[i]["k_used"] for i in (0, 3, 4, 5)]
    assert len(set(ks)) > 1, ks
    Y = host(Y)
    for i in (0, 1, 3, 4, 5):
        assert rel(Y[i], haar4_sign @ B[i]) < 1e-9, i
    ctx.set_opts(k_max=400, check_every=20, max_batch=2)
    Y2, inf2, st2 = ctx.apply(dev(B), tol=1e-10, check=False)
    assert st2 == -4 and [i["batch"] for i in inf2] == [2, 2, 2, 2, 2, 2]
    Y2 = host(Y2)
    for i in (0, 1, 3, 4, 5):
        assert np.array_equal(Y2[i], Y[i]), i
        assert inf2[i]["k_used"] == inf[i]["k_used"]
    ctx.close()


def test_stencil_many_rhs(osa):
    """70 right-hand sides: more than one launch group of the batched stencil."""
    dims = (2, 2, 3, 2)
    links = LI.make_links(dims, "haar", cfg=9, inst=24)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((70, 12 * 24)) + 1j * rng.standard_normal((70, 12 * 24))
    say("stencil with 70 rhs")
    ctx = osa.Context(dev(links), dims, 0.4, -1.5)
    Y = host(ctx.apply_hw(dev(X)))
    h = O.hermitian_wilson_sparse(links, dims, 0.4, -1.5)
    for i in (0, 33, 63, 64, 69):
        assert rel(Y[i], h @ X[i]) < 1e-14, i
    ctx.close()


# ------------------------------------------------------------- uneven batch
def test_uneven_batch_matches_single_and_dense(osa):
    """Instances of different lattices, mu, m_w and deflation sizes solved
    concurrently give bitwise the single-context results; two are checked
    against the dense oracle; a context listed twice is an argument error."""
    import torch
    cases = [((2, 2, 2, 4), 0.3, -1.5, 4, 0.6), ((3, 3, 3, 3), 0.1, -1.8, 6, 0.9),
             ((2, 3, 2, 4), 0.45, -1.2, 0, 0.3), ((3, 2, 3, 2), 0.2, -1.6, 3, 0.5),
             ((2, 2, 3, 3), 0.05, -1.9, 5, 1.0)]
    ctxs, srcs, dense = [], [], []
    for n, (dims, mu, mw, m, eps) in enumerate(cases):
        links = LI.make_links(dims, "disordered", eps=eps, cfg=9, inst=30 + n)
        b = LI.gaussian_source(dims, cfg=9, inst=30 + n)
        c = osa.Context(dev(links), dims, mu, mw, k_max=900, check_every=20,
                        stream=torch.cuda.Stream())
        if m:
            c.deflate(m)
        ctxs.append(c)
        srcs.append(dev(b))
        dense.append((links, dims, mu, mw, b))
    say("uneven batch of 5 instances")
    ys, infos, st = osa.batch_apply(ctxs, srcs, tol=1e-10)
    assert st == osa.OSA_OK, [i["status"] for i in infos]
    for c, b, y in zip(ctxs, srcs, ys):
        y1, _, _ = c.apply(b, tol=1e-10)
        assert torch.equal(y1, y)
    for n in (0, 1):
        links, dims, mu, mw, b = dense[n]
        h = O.hermitian_wilson_dense(links, dims, mu, mw)
        assert rel(host(ys[n]), O.sign_eig_apply(h, b)) < 1e-9
    with pytest.raises(osa.OsaError) as e:
        osa.batch_apply([ctxs[0], ctxs[1], ctxs[0]], srcs[:3], tol=1e-10)
    assert e.value.status == -1
    for c in ctxs:
        c.close()


# -------------------------------------------------- adjoint and overlap operator
def test_adjoint_and_overlap_match_oracle(osa, haar4_dense):
    """osa_apply_adjoint reuses the deflation data of H(mu) for sign(H)^dag =
    sign(H(-mu)) (left and right vectors swapped, lambda -> conj lambda);
    osa_apply_overlap returns b + gamma_5 sign(H) b (Eq. 1)."""
    dims, links, b, h, yref = haar4_dense
    say("adjoint and overlap, haar4, m = 10 and m = 0")
    rng = np.random.default_rng(21)
    a = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    a /= np.linalg.norm(a)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=500, check_every=25)
    ctx.deflate(10)
    ref_adj = O.sign_adjoint_apply(h, a)
    ya, ia, st = ctx.apply_adjoint(dev(a), tol=1e-11)
    assert st == osa.OSA_OK and rel(host(ya), ref_adj) < 1e-9
    yo, io, st = ctx.apply_overlap(dev(b), tol=1e-11)
    assert st == osa.OSA_OK and rel(host(yo), O.overlap_apply(h, b)) < 1e-9
    # the adjoint identity on the GPU results: <a, sign(H) b> = <sign(H)^dag a, b>
    ys, _, _ = ctx.apply(dev(b), tol=1e-11)
    lhs, rhs = np.vdot(a, host(ys)), np.vdot(host(ya), b)
    assert abs(lhs - rhs) < 1e-9 * abs(lhs)
    # a batch of adjoint solves is bitwise the single-source result
    A2 = np.stack([a, b])
    Y2, _, st = ctx.apply_adjoint(dev(A2), tol=1e-11)
    assert st == osa.OSA_OK and np.array_equal(host(Y2)[0], host(ya))
    # without deflation
    ctx.set_active_deflation(0)
    ya0, _, st = ctx.apply_adjoint(dev(a), tol=1e-10)
    assert st == osa.OSA_OK and rel(host(ya0), ref_adj) < 1e-8
    ctx.close()


# -------------------------------------------------- Fig. 1 convergence trends
def test_fig1_trends_haar4(osa, haar4_dense):
    """The results section's study at 4^4, mu = 0.3, x = (1, ..., 1): the error of
    fixed-k GPU solves against the dense sign falls with the Krylov size k and with
    the number m of deflated pairs (LR deflation)."""
    dims, links, _, h, _ = haar4_dense
    say("fig1 trends 4^4: dense sign of the ones source")
    x = LI.ones_source(dims)
    yx = O.sign_eig_apply(h, x)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=400, check_every=25)
    ctx.deflate(25)
    ks, ms = (50, 100, 200, 300), (0, 10, 25)
    eps = {}
    for m in ms:
        ctx.set_active_deflation(m)
        for k in ks:
            ctx.set_opts(k_max=k, check_every=-1)
            y, _, st = ctx.apply(dev(x), tol=1e-12)
            eps[m, k] = rel(host(y), yx)
    say("  " + "  ".join(f"m={m},k={k}:{e:.1e}" for (m, k), e in eps.items()))
    for m in ms:
        assert eps[m, 300] < eps[m, 100] < eps[m, 50]
    for k in (100, 200, 300):
        assert eps[25, k] < eps[10, k] < eps[0, k]
    assert eps[25, 300] < 1e-9 and eps[0, 300] > 10 * eps[25, 300]
    ctx.close()


# -------------------------------------------------- Schur deflation (Eq. 13-19)
@pytest.fixture(scope="module")
def haar3_schur():
    """3^4 Haar links, mu = 0.3, m_w = -1.5: the oracle's Schur data for m = 10 (a
    gap in |Re lambda| after the 10th eigenvalue) and the dense sign."""
    dims = (3, 3, 3, 3)
    links = LI.make_links(dims, "haar", cfg=0, inst=11)
    b = LI.gaussian_source(dims, cfg=0, inst=11)
    h = O.hermitian_wilson_dense(links, dims, 0.3, -1.5)
    say("dense oracle 3^4: sign and critical eigenpairs")
    r, l, lam = O.critical_dense(h, 10)
    s, t = O.schur_basis(r, lambda x: h @ x)
    return dims, links, b, h, r, s, t, O.sign_eig_apply(h, b)


def test_schur_deflation_matches_oracle(osa, haar3_schur):
    """Fixed-k Schur-deflated solves equal the oracle's Eq. 19 at the same (m, k);
    the converged solve equals the dense sign; the eigensolver ran one side only."""
    dims, links, b, h, r, s, t, yx = haar3_schur
    say("schur 3^4: deflate (right vectors only), fixed k, converged")
    mv = lambda x: h @ x  # noqa: E731
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=400, check_every=20,
                      deflation=osa.SCHUR)
    dinfo = ctx.deflate(10)
    assert dinfo["max_eig_resid"] < 1e-10
    for k, orth in ((30, 0), (60, 0), (120, 0), (60, 1)):   # delayed and plain CGS2
        ctx.set_opts(k_max=k, check_every=-1, deflation=osa.SCHUR, orth=orth)
        y, _, st = ctx.apply(dev(b))
        yo, info = O.schur_arnoldi_sign(mv, b, s, t, k=k)
        assert st == osa.OSA_OK and rel(host(y), yo) < 1e-9, (k, orth)
    ctx.set_opts(k_max=400, check_every=20, deflation=osa.SCHUR)
    y, infos, st = ctx.apply(dev(b), tol=1e-11)
    assert st == osa.OSA_OK and rel(host(y), yx) < 1e-9
    # a batch: the source, a source inside Omega_m (from the oracle's vectors) and
    # zero (no Krylov step: sign(T) c0 alone); the first bitwise as alone
    xin = r @ (np.arange(1, 11) + 0.5j)
    B = np.stack([b, xin, np.zeros_like(b)])
    Y, infs, st = ctx.apply(dev(B), tol=1e-11)
    Y = host(Y)
    assert st == osa.OSA_OK
    assert np.array_equal(Y[0], host(y))
    assert rel(Y[1], O.sign_eig_apply(h, xin)) < 1e-9
    assert not Y[2].any() and infs[2]["k_used"] == 0
    # fewer active pairs rebuild S and T from the leading right vectors
    ctx.set_active_deflation(6)
    ctx.set_opts(k_max=60, check_every=-1, deflation=osa.SCHUR)
    y6, _, st = ctx.apply(dev(b))
    s6, t6 = O.schur_basis(r[:, :6], mv)
    assert st == osa.OSA_OK
    assert rel(host(y6), O.schur_arnoldi_sign(mv, b, s6, t6, k=60)[0]) < 1e-9
    ctx.close()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_schur_vs_lr_and_state_errors(osa, haar3_schur):
    """Results section: Schur deflation needs only right eigenvectors (about half
    the eigensolver's stencil applications of LR) at about LR's accuracy.  Data
    without left vectors refuses LR and adjoint solves with OSA_ERR_STATE."""
    dims, links, b, h, r, s, t, yx = haar3_schur
    say("schur vs lr 3^4")
    cs = osa.Context(dev(links), dims, 0.3, -1.5, k_max=60, check_every=-1, deflation=osa.SCHUR)
    cl = osa.Context(dev(links), dims, 0.3, -1.5, k_max=60, check_every=-1)
    ds, dl = cs.deflate(10), cl.deflate(10)
    assert ds["eig_matvecs"] < 0.7 * dl["eig_matvecs"]
    es = rel(host(cs.apply(dev(b))[0]), yx)
    el = rel(host(cl.apply(dev(b))[0]), yx)
    assert 0.1 < es / el < 10.0, (es, el)
    _, _, st = cs.apply_adjoint(dev(b), check=False)
    assert st == osa.OSA_ERR_STATE
    cs.set_opts(k_max=60, check_every=-1)          # LR solve on right-only data
    _, _, st = cs.apply(dev(b), check=False)
    assert st == osa.OSA_ERR_STATE
    # right-only data moves between contexts: export without L, import with L = None
    with pytest.raises(osa.OsaError):
        cs.get_deflation()                          # no left vectors to export
    R, _, lam = cs.get_deflation(left=False)
    cs.set_opts(k_max=60, check_every=-1, deflation=osa.SCHUR)
    c2 = osa.Context(dev(links), dims, 0.3, -1.5, k_max=60, check_every=-1, deflation=osa.SCHUR)
    c2.set_deflation(R, None, lam)
    assert torch_equal(cs.apply(dev(b))[0], c2.apply(dev(b))[0])
    c2.close()
    # LR data serves Schur solves as well (only R is used)
    cl.set_opts(k_max=60, check_every=-1, deflation=osa.SCHUR)
    ys = host(cl.apply(dev(b))[0])
    assert rel(ys, O.schur_arnoldi_sign(lambda x: h @ x, b, s, t, k=60)[0]) < 1e-9
    cs.close()
    cl.close()


def test_torch_allocator_hook(osa):
    """Workspace from PyTorch's caching allocator (osa_set_allocator): the same
    solve gives bitwise the hipMalloc result; torch accounts for the workspace
    while the context lives and gets it back when the context is destroyed."""
    import torch
    dims = (3, 3, 3, 3)
    links = dev(LI.make_links(dims, "haar", cfg=0, inst=11))
    b = dev(LI.gaussian_source(dims, cfg=0, inst=11))
    say("allocator hook: hipMalloc run, then torch caching allocator run")
    c0 = osa.Context(links, dims, 0.3, -1.5, k_max=300, check_every=20)
    c0.deflate(8)
    y0, _, st0 = c0.apply(b, tol=1e-10)
    c0.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    osa.use_torch_allocator(True)
    try:
        c1 = osa.Context(links, dims, 0.3, -1.5, k_max=300, check_every=20)
        c1.deflate(8)
        y1, _, st1 = c1.apply(b, tol=1e-10)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        assert st0 == st1 == osa.OSA_OK
        assert torch.equal(y0, y1)
        assert held > 300 * 12 * 81 * 16          # at least the Krylov basis
        c1.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - base < held
    finally:
        osa.use_torch_allocator(False)


# -------------------------------------------- invariants at the 8^4 bench lattice
def test_invariants_at_8_4(osa):
    """Beyond dense sizes: sign(sign(H) b) = b (sign(A)^2 = 1); sign(H)(H b) =
    H sign(H) b (commutation); <a, sign(H) b> = <sign(H)^dag a, b> (adjoint); and
    the whole solver on the free field against the momentum-space closed form."""
    dims = (8, 8, 8, 8)
    links = LI.make_links(dims, "disordered", eps=0.6, cfg=1, inst=0)
    b = dev(LI.gaussian_source(dims, cfg=1, inst=0))
    say("invariants 8^4: deflate 20 at mu = 0.1")
    ctx = osa.Context(dev(links), dims, 0.1, -1.5, k_max=900, check_every=50)
    ctx.deflate(20)
    tol = 1e-10
    y, _, st = ctx.apply(b, tol=tol)
    assert st == osa.OSA_OK
    z, _, st = ctx.apply(y, tol=tol)
    assert st == osa.OSA_OK and rel(host(z), host(b)) < 10 * tol
    hb = ctx.apply_hw(b)
    shb, _, st = ctx.apply(hb, tol=tol)
    hy = ctx.apply_hw(y)
    assert st == osa.OSA_OK and rel(host(shb), host(hy)) < 10 * tol
    rng = np.random.default_rng(17)
    a = rng.standard_normal(b.shape[0]) + 1j * rng.standard_normal(b.shape[0])
    a /= np.linalg.norm(a)
    ya, _, st = ctx.apply_adjoint(dev(a), tol=tol)
    assert st == osa.OSA_OK
    lhs, rhs = np.vdot(a, host(y)), np.vdot(host(ya), host(b))
    assert abs(lhs - rhs) < 10 * tol
    ctx.close()
    say("invariants 8^4: free-field solve against the closed form")
    u = LI.make_links(dims, "unit")
    bf = LI.gaussian_source(dims, cfg=9, inst=5)
    # mu = 0.3: the free spectrum keeps |Re lambda| >= 0.135 (at mu = 0.5 one momentum
    # sits on the imaginary axis, where the sign is undefined)
    cf = osa.Context(dev(u), dims, 0.3, -1.5, k_max=900, check_every=50)
    yf, _, st = cf.apply(dev(bf), tol=tol)
    assert st == osa.OSA_OK
    assert rel(host(yf), O.free_field_sign_apply(dims, 0.3, -1.5, bf)) < 10 * tol
    cf.close()
