"""GPU parity of the two-step block form of the Arnoldi recurrence (opts.orth =
2: the basis grows by H u and H^2 u per outer step, one dot pass and one
update pass over the basis per two steps).  It builds the same Arnoldi
decomposition (Eq. 7) as the oracle's CGS2 recurrence in exact arithmetic, so
Eq. 22 at a fixed k (even or odd) matches the oracle to the FP64 bar (1e-10) and the
one-step delayed form to 1e-12; converged solves meet the dense sign; batches
stay bitwise equal to single-source solves.
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


def _solve_fixed(osa, links, dims, mu, b, k, orth, defl=None, reproject=True):
    ctx = osa.Context(dev(links), dims, mu, -1.5, k_max=k, check_every=-1, orth=orth,
                      no_reproject=not reproject)
    if defl is not None:
        ctx.set_deflation(dev(defl.r.T.copy()), dev(defl.l.T.copy()), defl.lam)
    y, infos, st = ctx.apply(dev(b), tol=1e-30)
    ctx.close()
    return host(y), infos[0]


@pytest.mark.parametrize("dims,kind,mu,m,k,reproject", [
    ((2, 2, 2, 2), "haar", 0.3, 0, 40, True),
    ((3, 4, 3, 4), "disordered", 0.5, 0, 90, True),
    ((3, 4, 3, 4), "disordered", 0.5, 8, 90, True),
    ((3, 4, 3, 4), "disordered", 0.5, 8, 60, False),
    ((4, 4, 4, 4), "haar", 0.3, 10, 150, True),
    ((2, 3, 2, 4), "haar", 0.4, 6, 2, True),       # a single outer step
])
def test_two_step_fixed_k_matches_oracle(osa, dims, kind, mu, m, k, reproject):
    say(f"two-step fixed k dims={dims} m={m} k={k} reproject={reproject}")
    links = LI.make_links(dims, kind, eps=0.6, cfg=9, inst=3)
    b = LI.gaussian_source(dims, cfg=9, inst=3)
    h = O.hermitian_wilson_sparse(links, dims, mu, -1.5)
    defl = None
    if m:
        r, l, lam = O.critical_dense(h.toarray(), m)
        defl = O.Deflation(r, l, lam)
    y2, i2 = _solve_fixed(osa, links, dims, mu, b, k, 2, defl, reproject)
    y0, i0 = _solve_fixed(osa, links, dims, mu, b, k, 0, defl, reproject)
    yo, info = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=k, reproject=reproject)
    assert i2["k_used"] == i0["k_used"] == info["k_used"] == k
    assert rel(y2, yo) < 1e-10
    assert rel(y2, y0) < 1e-12


@pytest.mark.parametrize("k", [61, 1])
def test_two_step_odd_fixed_k(osa, k):
    """An odd size: the outer step n = k completes size k + 1, the check uses k."""
    dims = (3, 4, 3, 4)
    links = LI.make_links(dims, "disordered", eps=0.6, cfg=9, inst=4)
    b = LI.gaussian_source(dims, cfg=9, inst=4)
    h = O.hermitian_wilson_sparse(links, dims, 0.5, -1.5)
    say(f"two-step, fixed odd k = {k}")
    y2, i2 = _solve_fixed(osa, links, dims, 0.5, b, k, 2)
    y0, i0 = _solve_fixed(osa, links, dims, 0.5, b, k, 0)
    yo, _ = O.lr_arnoldi_sign(lambda x: h @ x, b, None, k=k)
    assert i2["k_used"] == i0["k_used"] == k
    assert rel(y2, yo) < 1e-10
    assert rel(y2, y0) < 1e-12


@pytest.fixture(scope="module")
def haar4():
    w = LI.WORKLOADS[0]
    dims = w["dims"]
    links = LI.make_links(dims, "haar", cfg=0, inst=0)
    h = O.hermitian_wilson_dense(links, dims, w["mu"], w["m_w"])
    return dims, links, h


def test_two_step_converged_batch_and_adjoint(osa, haar4):
    """Converged solves with GPU deflation: against the dense sign and its
    adjoint; a lockstep batch of point and Gaussian sources is bitwise the
    single-source results; the checks fall at the one-step form's sizes."""
    dims, links, h = haar4
    say("two-step converged haar4 (GPU deflation, m = 10)")
    srcs = [LI.gaussian_source(dims, cfg=0, inst=0)] + [LI.point_source(dims, 0, s, 0)
                                                        for s in range(3)]
    B = np.stack(srcs)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=501, check_every=25, orth=2)
    ctx.deflate(10)
    yb, infos, st = ctx.apply(dev(B), tol=1e-11)
    assert st == osa.OSA_OK
    yb = host(yb)
    sgn = O.sign_eig(h)   # the dense sign, once
    for i, src in enumerate(srcs):
        assert infos[i]["k_used"] % 25 == 0 or infos[i]["k_used"] == 501
        assert rel(yb[i], sgn @ src) < 1e-10
        y1, inf1, _ = ctx.apply(dev(src), tol=1e-11)
        assert inf1[0]["k_used"] == infos[i]["k_used"]
        assert np.array_equal(host(y1), yb[i])
    ya, ia, sa = ctx.apply_adjoint(dev(srcs[0]), tol=1e-11)
    assert sa == osa.OSA_OK
    assert rel(host(ya), sgn.conj().T @ srcs[0]) < 1e-10   # sign(H)^dag
    ctx.close()


def test_two_step_breakdown_and_not_converged(osa):
    say("two-step: breakdown on a free plane wave")
    dims = (2, 2, 2, 4)
    u = LI.make_links(dims, "unit")
    t = np.arange(dims[3])
    wave = np.exp(2j * np.pi * t / dims[3])[:, None, None, None, None, None] * np.ones((1, 2, 2, 2, 4, 3))
    chi = np.zeros((4, 3), dtype=complex)
    chi[0, 0] = 1.0
    b = (wave * chi).reshape(-1)
    b /= np.linalg.norm(b)
    ctx = osa.Context(dev(u), dims, 0.3, -1.5, k_max=50, check_every=6, orth=2)
    y, infos, st = ctx.apply(dev(b), tol=1e-12)
    assert infos[0]["breakdown"] == 1 and infos[0]["k_used"] <= 4
    assert rel(host(y), O.free_field_sign_apply(dims, 0.3, -1.5, b)) < 1e-12
    ctx.close()
    say("two-step: not converged at an odd k_max = 21")
    dims = (3, 3, 3, 3)
    links = LI.make_links(dims, "haar", cfg=9, inst=7)
    b = LI.gaussian_source(dims, cfg=9, inst=7)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=21, check_every=10, orth=2)
    y, infos, st = ctx.apply(dev(b), tol=1e-14)
    assert st == osa.OSA_NOT_CONVERGED and infos[0]["k_used"] == 21
    ctx.close()


def test_two_step_batch_beyond_one_projection_group(osa, haar4):
    """14 sources in lockstep: the two new columns of every source make 28
    projected vectors, more than one projection launch takes (24), so the
    dots and the update run in two groups; each source stays bitwise its
    single-source solve (fixed k, LR deflation with the re-projection)."""
    dims, links, h = haar4
    say("two-step lockstep batch of 14 sources (two projection groups)")
    srcs = [LI.point_source(dims, 0, s, c) for s in range(4) for c in range(3)]
    srcs += [LI.gaussian_source(dims, cfg=0, inst=i) for i in (2, 3)]
    B = np.stack(srcs)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=40, check_every=-1, orth=2,
                      max_batch=16)
    ctx.deflate(10)
    yb, infos, st = ctx.apply(dev(B), tol=1e-30, check=False)
    yb = host(yb)
    assert all(i["k_used"] == 40 for i in infos)
    for i in (0, 7, 12, 13):
        y1, inf1, _ = ctx.apply(dev(srcs[i]), tol=1e-30, check=False)
        assert inf1[0]["k_used"] == 40
        assert np.array_equal(host(y1), yb[i])
    ctx.close()


def test_two_step_64_pairs(osa):
    """The largest deflation (64 pairs, the widest projection kernel shape):
    Eq. 22 at a fixed k against the oracle (1e-10) and the one-step form
    (1e-12), a batch bitwise equal to single-source solves; 65 pairs are
    rejected."""
    dims = (3, 3, 3, 3)
    links = LI.make_links(dims, "haar", cfg=9, inst=8)
    h = O.hermitian_wilson_sparse(links, dims, 0.3, -1.5)
    r, l, lam = O.critical_dense(h.toarray(), 65)
    defl = O.Deflation(r[:, :64], l[:, :64], lam[:64])
    srcs = [LI.gaussian_source(dims, cfg=9, inst=30 + i) for i in range(3)]
    say("two-step with 64 deflation pairs, fixed k = 30")
    y2, i2 = _solve_fixed(osa, links, dims, 0.3, srcs[0], 30, 2, defl)
    y0, i0 = _solve_fixed(osa, links, dims, 0.3, srcs[0], 30, 0, defl)
    yo, info = O.lr_arnoldi_sign(lambda x: h @ x, srcs[0], defl, k=30)
    assert i2["k_used"] == i0["k_used"] == info["k_used"] == 30
    assert rel(y2, yo) < 1e-10
    assert rel(y2, y0) < 1e-12
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=30, check_every=-1, orth=2)
    ctx.set_deflation(dev(defl.r.T.copy()), dev(defl.l.T.copy()), defl.lam)
    yb, _, _ = ctx.apply(dev(np.stack(srcs)), tol=1e-30, check=False)
    yb = host(yb)
    for i, s in enumerate(srcs):
        y1, _, _ = ctx.apply(dev(s), tol=1e-30, check=False)
        assert np.array_equal(host(y1), yb[i])
    with pytest.raises(osa.OsaError):
        ctx.set_deflation(dev(r.T.copy()), dev(l.T.copy()), lam)
    ctx.close()
