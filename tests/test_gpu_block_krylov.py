"""The block Krylov variant (osa_apply_block) against the oracle's block Arnoldi
(oracle/block_krylov.py) through the C ABI.  Not the paper's method: one
Krylov space for several sources, the block analogue of Eq. 11 / Eq. 22 with the
same LR deflation.  Fixed K: element by element to the FP64 bar 1e-10; one
source: the single-source Eq. 22; converged: within tolerance of the dense
sign (Eq. 4-6)."""
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


@pytest.fixture(scope="module")
def haar4():
    w = LI.WORKLOADS[0]
    dims = w["dims"]
    links = LI.make_links(dims, "haar", cfg=0, inst=0)
    h = O.hermitian_wilson_dense(links, dims, w["mu"], w["m_w"])
    return dims, links, h


@pytest.mark.parametrize("s,kb,m", [(4, 30, 10), (3, 17, 0), (12, 8, 10)])
def test_block_fixed_k_matches_oracle(osa, haar4, s, kb, m):
    dims, links, h = haar4
    rng = np.random.default_rng(100 + s)
    B = rng.standard_normal((s, h.shape[0])) + 1j * rng.standard_normal((s, h.shape[0]))
    say(f"block fixed K={kb}, s={s}, m={m}")
    defl = O.Deflation(*O.critical_dense(h, m)) if m else None
    yo, info = O.block_lr_sign(lambda x: h @ x, B.T.copy(), defl, kb)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, check_every=-1)
    if m:
        ctx.set_deflation(dev(defl.r.T.copy()), dev(defl.l.T.copy()), defl.lam)
    Y, infos, st = ctx.apply_block(dev(B), tol=1.0, k_blocks=kb)
    Y = host(Y)
    ctx.close()
    assert infos[0]["k_used"] == info["dim"] == kb * s
    for i in range(s):
        err = rel(Y[i], yo[:, i])
        assert err < 1e-10, (i, err)


def test_block_one_source_is_eq22(osa, haar4):
    dims, links, h = haar4
    b = LI.gaussian_source(dims, cfg=0, inst=3)
    defl = O.Deflation(*O.critical_dense(h, 10))
    yo, _ = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=60)
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, check_every=-1)
    ctx.set_deflation(dev(defl.r.T.copy()), dev(defl.l.T.copy()), defl.lam)
    Y, _, _ = ctx.apply_block(dev(b[None, :]), tol=1.0, k_blocks=60)
    assert rel(host(Y)[0], yo) < 1e-10
    ctx.close()


def test_block_converged_point_sources(osa, haar4):
    """The 12 spin-colour point sources of site 0 solved together to tol 1e-9
    against the dense sign (the block space needs about 200 block steps here,
    dimension 2400 of N = 3072)."""
    dims, links, h = haar4
    n = h.shape[0]
    B = np.zeros((12, n), dtype=np.complex128)
    for sc in range(12):
        B[sc, sc] = 1.0
    S = O.sign_eig(h)
    say("block: 12 point sources to tol 1e-9")
    ctx = osa.Context(dev(links), dims, 0.3, -1.5, k_max=500, check_every=25, max_batch=12)
    ctx.deflate(10)
    Yb, infos, st = ctx.apply_block(dev(B), tol=1e-9, k_blocks=240)
    assert st == osa.OSA_OK
    Yb = host(Yb)
    say(f"  K s = {infos[0]['k_used']}, max est {max(i['resid_est'] for i in infos):.1e}")
    for i in range(12):
        assert rel(Yb[i], S[:, i]) < 1e-8
    ctx.close()
