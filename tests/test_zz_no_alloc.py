"""The allocation-free small sign (osa_small_sign_noalloc) against the allocating
osa_small_sign, through the C ABI: bitwise equal results on two calls in a row
on the shared device scratch array, the second with a smaller matrix, both
checked against the spectral sign (Eq. 4-6) of the oracle; sizes beyond the
array's limit are rejected before any device work."""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def osa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_0710_0341_amd as osa_mod
    osa_mod.lib()
    return osa_mod


def hessenberg_case(k, seed):
    """An upper Hessenberg matrix with the spectrum of a Krylov H_k: a shifted
    random Hessenberg with eigenvalues away from the imaginary axis."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    a = np.triu(a, -1) / np.sqrt(k)
    return a + np.diag(np.where(np.arange(k) % 2 == 0, 1.5, -1.5))


def test_noalloc_small_sign_matches_allocating(osa):
    for k, seed in ((240, 1), (57, 2)):          # second call smaller than the first
        print(f"noalloc small sign k={k}", flush=True)
        sys.stdout.flush()
        a = hessenberg_case(k, seed)
        A = torch.from_numpy(a).to("cuda:0")
        s_ref, it_ref = osa.small_sign(A)
        s_na, it_na = osa.small_sign(A, noalloc=True)
        torch.cuda.synchronize()
        assert it_na == it_ref
        assert torch.equal(s_na, s_ref)
        exact = O.sign_eig(a)[:, 0]
        got = s_na.cpu().numpy()
        assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-10


def test_noalloc_rejects_beyond_limit(osa):
    L = osa.lib()
    A = torch.zeros((300, 300), dtype=torch.complex128, device="cuda:0")
    s = torch.empty(300, dtype=torch.complex128, device="cuda:0")
    it = ctypes.c_int32(0)
    st = L.osa_small_sign_noalloc(257, ctypes.c_void_p(A.data_ptr()),
                                  ctypes.c_void_p(s.data_ptr()), ctypes.byref(it), None)
    assert st == -1
