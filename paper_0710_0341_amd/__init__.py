"""Python binding of libosa: y = sign(H_w(mu)) b on MI355X.

Thin ctypes layer over the C ABI in include/osa.h: argument checks and
marshalling only.  Every step of the computation runs in the library's HIP
kernels; PyTorch supplies device memory (torch.empty on the GPU) and the
current stream.  There is no CPU fallback: if libosa.so is missing or the
device is not a GPU, the calls raise.

Layouts (boundary, identical to the C ABI):
  links: complex128 or complex64 tensor of shape (V, 4, 3, 3)
         (site = x + Lx*(y + Ly*(z + Lz*t)), direction 3 = time)
  vectors: complex128 tensor of shape (N,) or (nrhs, N), N = 12 V,
           index (site*4 + spin)*3 + color.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libosa.so")

OSA_OK = 0
OSA_NOT_CONVERGED = 1
OSA_ERR_STATE = -8
STATUS_NAMES = {0: "OSA_OK", 1: "OSA_NOT_CONVERGED", -1: "OSA_ERR_ARG", -2: "OSA_ERR_HIP",
                -3: "OSA_ERR_OOM", -4: "OSA_ERR_NONFINITE", -5: "OSA_ERR_IMAG_AXIS",
                -6: "OSA_ERR_EIG_NOCONV", -7: "OSA_ERR_NEWTON_NOCONV", -8: "OSA_ERR_STATE"}
FP64, FP32 = 0, 1
LR, SCHUR = 0, 1   # osa_opts.deflation

EXPORTS = ["overlap_sign_apply", "osa_create", "osa_deflate", "osa_set_deflation",
           "osa_get_deflation", "osa_set_active_deflation", "osa_apply", "osa_apply_adjoint",
           "osa_apply_overlap", "osa_apply_block", "osa_batch_apply",
           "osa_set_opts", "osa_apply_hw", "osa_apply_hw32", "osa_krylov_h2", "osa_small_sign", "osa_small_sign_noalloc",
           "osa_small_gemm", "osa_small_schur",
           "osa_set_links",
           "osa_profile_enable", "osa_profile_read", "osa_last_message", "osa_destroy",
           "osa_status_string", "osa_set_allocator", "osa_set_autotune", "osa_autotune_table",
           "osa_graph_stats", "osa_version"]

# device workspace allocator hook: alloc(bytes, stream, user), dealloc(ptr, stream, user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_hooks = []   # every registered callback pair stays alive: buffers return through their own


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("antiperiodic_t", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("no_reproject", ctypes.c_int32), ("eig_ncv", ctypes.c_int32),
                ("eig_max_restarts", ctypes.c_int32), ("eig_prec", ctypes.c_int32),
                ("eig_tol", ctypes.c_double), ("max_batch", ctypes.c_int32),
                ("orth", ctypes.c_int32), ("eig_filter", ctypes.c_int32),
                ("deflation", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("no_graphs", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("resid_est", ctypes.c_double), ("min_abs_re_lambda", ctypes.c_double),
                ("max_eig_resid", ctypes.c_double), ("t_init_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("k_used", ctypes.c_int32),
                ("n_defl", ctypes.c_int32), ("status", ctypes.c_int32),
                ("newton_iters", ctypes.c_int32), ("eig_matvecs", ctypes.c_int64),
                ("eig_restarts", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("batch", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


NPROF = 7   # OSA_PROFILE_CLASSES


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NPROF), ("bytes", ctypes.c_double * NPROF),
                ("launches", ctypes.c_int64 * NPROF), ("counters", ctypes.c_int64 * 4),
                ("calls", ctypes.c_int64 * NPROF), ("flops", ctypes.c_double * NPROF)]

    CLASSES = ("cgs_dot", "cgs_update", "stencil", "small_inverse", "small_schur",
               "eig_restart", "small_gemm")

    COUNTERS = ("schur_sweeps", "schur_rotations", "newton_iterations", "eig_arnoldi_steps")

    def as_dict(self):
        d = {name: dict(ms=self.ms[i], bytes=self.bytes[i], launches=self.launches[i],
                        calls=self.calls[i], flops=self.flops[i])
             for i, name in enumerate(self.CLASSES)}
        d["counters"] = {name: int(self.counters[i]) for i, name in enumerate(self.COUNTERS)}
        return d


class OsaError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libosa.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libosa.so not found at {LIB_PATH}; run paper_0710_0341_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.overlap_sign_apply.argtypes = [ctypes.POINTER(Lattice), vp, i32, dbl, dbl, vp, dbl, i32, vp,
                                     ctypes.POINTER(dbl), vp]
    L.osa_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Lattice), vp, i32, dbl, dbl,
                             ctypes.POINTER(Opts), vp]
    L.osa_deflate.argtypes = [vp, i32, ctypes.POINTER(Info)]
    L.osa_set_deflation.argtypes = [vp, i32, vp, vp, ctypes.POINTER(dbl)]
    L.osa_get_deflation.argtypes = [vp, ctypes.POINTER(i32), vp, vp, ctypes.POINTER(dbl)]
    L.osa_set_active_deflation.argtypes = [vp, i32]
    L.osa_apply.argtypes = [vp, i32, vp, vp, dbl, ctypes.POINTER(Info)]
    L.osa_apply_adjoint.argtypes = [vp, i32, vp, vp, dbl, ctypes.POINTER(Info)]
    L.osa_apply_overlap.argtypes = [vp, i32, vp, vp, dbl, ctypes.POINTER(Info)]
    L.osa_apply_block.argtypes = [vp, i32, vp, vp, dbl, i32, ctypes.POINTER(Info)]
    L.osa_batch_apply.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  dbl, ctypes.POINTER(Info)]
    L.osa_set_opts.argtypes = [vp, ctypes.POINTER(Opts)]
    L.osa_apply_hw.argtypes = [vp, i32, vp, vp]
    L.osa_apply_hw32.argtypes = [vp, i32, vp, vp]
    L.osa_krylov_h2.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.osa_small_sign.argtypes = [i32, vp, vp, ctypes.POINTER(i32), vp]
    L.osa_small_schur.argtypes = [i32, vp, vp, vp, vp, i32, vp]
    L.osa_small_gemm.argtypes = [i32, i32, vp, vp, vp, vp]
    L.osa_small_sign_noalloc.argtypes = [i32, vp, vp, ctypes.POINTER(i32), vp]
    L.osa_set_links.argtypes = [vp, vp]
    L.osa_profile_enable.argtypes = [vp, i32]
    L.osa_profile_read.argtypes = [vp, ctypes.POINTER(Profile)]
    L.osa_last_message.argtypes = [vp]
    L.osa_last_message.restype = ctypes.c_char_p
    L.osa_destroy.argtypes = [vp]
    L.osa_destroy.restype = None
    L.osa_status_string.argtypes = [i32]
    L.osa_status_string.restype = ctypes.c_char_p
    L.osa_version.restype = ctypes.c_char_p
    L.osa_set_allocator.argtypes = [ALLOC_FN, DEALLOC_FN, vp]
    L.osa_set_autotune.argtypes = [i32]
    L.osa_autotune_table.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), i32]
    L.osa_autotune_table.restype = i32
    L.osa_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTS:
        if name not in ("osa_destroy", "osa_status_string", "osa_version", "osa_last_message",
                        "osa_autotune_table"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def use_torch_allocator(enable=True):
    """Route the library's device workspace through PyTorch's caching allocator
    (osa_set_allocator), or back to hipMalloc with enable=False.  Contexts keep
    the allocator they were given buffers from."""
    L = lib()
    if not enable:
        _check(L.osa_set_allocator(ALLOC_FN(), DEALLOC_FN(), None), "osa_set_allocator", False)
        return
    torch = _torch()

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:   # out of memory: the library reports OSA_ERR_OOM
            return None

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    pair = (ALLOC_FN(_alloc), DEALLOC_FN(_free))
    _hooks.append(pair)
    _check(L.osa_set_allocator(pair[0], pair[1], None), "osa_set_allocator", False)


def _check(status, where, allow_not_converged=True):
    if status == OSA_OK or (allow_not_converged and status == OSA_NOT_CONVERGED):
        return status
    raise OsaError(status, where)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _lattice(dims, antiperiodic_t=False):
    lat = Lattice()
    for i in range(4):
        lat.dims[i] = int(dims[i])
    lat.antiperiodic_t = 1 if antiperiodic_t else 0
    return lat


def make_opts(k_max=0, check_every=0, no_reproject=False, eig_ncv=0, eig_max_restarts=0,
              eig_prec=FP64, eig_tol=0.0, max_batch=0, orth=0, eig_filter=0, deflation=LR,
              stop_rule=0, no_graphs=False):
    o = Opts()
    o.k_max, o.check_every, o.no_reproject = int(k_max), int(check_every), int(bool(no_reproject))
    o.eig_ncv, o.eig_max_restarts, o.eig_prec = int(eig_ncv), int(eig_max_restarts), int(eig_prec)
    o.eig_tol = float(eig_tol)
    o.max_batch = int(max_batch)
    o.orth = int(orth)
    o.eig_filter = int(eig_filter)
    o.deflation = int(deflation)
    o.stop_rule = int(stop_rule)
    o.no_graphs = int(bool(no_graphs))
    return o


def _link_prec(links):
    torch = _torch()
    if links.dtype == torch.complex128:
        return FP64
    if links.dtype == torch.complex64:
        return FP32
    raise TypeError("links must be complex128 or complex64")


def overlap_sign_apply(links, dims, mu, m_w, b, tol, n_defl, antiperiodic_t=False):
    """One-shot y = sign(H_w(mu)) b.  Returns (y, resid_est, status)."""
    torch = _torch()
    prec = _link_prec(links)
    lp = _dev_ptr(links, links.dtype, "links")
    bp = _dev_ptr(b, torch.complex128, "b")
    y = torch.empty_like(b)
    est = ctypes.c_double(0.0)
    lat = _lattice(dims, antiperiodic_t)
    st = lib().overlap_sign_apply(ctypes.byref(lat), lp, prec, float(mu), float(m_w), bp,
                                  float(tol), int(n_defl), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.byref(est), _stream())
    _check(st, "overlap_sign_apply")
    return y, est.value, st


sign_apply = overlap_sign_apply


class Context:
    """Reusable context: create once, deflate once, apply to many sources."""

    def __init__(self, links, dims, mu, m_w, antiperiodic_t=False, stream=None, **opts):
        """stream: a torch.cuda.Stream for all work of this context (default: the
        current stream)."""
        self._h = ctypes.c_void_p(None)
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.N = 12 * self.V
        self.mu, self.m_w = float(mu), float(m_w)
        prec = _link_prec(links)
        lp = _dev_ptr(links, links.dtype, "links")
        if links.numel() != self.V * 36:
            raise ValueError("links must have V*4*3*3 entries")
        self._opts = make_opts(**opts)
        lat = _lattice(dims, antiperiodic_t)
        st = _stream() if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self.stream = stream
        _check(lib().osa_create(ctypes.byref(self._h), ctypes.byref(lat), lp, prec, self.mu,
                                self.m_w, ctypes.byref(self._opts), st), "osa_create",
               allow_not_converged=False)

    def close(self):
        if self._h:
            lib().osa_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_opts(self, **opts):
        self._opts = make_opts(**opts)
        _check(lib().osa_set_opts(self._h, ctypes.byref(self._opts)), "osa_set_opts", False)

    def deflate(self, n_defl):
        info = Info()
        st = lib().osa_deflate(self._h, int(n_defl), ctypes.byref(info))
        if st != OSA_OK:
            raise OsaError(st, "osa_deflate (" + lib().osa_last_message(self._h).decode() + ")")
        return info.as_dict()

    def set_deflation(self, R, L, lam):
        """R, L: complex128 GPU tensors (m, N); lam: m complex numbers (host).
        L may be None under Schur deflation."""
        torch = _torch()
        m = int(R.shape[0]) if R is not None else 0
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
        lam_d = lam.view(np.float64)
        if m:
            rp = _dev_ptr(R, torch.complex128, "R")
            lpp = _dev_ptr(L, torch.complex128, "L") if L is not None else ctypes.c_void_p(None)
        else:
            rp = lpp = ctypes.c_void_p(None)
        self._after_current()
        _check(lib().osa_set_deflation(self._h, m, rp, lpp,
                                       lam_d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "osa_set_deflation", False)

    def get_deflation(self, device="cuda", left=True):
        """(R, L, lambda); left=False skips L (returned as None), which a
        Schur-mode deflation does not hold."""
        torch = _torch()
        m = ctypes.c_int32(0)
        _check(lib().osa_get_deflation(self._h, ctypes.byref(m), None, None, None),
               "osa_get_deflation", False)
        mm = m.value
        R = torch.empty((mm, self.N), dtype=torch.complex128, device=device)
        L = torch.empty((mm, self.N), dtype=torch.complex128, device=device) if left else None
        lam = np.zeros(2 * max(mm, 1))
        _check(lib().osa_get_deflation(self._h, ctypes.byref(m), ctypes.c_void_p(R.data_ptr()),
                                       ctypes.c_void_p(L.data_ptr() if left else None),
                                       lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "osa_get_deflation", False)
        return R, L, lam[: 2 * mm].view(np.complex128)

    def set_active_deflation(self, m):
        _check(lib().osa_set_active_deflation(self._h, int(m)), "osa_set_active_deflation", False)

    def apply(self, B, tol=1e-10, check=True):
        """Y = sign(H) B for B of shape (N,) or (nrhs, N).  Returns (Y, infos, status).
        Up to max_batch sources run in lockstep.  check=False returns error
        statuses instead of raising (per-source statuses are in infos)."""
        return self._apply("osa_apply", B, tol, check)

    def apply_adjoint(self, B, tol=1e-10, check=True):
        """Y = sign(H)^dag B = sign(H(-mu)) B, with the same deflation data."""
        return self._apply("osa_apply_adjoint", B, tol, check)

    def apply_overlap(self, B, tol=1e-10, check=True):
        """Y = D_ov B = B + gamma_5 sign(H) B (the overlap operator)."""
        return self._apply("osa_apply_overlap", B, tol, check)

    def apply_block(self, B, tol=1e-10, k_blocks=0, check=True):
        """Y = sign(H) B for the s rows of B by the block Krylov variant (one Krylov
        space for all s sources).  Returns (Y, infos, status)."""
        torch = _torch()
        bp = _dev_ptr(B, torch.complex128, "B")
        s = 1 if B.dim() == 1 else int(B.shape[0])
        Y = torch.zeros_like(B)
        self._after_current()
        infos = (Info * s)()
        st = lib().osa_apply_block(self._h, s, bp, ctypes.c_void_p(Y.data_ptr()), float(tol),
                                   int(k_blocks), infos)
        if check:
            _check(st, "osa_apply_block")
        return Y, [i.as_dict() for i in infos], st

    def _apply(self, name, B, tol, check):
        torch = _torch()
        bp = _dev_ptr(B, torch.complex128, "B")
        nrhs = 1 if B.dim() == 1 else int(B.shape[0])
        Y = torch.zeros_like(B)
        self._after_current()
        infos = (Info * nrhs)()
        st = getattr(lib(), name)(self._h, nrhs, bp, ctypes.c_void_p(Y.data_ptr()), float(tol),
                                  infos)
        if check:
            _check(st, name)
        return Y, [i.as_dict() for i in infos], st

    def _after_current(self):
        """Order this context's stream after the work queued so far on the current
        stream (inputs, output allocation)."""
        if self.stream is not None:
            self.stream.wait_stream(_torch().cuda.current_stream())

    def set_links(self, links):
        """Re-ingest new links (same lattice and precision); drops the deflation data."""
        lp = _dev_ptr(links, links.dtype, "links")
        self._after_current()
        _check(lib().osa_set_links(self._h, lp), "osa_set_links", False)

    def profile(self, enable=True, every=1):
        """Event timing of kernel classes; every=n brackets one launch in n per class."""
        n = max(1, int(every)) if enable else 0
        _check(lib().osa_profile_enable(self._h, n), "osa_profile_enable", False)

    def profile_read(self):
        out = Profile()
        _check(lib().osa_profile_read(self._h, ctypes.byref(out)), "osa_profile_read", False)
        return out.as_dict()

    def graph_stats(self):
        """(segments recorded as HIP graphs, graph launches) of this context."""
        cap, lau = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().osa_graph_stats(self._h, ctypes.byref(cap), ctypes.byref(lau)),
               "osa_graph_stats", False)
        return cap.value, lau.value

    def apply_hw(self, X):
        """Y = H_w(mu) X (stencil only)."""
        torch = _torch()
        xp = _dev_ptr(X, torch.complex128, "X")
        nrhs = 1 if X.dim() == 1 else int(X.shape[0])
        Y = torch.empty_like(X)
        self._after_current()
        _check(lib().osa_apply_hw(self._h, nrhs, xp, ctypes.c_void_p(Y.data_ptr())),
               "osa_apply_hw", False)
        return Y

    def apply_hw32(self, X):
        """Y = H_w(mu) X with the FP32 stencil (X, Y complex64)."""
        torch = _torch()
        xp = _dev_ptr(X, torch.complex64, "X")
        nrhs = 1 if X.dim() == 1 else int(X.shape[0])
        if X.numel() != nrhs * self.N:
            raise ValueError(f"X must hold nrhs x {self.N} entries")
        Y = torch.empty_like(X)
        self._after_current()
        _check(lib().osa_apply_hw32(self._h, nrhs, xp, ctypes.c_void_p(Y.data_ptr())),
               "osa_apply_hw32", False)
        return Y

    def krylov_h2(self, x, k, prec=FP64, adjoint=False):
        """k Arnoldi steps on H(mu)^2 (or H(-mu)^2) from x, as in the eigensearch.
        Returns (V, S): V (k+1, N) complex128, S (k+1, k) complex128 with
        A V[:k].T = V.T S."""
        torch = _torch()
        xp = _dev_ptr(x, torch.complex128, "x")
        if x.numel() != self.N:
            raise ValueError(f"x must hold {self.N} entries")
        V = torch.empty((k + 1, self.N), dtype=torch.complex128, device=x.device)
        S = torch.empty((k, k + 1), dtype=torch.complex128, device=x.device)
        self._after_current()
        _check(lib().osa_krylov_h2(self._h, prec, 1 if adjoint else 0, k, xp,
                                   ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(S.data_ptr())),
               "osa_krylov_h2", False)
        return V, S.T


def set_autotune(on=True):
    """Switch the dot-kernel autotuner on or off (process-wide)."""
    _check(lib().osa_set_autotune(1 if on else 0), "osa_set_autotune", False)


def autotune_table():
    """[(n, column bucket, chunk count)] of the keys tuned so far."""
    L = lib()
    total = L.osa_autotune_table(None, None, None, 0)
    n = (ctypes.c_int64 * max(total, 1))()
    b = (ctypes.c_int32 * max(total, 1))()
    w = (ctypes.c_int32 * max(total, 1))()
    L.osa_autotune_table(n, b, w, total)
    return [(int(n[i]), int(b[i]), int(w[i])) for i in range(total)]


def batch_apply(contexts, sources, tol=1e-10, check=True):
    """Uneven batch: one source per context, instances solved concurrently.
    Returns (outputs, infos, status); check=False returns error statuses
    instead of raising."""
    torch = _torch()
    n = len(contexts)
    outs = [torch.zeros_like(b) for b in sources]
    for c in contexts:
        c._after_current()
    hs = (ctypes.c_void_p * n)(*[c._h.value for c in contexts])
    bs = (ctypes.c_void_p * n)(*[_dev_ptr(b, torch.complex128, "B").value for b in sources])
    ys = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    infos = (Info * n)()
    st = lib().osa_batch_apply(n, hs, bs, ys, float(tol), infos)
    if check:
        _check(st, "osa_batch_apply")
    return outs, [i.as_dict() for i in infos], st


def small_schur(A, mode=0):
    """(T, Z, w) with A = Z T Z^H for a square complex128 GPU tensor A (p <= 96)."""
    torch = _torch()
    p = int(A.shape[0])
    Acm = A.t().contiguous()
    T = torch.empty((p, p), dtype=torch.complex128, device=A.device)
    Z = torch.empty((p, p), dtype=torch.complex128, device=A.device)
    w = torch.empty(p, dtype=torch.complex128, device=A.device)
    _check(lib().osa_small_schur(p, ctypes.c_void_p(Acm.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                 ctypes.c_void_p(Z.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                 int(mode), _stream()), "osa_small_schur", False)
    return T.t(), Z.t(), w          # column-major storage -> row-major views


def small_gemm(A, B):
    """C = A @ B for complex128 GPU tensors of shape (n, n) or (nb, n, n), on the
    library's FP64 matrix-core kernel."""
    torch = _torch()
    single = A.dim() == 2
    A3 = A.unsqueeze(0) if single else A
    B3 = B.unsqueeze(0) if single else B
    nb, n = int(A3.shape[0]), int(A3.shape[1])
    Acm = A3.transpose(1, 2).contiguous()      # column-major storage per problem
    Bcm = B3.transpose(1, 2).contiguous()
    C = torch.empty_like(Acm)
    _check(lib().osa_small_gemm(n, nb, ctypes.c_void_p(Acm.data_ptr()),
                                ctypes.c_void_p(Bcm.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                _stream()), "osa_small_gemm", False)
    C = C.transpose(1, 2)
    return C[0] if single else C


def small_sign(A, noalloc=False):
    """s = sign(A) e_1 for a square complex128 GPU tensor A (the Newton kernel).
    noalloc=True calls osa_small_sign_noalloc (workspace in the library's static
    device array, k <= 256)."""
    torch = _torch()
    k = int(A.shape[0])
    Acm = A.t().contiguous()          # column-major storage
    s = torch.empty(k, dtype=torch.complex128, device=A.device)
    it = ctypes.c_int32(0)
    name = "osa_small_sign_noalloc" if noalloc else "osa_small_sign"
    _check(getattr(lib(), name)(k, ctypes.c_void_p(Acm.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                ctypes.byref(it), _stream()), name, False)
    return s, it.value
