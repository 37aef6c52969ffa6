// Host driver and C ABI of the osa library.
//
// Hot path (Eq. 22 of the LR-deflation section):
//   c       = (L^dag R)^{-1} L^dag b                       (Eq. 21, oblique projector)
//   x_ominus = b - R c ,  beta = |x_ominus|,  v_1 = x_ominus / beta
//   Arnoldi with classical Gram-Schmidt applied twice   (Eq. 7)
//   s       = sign(H_k) e_1 by the scaled Newton iteration
//   y       = R sgn(Re Lambda) c + beta V_k s           (Eq. 22)
// Critical eigenpairs (Eq. 20): Krylov-Schur on H^2 (smallest |lambda|^2),
// then a Rayleigh-Ritz step with H; left vectors from H(-mu) = H(mu)^dag.
//
// The host only sequences kernels and reads back a few scalars at
// checkpoints; every vector and matrix operation runs on the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <exception>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"

using namespace osa;

namespace {

// Process-wide allocation hook for device workspace (osa_set_allocator); each
// buffer keeps the hook that allocated it, so a later change of the hook does
// not mix allocators.
struct AllocHook {
    void* (*alloc)(size_t, void*, void*) = nullptr;   // (bytes, stream, user)
    void (*dealloc)(void*, void*, void*) = nullptr;   // (ptr, stream, user)
    void* user = nullptr;
};
std::mutex g_alloc_mu;
AllocHook g_alloc;

AllocHook current_alloc_hook() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

// Bumped by every device workspace (re)allocation and release: captured graphs
// hold raw pointers, so a graph recorded before the last change is stale.
std::atomic<uint64_t> g_alloc_epoch{1};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    AllocHook hook{};
    bool borrowed = false;   // memory owned elsewhere: never freed, never grown
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void borrow(void* q, size_t b) {
        release();
        p = q;
        bytes = b;
        borrowed = true;
    }
    void release() {
        if (borrowed) {
            p = nullptr;
            bytes = 0;
            borrowed = false;
            return;
        }
        if (p) {
            g_alloc_epoch.fetch_add(1);
            if (hook.dealloc) {
                // the hook's allocator may hand the block out again at once: let
                // every queued kernel finish first (hipFree does the same)
                (void)hipDeviceSynchronize();
                hook.dealloc(p, nullptr, hook.user);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
        hook = AllocHook{};
    }
    void ensure(size_t b) {
        if (b <= bytes && p) return;
        if (borrowed) throw std::length_error("borrowed workspace too small");
        release();
        g_alloc_epoch.fetch_add(1);
        if (b == 0) b = 16;
        const AllocHook h = current_alloc_hook();
        if (h.alloc) {
            p = h.alloc(b, nullptr, h.user);
            if (!p) throw std::bad_alloc();
            // the block may come from work still queued on another stream
            if (hipDeviceSynchronize() != hipSuccess) {
                (void)hipGetLastError();
                h.dealloc(p, nullptr, h.user);
                p = nullptr;
                throw std::bad_alloc();
            }
            hook = h;
            bytes = b;
            return;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw std::bad_alloc();
        }
        bytes = b;
    }
    template <typename T> T* as() const { return (T*)p; }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;   // ordinary host memory owned elsewhere
    ~PinnedBuf() {
        if (p && !borrowed) (void)hipHostFree(p);
    }
    void borrow(void* q, size_t b) {
        if (p && !borrowed) (void)hipHostFree(p);
        p = q;
        bytes = b;
        borrowed = true;
    }
    void ensure(size_t b) {
        if (b <= bytes && p) return;
        if (borrowed) throw std::length_error("borrowed host staging too small");
        if (p) (void)hipHostFree(p);
        p = nullptr;
        if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw std::bad_alloc();
        }
        bytes = b;
    }
    template <typename T> T* as() const { return (T*)p; }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct OsaError {
    osa_status s;
    std::string why = "";
};

// Per-problem block of the small data of a solve (in cd entries): the
// Hessenberg matrix (ldh = kcap + 1 rows, kcap + 1 columns: the delayed
// reorthogonalisation writes the first pass of one column ahead), the
// coefficient vectors, the two-vector dot products and a few scalar slots.  One stride covers all of them, so a batched
// launch reaches any of them with the same per-problem offset.
struct ArenaLayout {
    int ldh = 0;
    int64_t vec_len = 0;   // entries of each vector slot
    int64_t H = 0, coef = 0, coef2 = 0, cdef = 0, craw = 0, tmp = 0, s_cur = 0, s_prev = 0, dc = 0,
            ds = 0;
    int64_t b2 = 0;   // two-step block Arnoldi workspace (13 slots + scalars)
    int64_t xs = 0;   // Schur deflation: X = S^dag H V_k (m x (kcap + 1), ld m)
    int m = 0;
    int64_t stride = 0;
    static ArenaLayout make(int kcap, int m) {
        ArenaLayout a;
        a.ldh = kcap + 1;
        a.m = m;
        // vectors of the small problem: Schur deflation solves it at size m + k
        a.vec_len = std::max<int64_t>(kcap + m + 2, 160);
        int64_t o = (int64_t)a.ldh * (kcap + 1);
        a.coef = o;   o += a.vec_len;
        a.coef2 = o;  o += a.vec_len;
        a.cdef = o;   o += a.vec_len;
        a.craw = o;   o += a.vec_len;
        a.tmp = o;    o += a.vec_len;
        a.s_cur = o;  o += a.vec_len;
        a.s_prev = o; o += a.vec_len;
        a.dc = o;     o += 2 * a.vec_len;
        a.ds = o;     o += 8;
        a.b2 = o;     o += 13 * a.vec_len + 16;
        a.xs = o;     o += (int64_t)m * (kcap + 1);
        a.stride = ceil_div(o, 16) * 16;
        return a;
    }
};

}  // namespace

// ============================================================== context
constexpr int kBatchWorkers = 8;   // concurrent instances in osa_batch_apply

struct osa_ctx {
    Geom g{};
    hipStream_t st = nullptr;
    bool links_fp32 = false;
    double mu = 0, m_w = 0, kappa = 0, hnorm_bound = 0;
    HopCoef hc{}, hc_adj{};   // H(mu) and H(-mu)
    osa_opts opts{};

    DevBuf U;        // internal links
    DevBuf U32;      // fp32 copy for an fp32 eigen-search on fp64 links
    const void* u_ext = nullptr;     // a worker clone reads its parent's links
    const void* u32_ext = nullptr;
    bool own_stream = false;
    const void* links() const { return u_ext ? u_ext : U.p; }
    const void* links32() const { return u_ext ? u32_ext : U32.p; }

    // deflation data (internal layout, m_alloc vectors each)
    int m_alloc = 0, m_active = 0;
    DevBuf R, L, Ginv, lam_dev, sgnc, gnorm;
    // adjoint solves, sign(H(mu))^dag = sign(H(-mu)): the stencil of H(-mu), and
    // the deflation data with the left and right vectors swapped and G^{-1}
    // replaced by its conjugate transpose (GinvH)
    bool adj = false;
    DevBuf GinvH;
    // Schur deflation (Eq. 13): orthonormal basis S of the first schur_m right
    // vectors and T = S^dag H S; have_left: L holds left vectors (an LR deflation)
    bool have_left = true;
    int schur_m = 0;
    DevBuf Sch, Tsch;
    std::vector<cd> lambda;
    double max_eig_resid = 0, min_abs_re = 0;
    int64_t eig_matvecs = 0;
    int eig_restarts = 0;
    double t_init_ms = 0;

    // Krylov workspace, for up to kbatch sources solved in lockstep
    int kcap = 0, kbatch = 0;
    int scap = 0;   // size cap of the small sign problem (kcap, + m under Schur deflation)
    DevBuf V, arena, w, x, y, coef, coef2, partial, normp, upd_scratch, dscal, flag, nflag, red;
    DevBuf sX, sM, sY, logpiv, gjws;
    DevBuf xio, yio;   // internal-layout sources and results of osa_apply
    // block Krylov variant (osa_apply_block): basis, block Hessenberg matrix,
    // work block, coefficient buffers and the small solution F E_1 R_0
    DevBuf Vblk, Hblk, Wblk, cblk2, cdefb, ctmpb, r0b, ysmb, ccoefb;
    ArenaLayout lay;
    int64_t part_stride = 0, normp_stride = 0, red_stride = 0, gj_stride = 0;
    PinnedBuf host;

    // optional kernel timing (events on st, resolved at synchronisation points)
    struct Pending { hipEvent_t a, b; int cls; double bytes, flops; };
    bool prof_on = false;
    int prof_every = 1;   // bracket one launch in prof_every of each class
    std::vector<Pending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    osa_profile prof{};
    std::string msg;
    // Arnoldi segments (the steps between two convergence checks) captured as
    // HIP graphs and replayed; see run_segment
    struct SegKey {
        int j0, j1, m, flags;
        uint64_t mask;
        bool operator<(const SegKey& o) const {
            if (j0 != o.j0) return j0 < o.j0;
            if (j1 != o.j1) return j1 < o.j1;
            if (m != o.m) return m < o.m;
            if (flags != o.flags) return flags < o.flags;
            return mask < o.mask;
        }
    };
    struct SegGraph { hipGraphExec_t exec = nullptr; int seen = 0; bool failed = false; };
    std::map<SegKey, SegGraph> seg_graphs;
    uint64_t seg_epoch = 0;
    hipStream_t cap_st = nullptr;   // private stream for graph capture
    int64_t graph_launches = 0, graph_captures = 0;
    void clear_graphs() {
        for (auto& kv : seg_graphs)
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        seg_graphs.clear();
    }
    ~osa_ctx() {
        clear_graphs();
        if (cap_st) (void)hipStreamDestroy(cap_st);
        for (auto& p : prof_pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto e : prof_pool) (void)hipEventDestroy(e);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }

    int64_t N() const { return g.N(); }
};

namespace {

// ------------------------------------------------------------- utilities
void prof_resolve(osa_ctx* c) {
    for (auto& p : c->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof.ms[p.cls] += ms;
            c->prof.bytes[p.cls] += p.bytes;
            c->prof.flops[p.cls] += p.flops;
            c->prof.launches[p.cls] += 1;
        } else {
            (void)hipGetLastError();
        }
        c->prof_pool.push_back(p.a);
        c->prof_pool.push_back(p.b);
    }
    c->prof_pending.clear();
}

void sync(osa_ctx* c) {
    OSA_HIP(hipStreamSynchronize(c->st));
    if (!c->prof_pending.empty()) prof_resolve(c);
}

hipEvent_t prof_event(osa_ctx* c) {
    if (c->prof_pool.empty()) {
        hipEvent_t e;
        OSA_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
}

// Brackets the launches issued by f() with events when profiling is on.
template <typename F>
void timed(osa_ctx* c, int cls, double bytes, F&& f, double flops = 0.0) {
    if (!c->prof_on) { f(); return; }
    if (c->prof.calls[cls]++ % c->prof_every != 0) { f(); return; }
    hipEvent_t a = prof_event(c), b = prof_event(c);
    OSA_HIP(hipEventRecord(a, c->st));
    f();
    OSA_HIP(hipEventRecord(b, c->st));
    c->prof_pending.push_back({a, b, cls, bytes, flops});
    if (c->prof_pending.size() > 4096) sync(c);
}

template <typename T>
void d2h(osa_ctx* c, const void* dsrc, size_t n, T* out) {
    c->host.ensure(n * sizeof(T));
    OSA_HIP(hipMemcpyAsync(c->host.p, dsrc, n * sizeof(T), hipMemcpyDeviceToHost, c->st));
    sync(c);
    std::memcpy(out, c->host.p, n * sizeof(T));
}

template <typename T>
void h2d(osa_ctx* c, void* ddst, const T* src, size_t n) {
    c->host.ensure(n * sizeof(T));
    std::memcpy(c->host.p, src, n * sizeof(T));
    OSA_HIP(hipMemcpyAsync(ddst, c->host.p, n * sizeof(T), hipMemcpyHostToDevice, c->st));
    sync(c);
}

// out = H in (adjoint: H(-mu) = H(mu)^dag).  Batch strides: basis (in), vec (out).
void apply_h(osa_ctx* c, const void* in, void* out, bool fp32, bool adjoint,
             const Batch& bt = Batch()) {
    const void* U = c->links();
    bool ufp32 = c->links_fp32;
    if (fp32 && !c->links_fp32 && c->links32()) { U = c->links32(); ufp32 = true; }
    // algorithmic bytes per site: spinor in + out per source, 8 links (4 own,
    // 4 backward neighbours') once for the whole batch
    const double sb = fp32 ? 8.0 : 16.0, lb = ufp32 ? 8.0 : 16.0;
    const double bytes = (double)c->g.V * (bt.n * 24.0 * sb + 36.0 * lb);
    timed(c, 2, bytes, [&] {
        launch_wilson_h(in, out, U, ufp32, fp32, c->g, adjoint ? c->hc_adj : c->hc, c->st, bt);
    });
}

// Links for the FP32 kernels: FP32-stored links as they are, FP64-stored ones
// rounded once into U32 (kept in step by osa_set_links).
void ensure_links32(osa_ctx* c) {
    if (!c->links_fp32 && !c->U32.p) {
        c->U32.ensure(sizeof(cf) * (size_t)c->g.Vp * 36);
        launch_convert(c->U.p, false, c->U32.p, true, (int64_t)c->g.Vp * 36, c->st);
    }
}

// nrhs contiguous vectors
void apply_h_contig(osa_ctx* c, const void* in, void* out, bool fp32, bool adjoint, int nrhs) {
    const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
    for (int r0 = 0; r0 < nrhs; r0 += kMaxBatch) {
        Batch bt;
        bt.n = std::min(kMaxBatch, nrhs - r0);
        bt.basis = bt.vec = c->N();
        const size_t off = (size_t)r0 * c->N() * es;
        apply_h(c, (const char*)in + off, (char*)out + off, fp32, adjoint, bt);
    }
}

// Norm of an internal vector, to the device scalar hsub (cd, real part).
void vec_norm(osa_ctx* c, const void* v, bool fp32, cd* out) {
    TsPlan p = ts_plan(c->N());
    launch_norm_partial(v, fp32, p, c->normp.as<double>(), c->st);
    launch_normalize(v, nullptr, fp32, p, c->normp.as<double>(), out, nullptr, 0.0, nullptr, 0,
                     nullptr, 0, c->st);
}

// Work buffers of the tall-skinny kernels (Gram-Schmidt against up to maxcols
// vectors, for up to nb problems at once), shared by the solve and the
// eigensolver.  Per-problem strides: partial maxcols*kMaxChunks,
// normp ceil(N/256) + 16.
void ensure_exec(osa_ctx* c, int maxcols, int nb = 1) {
    const int64_t N = c->N();
    const size_t vb = (size_t)N * sizeof(cd);
    maxcols = std::max(maxcols, 160);
    c->coef.ensure(sizeof(cd) * maxcols);
    c->coef2.ensure(sizeof(cd) * maxcols);
    c->part_stride = std::max<int64_t>(c->part_stride, (int64_t)maxcols * kMaxChunks);
    c->normp_stride = ceil_div(N, 256) + 16;
    c->partial.ensure(sizeof(cd) * (size_t)c->part_stride * nb);
    c->normp.ensure(sizeof(double) * (size_t)c->normp_stride * nb);
    // column-split scratch (16 n per problem), only where rows alone cannot fill the GPU
    c->upd_scratch.ensure(ceil_div(N, 256) < 1024 ? vb * 16 * nb : 256);
    c->dscal.ensure(sizeof(cd) * 16);
    c->flag.ensure(sizeof(int) * 4 * nb);
    c->nflag.ensure(sizeof(int) * 4 * nb);
    c->host.ensure(1 << 16);
}

// Workspace of a lockstep solve of nb sources with Krylov size up to kcap:
//   V      nb bases of kcap+2 vectors (problem b at b*(kcap+2)*N)
//   arena  nb per-problem blocks of small data, see ArenaLayout
//   w, x   nb vectors each
//   sX, sM, sY, logpiv, gjws, red: nb copies of the small-sign workspace
void ensure_krylov(osa_ctx* c, int kcap, int nb = 1) {
    // Schur deflation solves the small sign at size m + k
    const int extra = c->opts.deflation == 1 ? c->m_alloc : 0;
    if (kcap <= c->kcap && nb <= c->kbatch && c->V.p && std::max(kcap, c->kcap) + extra <= c->scap)
        return;
    kcap = std::max(kcap, c->kcap);
    nb = std::max(nb, c->kbatch);
    const int scap = std::max(kcap + extra, c->scap);
    const int64_t N = c->N();
    const size_t vb = (size_t)N * sizeof(cd);
    c->V.release();   // the largest buffer: free before growing
    c->V.ensure(vb * (size_t)(kcap + 2) * nb);
    c->lay = ArenaLayout::make(kcap, std::max(c->m_alloc, 1));
    c->arena.ensure(sizeof(cd) * (size_t)c->lay.stride * nb);
    c->w.ensure(vb * nb);
    c->x.ensure(vb * nb);
    c->y.ensure(vb);
    ensure_exec(c, 2 * (kcap + 2), nb);
    c->red_stride = newton_red_len(scap) + 16;
    c->red.ensure(sizeof(double) * (size_t)c->red_stride * nb);
    c->sX.ensure(sizeof(cd) * (size_t)scap * scap * nb);
    c->sM.ensure(sizeof(cd) * (size_t)scap * scap * nb);
    c->sY.ensure(sizeof(cd) * (size_t)scap * scap * nb);
    c->logpiv.ensure(sizeof(double) * (size_t)scap * nb);
    c->gj_stride = (int64_t)ceil_div((int64_t)gj_ws_bytes(scap), 256) * 256;
    c->gjws.ensure((size_t)c->gj_stride * nb);
    c->kcap = kcap;
    c->scap = scap;
    c->kbatch = nb;
}

__global__ void k_axpy_c(int n, cd alpha, const cd* __restrict__ a, cd* __restrict__ cvec) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cvec[i] = cadd(cvec[i], cmul(alpha, a[i]));
}

void axpy_c(osa_ctx* c, int n, cd alpha, const cd* a, cd* cvec) {
    hipLaunchKernelGGL(k_axpy_c, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->st, n, alpha,
                       a, cvec);
    OSA_LAUNCH_CHECK();
}

Batch batch_of(const std::vector<int>& probs) {
    Batch bt;
    bt.n = (int)probs.size();
    for (int i = 0; i < bt.n; ++i) bt.idx[i] = (int16_t)probs[i];
    return bt;
}

// ------------------------------------------------------- Gram-Schmidt
// w <- w - B (B^H w) twice (CGS2); coefficients h = h1 + h2 written to hcol
// (device, ncols entries); co holds the pass-2 coefficients.  Leaves per-block
// norm partials of the result in normp.  B has ncols vectors of length n,
// spaced by ld.  Batch strides: vec (w), basis (B), small (hcol, co).
void cgs2(osa_ctx* c, void* wv, const void* B, int64_t ld, int ncols, bool fp32, cd* hcol,
          cd* co, const Batch& bt = Batch()) {
    const TsPlan p = ts_plan(c->N());
    const int64_t scratch_len = (int64_t)(c->upd_scratch.bytes / sizeof(cd));
    cd* part = c->partial.as<cd>();
    Batch bd = bt, bu = bt;
    bd.part = c->part_stride;
    bu.part = c->normp_stride;
    const double eb = fp32 ? 8.0 : 16.0;
    const double n = (double)c->N() * bt.n;
    const double dot_bytes = (ncols + 1.0) * n * eb;     // read V_j and w
    const double upd_bytes = (ncols + 2.0) * n * eb;     // read V_j and w, write w
    // pass 1
    int nch = 0;
    timed(c, 0, dot_bytes, [&] { nch = launch_dot_partial(B, ld, ncols, wv, fp32, p, part, c->st, bd); });
    launch_reduce_partial(part, nch, ncols, hcol, nullptr, nullptr, nullptr, c->st, bd);
    timed(c, 1, upd_bytes, [&] {
        launch_update(wv, B, ld, ncols, hcol, fp32, p, nullptr, c->upd_scratch.as<cd>(),
                      scratch_len, c->st, bu);
    });
    // pass 2
    timed(c, 0, dot_bytes, [&] { nch = launch_dot_partial(B, ld, ncols, wv, fp32, p, part, c->st, bd); });
    launch_reduce_partial(part, nch, ncols, co, hcol, nullptr, nullptr, c->st, bd);  // h += h2
    timed(c, 1, upd_bytes, [&] {
        launch_update(wv, B, ld, ncols, co, fp32, p, c->normp.as<double>(),
                      c->upd_scratch.as<cd>(), scratch_len, c->st, bu);
    });
}

// Oblique projection w <- w - R G^{-1} L^dag w (Eq. 21) with the active pairs,
// shared by every problem of the batch, for nv (1 or 2) vectors per problem:
// vector t at wv + b*bt.vec + t*off2.  The coefficients G^{-1} L^dag w of vector
// t are left in cout + t*m; tmp is nv*m scratch entries.  Under Schur deflation
// the projection is orthogonal, w <- w - S S^dag w, and cout = S^dag w.  Batch
// strides: vec (w), small (cout, tmp).
void project_out(osa_ctx* c, void* wv, cd* cout, cd* tmp, const Batch& bt, int nv = 1,
                 int64_t off2 = 0) {
    const int m = c->m_active;
    if (m == 0) return;
    const int64_t N = c->N();
    cd* part = c->partial.as<cd>();
    Batch bd = bt, bu = bt;
    bd.basis = bu.basis = 0;   // L and R are shared
    bd.part = c->part_stride;
    bu.part = 0;
    // Schur deflation: the orthogonal projector 1 - S S^dag (Eq. 14)
    const bool sch = c->opts.deflation == 1;
    const void* Lp = sch ? c->Sch.p : (c->adj ? c->R.p : c->L.p);
    const void* Rp = sch ? c->Sch.p : (c->adj ? c->L.p : c->R.p);
    const cd* Gi = sch ? nullptr : (c->adj ? c->GinvH.as<cd>() : c->Ginv.as<cd>());
    cd* w = (cd*)wv;
    // the LDS-tiled dots read L once for up to 24 vectors (m <= 64, the
    // deflation size limit); their summation order depends on (N, m) only, so
    // one source and a batch agree bitwise
    const int nch = launch_pdot_partial((const cd*)Lp, N, m, w, off2, nv, N, part, c->st, bd);
    for (int t = 0; t < nv; ++t)
        launch_reduce_partial(part + (size_t)t * m * nch, nch, m, cout + t * m, nullptr, Gi,
                              tmp + t * m, c->st, bd);
    if (bt.n * nv > 1 && mupdate_matches_single(N, m)) {
        launch_mupdate(w, (const cd*)Rp, N, m, cout, N, c->st, bu, nv, off2, m);
        return;
    }
    for (int t = 0; t < nv; ++t)
        launch_update(w + t * off2, Rp, N, m, cout + t * m, false, ts_plan(N), nullptr,
                      c->upd_scratch.as<cd>(), (int64_t)(c->upd_scratch.bytes / sizeof(cd)),
                      c->st, bu);
}

// Strided device-to-host copy of `width` bytes from each of the problems in
// probs (byte stride `stride` from src); out[i] receives problem probs[i].
template <typename T>
void d2h_strided(osa_ctx* c, const void* src, int64_t stride, int count,
                 const std::vector<int>& probs, std::vector<T>& out) {
    int nb = 0;
    for (int b : probs) nb = std::max(nb, b + 1);
    const size_t w = sizeof(T) * count;
    c->host.ensure(w * nb + 16);
    OSA_HIP(hipMemcpy2DAsync(c->host.p, w, src, (size_t)stride, w, nb, hipMemcpyDeviceToHost,
                             c->st));
    sync(c);
    out.resize((size_t)count * probs.size());
    for (size_t i = 0; i < probs.size(); ++i)
        std::memcpy(&out[i * count], c->host.as<char>() + w * probs[i], w);
}

}  // namespace

namespace {

// ------------------------------------------------------------- small sign
// s = sign(A) e_1 for the problems in probs (k x k each, A of problem b at
// A + b*a_stride with leading dimension lda; s written at s_out + b*s_stride)
// by the scaled Newton iteration (Eq. 11): determinantal scaling until the
// relative change drops below kNsSwitch (5e-2), then Newton-Schulz steps on the
// matrix cores while |X^2 - I|_F < 0.5; stop once the change is below 1e-14,
// or below 1e-8 and no longer halving; at most 100 iterations.  All problems
// of the group share every launch; each stops on its own.
// iters[b] > 0: iterations used, ok[b] = 1 on convergence; iters[b] < 0: a
// singular or non-finite iterate at iteration -iters[b].
// The small problem of Schur deflation (Eq. 15-19): the block matrix
// [[T, X], [0, H_k]] of size m + k.  T is shared; X (ld m), the coefficients
// c0 = S^dag b and the slot holding beta sit in each problem's arena block.
struct SchurBlock {
    int m = 0;
    const cd* T = nullptr;
    const cd* X = nullptr;
    const cd* c0 = nullptr;
    const cd* beta = nullptr;
    int64_t stride = 0;   // arena stride
};

// out = [[T, X], [0, H]] (n = m + k, ld n).  Batch strides: small (X, H), mat (out).
__global__ void k_schur_block(int m, int k, const cd* __restrict__ T, const cd* __restrict__ X,
                              const cd* __restrict__ H, int ldh, cd* __restrict__ out, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    X += pb * bt.small;
    H += pb * bt.small;
    out += pb * bt.mat;
    const int n = m + k;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e % n), j = (int)(e / n);
    cd v = mk(0.0, 0.0);
    if (j < m) {
        if (i < m) v = T[i + (int64_t)j * m];
    } else if (i < m) {
        v = X[i + (int64_t)(j - m) * m];
    } else {
        v = H[(i - m) + (int64_t)(j - m) * ldh];
    }
    out[e] = v;
}

// s = F [c0; beta e_1] for F = sign of the block matrix (n = m + k, ld n); the
// beta column only when k > 0.  Eq. 19 is then y = S s[0:m] + V_k s[m:n].
// Batch strides: mat (F), small (c0, s), scal (beta).
__global__ void k_schur_rhs(int m, int k, const cd* __restrict__ F, const cd* __restrict__ c0,
                            const cd* __restrict__ beta, cd* __restrict__ s, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    F += pb * bt.mat;
    c0 += pb * bt.small;
    s += pb * bt.small;
    beta += pb * bt.scal;
    const int n = m + k;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cd a = k > 0 ? cscale(F[i + (int64_t)m * n], beta->x) : mk(0.0, 0.0);
    for (int j = 0; j < m; ++j) a = cadd(a, cmul(F[i + (int64_t)j * n], c0[j]));
    s[i] = a;
}

// Delayed reorthogonalisation under Schur deflation: H was applied to the
// tentative column u_j = r v_j + V_{<j} s, so the projection left S^dag H u_j
// in column j of X; S^dag H v_j = (X_j - X_{<j} s) / r, with s = d[0:j] and
// 1/r in sc[0].  One block per (row i, problem): 256 threads split the j
// terms, then a fixed-order block reduction.  Batch strides: small (X, d),
// scal (sc).
__global__ __launch_bounds__(256) void k_schur_x_fix(int m, int j, cd* __restrict__ X,
                                                     const cd* __restrict__ d,
                                                     const cd* __restrict__ sc, Batch bt) {
    __shared__ double red[2][4];
    const int pb = bt.idx[blockIdx.y];
    const int i = blockIdx.x;
    X += pb * bt.small;
    d += pb * bt.small;
    sc += pb * bt.scal;
    double ax = 0.0, ay = 0.0;
    for (int l = threadIdx.x; l < j; l += 256) {
        const cd p = cmul(X[i + (int64_t)l * m], d[l]);
        ax += p.x;
        ay += p.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ax += __shfl_xor(ax, off, 64);
        ay += __shfl_xor(ay, off, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = ax;
        red[1][wave] = ay;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const cd acc = mk(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                          red[1][0] + red[1][1] + red[1][2] + red[1][3]);
        const cd a = csub(X[i + (int64_t)j * m], acc);
        X[i + (int64_t)j * m] = cscale(a, sc[0].x);
    }
}

// M <- M - I (n x n, ld n)
__global__ void k_sub_identity(cd* M, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) M[i + (int64_t)i * n].x -= 1.0;
}

// Newton change below which the small sign continues by Newton-Schulz steps
// (determinantal scaling stops there too)
constexpr double kNsSwitch = 5e-2;

// sign of the k x k matrices A (or, with sb, of the Schur block matrices of
// size m + k); s_out receives the first column (with sb: sign times [c0; beta e_1])
void small_sign_batch(osa_ctx* c, const std::vector<int>& probs, int k, const cd* A, int lda,
                      int64_t a_stride, cd* s_out, int64_t s_stride, std::vector<int>& iters,
                      std::vector<char>& ok, const SchurBlock* sb = nullptr) {
    const int n = sb ? sb->m + k : k;
    if (n > c->scap) throw OsaError{OSA_ERR_ARG, "small sign beyond its workspace"};
    const int64_t ms = (int64_t)c->scap * c->scap;
    cd* X = c->sX.as<cd>();
    cd* M = c->sM.as<cd>();
    cd* Y = c->sY.as<cd>();
    Batch bt;   // strides of the Newton workspace
    bt.basis = a_stride;
    bt.mat = ms;
    bt.small = c->scap;   // logpiv (doubles)
    bt.flag = 4;
    bt.ws = c->gj_stride;
    bt.part = c->red_stride;
    for (int b : probs) { iters[b] = 0; ok[b] = 0; }
    std::vector<int> act = probs;
    {
        Batch b0 = bt;
        b0.n = (int)act.size();
        for (int i = 0; i < b0.n; ++i) b0.idx[i] = (int16_t)act[i];
        if (sb) {
            Batch bb = b0;
            bb.small = sb->stride;
            if (b0.n > 0) {
                hipLaunchKernelGGL(k_schur_block, dim3((unsigned)ceil_div((int64_t)n * n, 256), b0.n),
                                   dim3(256), 0, c->st, sb->m, k, sb->T, sb->X, A, lda, X, bb);
                OSA_LAUNCH_CHECK();
            }
        } else {
            launch_copy_square(A, lda, X, k, c->st, b0);
        }
    }
    launch_fill_zero(c->nflag.p, c->nflag.bytes, c->st);   // a kernel, not a memset node
    uint64_t scale = ~0ULL;
    std::vector<double> prev(c->kbatch, INFINITY);
    // problems in the Newton-Schulz phase: X <- (3X - X^3)/2 by two GEMMs on the
    // FP64 matrix cores instead of an inverse, once the unscaled Newton change is
    // below kNsSwitch.  With X = S(1 + E) (every iterate is a function of H, so E
    // commutes with S) the error maps to E' = -(3/2)E^2 - E^3/2, quadratic as in
    // Newton's E^2/(2(1+E)).  A step that does not halve the change returns the
    // problem to Newton.  A problem whose X^2 - I was too large for the step
    // (nsblock = the change at that test) waits until its change has halved.
    std::vector<char> nsm(c->kbatch, 0);
    std::vector<double> nsblock(c->kbatch, INFINITY);
    double* red = c->red.as<double>();
    std::vector<double> hred, hns;
    std::vector<int> hflag;
    for (int it = 1; it <= 100 && !act.empty(); ++it) {
        Batch ba = bt;
        ba.n = (int)act.size();
        for (int i = 0; i < ba.n; ++i) ba.idx[i] = (int16_t)act[i];
        std::vector<int> gjl, nsc, nsl;
        for (int b : act) (nsm[b] ? nsc : gjl).push_back(b);
        if (!nsc.empty()) {
            // Newton-Schulz candidates: D = X X - I and |D|_F^2 (into red[0]) for all
            // of them in one launch, one read-back.  The step converges to sign(X)
            // when |I - X^2| < 1 (Frobenius norm here, with margin 0.5); otherwise an
            // eigenvalue of X may lie where (3x - x^3)/2 flips its sign, and the
            // problem takes a Newton step instead.
            Batch bn = batch_of(nsc);
            bn.mat = ms;
            bn.part = c->red_stride;
            bn.scal = c->red_stride;
            timed(c, 6, 2.0 * 16.0 * n * (double)n * bn.n, [&] {
                launch_zgemm_sq(n, mk(1.0, 0.0), X, X, 0.0, nullptr, -1.0, M, red + 2, red, c->st,
                                bn);
            }, 8.0 * n * (double)n * n * bn.n);
            d2h_strided(c, red, c->red_stride * (int64_t)sizeof(double), 1, nsc, hns);
            for (size_t i = 0; i < nsc.size(); ++i) {
                const int b = nsc[i];
                if (std::sqrt(hns[i]) < 0.5) {
                    nsl.push_back(b);
                } else {
                    nsm[b] = 0;
                    nsblock[b] = prev[b];
                    gjl.push_back(b);
                }
            }
            std::sort(gjl.begin(), gjl.end());
        }
        if (!gjl.empty()) {
            Batch bg = bt;
            bg.n = (int)gjl.size();
            for (int i = 0; i < bg.n; ++i) bg.idx[i] = (int16_t)gjl[i];
            Batch bc = bg;   // M <- X: X has leading dimension n
            bc.basis = ms;
            launch_copy_square(X, n, M, n, c->st, bc);
            timed(c, 3, 2.0 * 16.0 * n * (double)n * bg.n, [&] {
                gj_invert(M, Y, n, c->logpiv.as<double>(), c->nflag.as<int>(), c->gjws.p, c->st,
                          bg);
            });
        }
        if (!nsl.empty()) {
            // Y = X - X D = 2X - X (X X), so that the combine (X + Y)/2 is the
            // Newton-Schulz step (3X - X^3)/2
            Batch bs = batch_of(nsl);
            bs.mat = ms;
            timed(c, 6, 4.0 * 16.0 * n * (double)n * bs.n, [&] {
                launch_zgemm_sq(n, mk(-1.0, 0.0), X, M, 1.0, X, 0.0, Y, nullptr, nullptr, c->st,
                                bs);
            }, 8.0 * n * (double)n * n * bs.n);
        }
        launch_newton_combine(X, Y, n, c->logpiv.as<double>(), scale, red, c->st, ba);
        d2h_strided(c, red, c->red_stride * (int64_t)sizeof(double), 2, act, hred);
        d2h_strided(c, c->nflag.p, 4 * (int64_t)sizeof(int), 1, act, hflag);
        std::vector<int> next;
        if (c->prof_on) c->prof.counters[2] += (int64_t)act.size();
        for (size_t i = 0; i < act.size(); ++i) {
            const int b = act[i];
            const double d2 = hred[2 * i], n2 = hred[2 * i + 1];
            iters[b] = it;
            if (hflag[i] || !std::isfinite(d2) || !std::isfinite(n2)) { iters[b] = -it; continue; }
            const double change = std::sqrt(d2 / n2);
            if (change < kNsSwitch) scale &= ~(1ULL << b);
            if (nsm[b] && !(change < 0.5 * prev[b])) nsm[b] = 0;   // back to Newton
            else if (!nsm[b] && change < kNsSwitch && !((scale >> b) & 1ULL) &&
                     change < 0.5 * nsblock[b])
                nsm[b] = 1;
            // converged: at rounding level, stagnating below 1e-8, or below 1e-8 in
            // the quadratic regime (change <= 10 prev^2), where the new iterate's
            // error is about change^2 and one more step would only confirm it
            if (change < 1e-14 || (change < 1e-8 && change > 0.5 * prev[b]) ||
                (change < 1e-8 && change <= 10.0 * prev[b] * prev[b])) {
                ok[b] = 1;
                continue;
            }
            prev[b] = change;
            next.push_back(b);
        }
        act.swap(next);
    }
    std::vector<int> good;
    for (int b : probs)
        if (iters[b] > 0) good.push_back(b);
    Batch bs = bt;
    bs.n = (int)good.size();
    for (int i = 0; i < bs.n; ++i) bs.idx[i] = (int16_t)good[i];
    bs.small = s_stride;
    if (sb) {
        bs.scal = sb->stride;
        if (bs.n > 0) {
            hipLaunchKernelGGL(k_schur_rhs, dim3((unsigned)ceil_div(n, 256), bs.n), dim3(256), 0,
                               c->st, sb->m, k, X, sb->c0, sb->beta, s_out, bs);
            OSA_LAUNCH_CHECK();
        }
    } else {
        launch_copy_col0(X, k, s_out, c->st, bs);
    }
}

// ------------------------------------------------------------- set deflation
__global__ void k_sign_coef(int m, const cd* __restrict__ lam, const cd* __restrict__ cin,
                            cd* __restrict__ cout, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    cin += pb * bt.small;
    cout += pb * bt.small;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) cout[i] = cscale(cin[i], lam[i].x > 0 ? 1.0 : -1.0);
}

// Adjoint assembly.  With the deflation data of H (H R = R Lambda, G = L^dag R)
// the deflated part of sign(H)^dag x is (R sgn(Lambda) G^{-1} L^dag)^dag x =
// L G^{-H} sgn(Lambda) R^dag x: the signs act on R^dag x (raw) before G^{-H},
// so the order of the columns of L is free.  cout = G^{-H} (sgn(Re lambda) . raw),
// one block per problem.  Batch strides: small (raw, cout).
__global__ __launch_bounds__(64) void k_adj_sign_coef(int m, const cd* __restrict__ lam,
                                                      const cd* __restrict__ ginvh,
                                                      const cd* __restrict__ raw,
                                                      cd* __restrict__ cout, Batch bt) {
    const int pb = bt.idx[blockIdx.x];
    raw += pb * bt.small;
    cout += pb * bt.small;
    for (int i = threadIdx.x; i < m; i += 64) {
        cd a = mk(0.0, 0.0);
        for (int j = 0; j < m; ++j)
            cfma(a, ginvh[i + (int64_t)j * m], cscale(raw[j], lam[j].x > 0 ? 1.0 : -1.0));
        cout[i] = a;
    }
}

// |V_j|^2 for the m columns of V (length n each): one block per column, fixed order.
__global__ __launch_bounds__(256) void k_col_norm2(const cd* __restrict__ V, int64_t n,
                                                   double* __restrict__ out) {
    __shared__ double sm[4];
    V += (int64_t)blockIdx.x * n;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) a += cabs2(V[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
}

// Gn[i, j] = G[i, j] / (|l_i| |r_j|) from the squared column norms nl2, nr2
__global__ void k_normalize_g(int m, const cd* __restrict__ G, const double* __restrict__ nl2,
                              const double* __restrict__ nr2, cd* __restrict__ Gn) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * m) return;
    const int i = e % m, j = e / m;
    Gn[e] = cscale(G[e], 1.0 / std::sqrt(nl2[i] * nr2[j]));
}

// G = L^H R for the first m pairs, then G^{-1}.  The vectors may carry any
// scale (only the projector R G^{-1} L^dag matters), so the conditioning test
// runs on G with unit columns of L and R: it is then nearly diagonal with
// entries cos(angle(l_i, r_i)) when L and R span dual invariant subspaces, and a
// Gauss-Jordan pivot below 1e-10 means they do not.
void build_ginv(osa_ctx* c, int m) {
    ensure_krylov(c, std::max(c->kcap, std::max(m + 1, 8)));
    c->Ginv.ensure(sizeof(cd) * (size_t)m * m + 16);
    const TsPlan p = ts_plan(c->N());
    cd* G = c->sM.as<cd>();
    for (int j = 0; j < m; ++j) {
        const int nch = launch_dot_partial(c->L.p, c->N(), m, c->R.as<cd>() + (size_t)j * c->N(),
                                           false, p, c->partial.as<cd>(), c->st);
        launch_reduce_partial(c->partial.as<cd>(), nch, m, G + (size_t)j * m, nullptr,
                              nullptr, nullptr, c->st);
    }
    // normalised copy for the conditioning test (in sY, free outside the small sign)
    c->gnorm.ensure(sizeof(double) * 2 * (size_t)m);
    double* nrm = c->gnorm.as<double>();
    hipLaunchKernelGGL(k_col_norm2, dim3(m), dim3(256), 0, c->st, c->L.as<cd>(), c->N(), nrm);
    hipLaunchKernelGGL(k_col_norm2, dim3(m), dim3(256), 0, c->st, c->R.as<cd>(), c->N(), nrm + m);
    cd* Gn = c->sY.as<cd>();
    hipLaunchKernelGGL(k_normalize_g, dim3((unsigned)ceil_div((int64_t)m * m, 256)), dim3(256), 0,
                       c->st, m, (const cd*)G, (const double*)nrm, (const double*)(nrm + m), Gn);
    OSA_LAUNCH_CHECK();
    OSA_HIP(hipMemsetAsync(c->flag.p, 0, sizeof(int) * 4, c->st));
    gj_invert(G, c->Ginv.as<cd>(), m, c->logpiv.as<double>(), c->flag.as<int>(), c->gjws.p, c->st);
    int hf = 0;
    d2h(c, c->flag.p, 1, &hf);
    if (hf) throw OsaError{OSA_ERR_EIG_NOCONV, "G = L^dag R is singular"};
    // Gauss-Jordan of the normalised G (its inverse goes to sX, unused)
    gj_invert(Gn, c->sX.as<cd>(), m, c->logpiv.as<double>(), c->flag.as<int>(), c->gjws.p, c->st);
    std::vector<double> lp(m);
    d2h(c, c->logpiv.p, (size_t)m, lp.data());
    d2h(c, c->flag.p, 1, &hf);
    double mn = INFINITY;
    for (double v : lp) mn = std::min(mn, v);
    if (hf || !(mn > std::log(1e-10)))
        throw OsaError{OSA_ERR_EIG_NOCONV,
                       "G = L^dag R is nearly singular: the left and right vectors do not span "
                       "dual invariant subspaces"};
}

void set_active(osa_ctx* c, int m) {
    c->m_active = m;
    if (m > 0 && c->have_left) build_ginv(c, m);
}

// Schur basis of the active deflation space (Eq. 13): classical Gram-Schmidt,
// applied twice, over the right eigenvectors in their order gives R = S U with
// U upper triangular, so T = S^dag H S = U Lambda U^{-1} is upper triangular
// (to the accuracy of the eigenvectors) with the eigenvalues on its diagonal.
void ensure_schur(osa_ctx* c) {
    const int m = c->m_active;
    if (m == 0 || c->schur_m == m) return;
    if ((int64_t)(c->kcap + 2) * c->kbatch < m) throw OsaError{OSA_ERR_ARG, "basis storage"};
    const int64_t N = c->N();
    const TsPlan p = ts_plan(N);
    c->Sch.ensure(sizeof(cd) * (size_t)N * m);
    c->Tsch.ensure(sizeof(cd) * (size_t)m * m + 16);
    cd* S = c->Sch.as<cd>();
    cd* w = c->w.as<cd>();
    for (int j = 0; j < m; ++j) {
        OSA_HIP(hipMemcpyAsync(w, c->R.as<cd>() + (size_t)j * N, sizeof(cd) * N,
                               hipMemcpyDeviceToDevice, c->st));
        if (j > 0)
            cgs2(c, w, S, N, j, false, c->coef.as<cd>(), c->coef2.as<cd>());
        else
            launch_norm_partial(w, false, p, c->normp.as<double>(), c->st);
        launch_normalize(w, S + (size_t)j * N, false, p, c->normp.as<double>(), c->dscal.as<cd>(),
                         nullptr, 0.0, nullptr, 0, nullptr, 0, c->st);
    }
    // T = S^dag (H S), H S in the Krylov basis storage (free between solves)
    cd* W = c->V.as<cd>();
    apply_h_contig(c, S, W, false, false, m);
    for (int j = 0; j < m; ++j) {
        const int nch = launch_dot_partial(S, N, m, W + (size_t)j * N, false, p,
                                           c->partial.as<cd>(), c->st);
        launch_reduce_partial(c->partial.as<cd>(), nch, m, c->Tsch.as<cd>() + (size_t)j * m,
                              nullptr, nullptr, nullptr, c->st);
    }
    c->schur_m = m;
}

// The deflation data has to fit the scheme of the solve: LR deflation and the
// adjoint need left vectors, and Schur deflation has no adjoint form here.
void check_deflation_state(osa_ctx* c) {
    if (c->m_active == 0) return;
    if (c->opts.deflation == 1 && c->adj)
        throw OsaError{OSA_ERR_STATE, "the adjoint solve needs LR deflation (deflation = 0)"};
    if (c->opts.deflation != 1 && !c->have_left)
        throw OsaError{OSA_ERR_STATE, "LR deflation needs left eigenvectors; this deflation "
                                      "data has none (computed for Schur deflation)"};
}

// ------------------------------------------------------------- solve
// Per-step rate rho of an error e_k = C rho^k from two successive checkpoint
// changes: est1 over a span of d1 steps, then est2 over the next d2 steps.
// With e_k geometric, est ~ e_{k-d} - e_k, so est2 / est1 =
// rho^d1 (1 - rho^d2) / (1 - rho^d1), increasing in rho from 0 to d2/d1;
// solved by bisection.  1 when the changes do not contract.
double geometric_rate(double est1, int d1, double est2, int d2) {
    if (!(est1 > 0) || !(est2 >= 0) || d1 <= 0 || d2 <= 0) return 1.0;
    if (est2 == 0) return 0.0;
    const double R = est2 / est1;
    if (!(R < 0.999 * (double)d2 / (double)d1)) return 1.0;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 80; ++it) {
        const double r = 0.5 * (lo + hi);
        const double f = std::pow(r, d1) * (1.0 - std::pow(r, d2)) / (1.0 - std::pow(r, d1));
        (f < R ? lo : hi) = r;
    }
    return hi;
}

struct SolveResult {
    osa_status st = OSA_OK;
    int k_used = 0;
    double est = NAN;
    int newton_iters = 0;
    int breakdown = 0;
    double bnorm = 0;
};

// Steps j0..j1 of a solve for the active problems act, as one HIP graph.  A
// segment's launches depend only on (j0, j1, the active set, m and the solve
// flags) and on the workspace pointers, so the graph recorded the second time a
// segment is seen (the first run tunes the dot kernels, so the graph records
// the tuned launches) is replayed every later time: one graph launch instead of
// about ten kernel launches per step, with results bitwise those of direct
// launches.  Recording runs on a private stream (capture cannot use the legacy
// default stream) and the graph is launched on the context's stream.  Any
// workspace (re)allocation invalidates every recorded graph.  Off while kernel
// timing is on (events would be recorded into the graph) or with
// opts.no_graphs; a segment whose capture fails runs directly from then on.
template <typename F>
void run_segment(osa_ctx* c, int j0, int j1, const std::vector<int>& act, int flags, F&& step) {
    const bool use = !c->opts.no_graphs && !c->prof_on && act.size() <= 64;
    if (!use) {
        for (int j = j0; j <= j1; ++j) step(j);
        return;
    }
    const uint64_t ep = g_alloc_epoch.load();
    if (ep != c->seg_epoch) {
        c->clear_graphs();
        c->seg_epoch = ep;
    }
    if (c->seg_graphs.size() > 512) c->clear_graphs();
    uint64_t mask = 0;
    for (int b : act) mask |= 1ULL << b;
    osa_ctx::SegGraph& g = c->seg_graphs[osa_ctx::SegKey{j0, j1, c->m_active, flags, mask}];
    if (g.exec) {
        OSA_HIP(hipGraphLaunch(g.exec, c->st));
        ++c->graph_launches;
        return;
    }
    if (g.failed || g.seen++ == 0) {
        for (int j = j0; j <= j1; ++j) step(j);
        return;
    }
    if (!c->cap_st) OSA_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
    hipStream_t own = c->st;
    hipGraph_t graph = nullptr;
    c->st = c->cap_st;
    bool ok = hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        try {
            for (int j = j0; j <= j1; ++j) step(j);
        } catch (...) {
            ok = false;
        }
        if (hipStreamEndCapture(c->cap_st, &graph) != hipSuccess) ok = false;
    }
    c->st = own;
    if (ok && graph && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        g.exec = nullptr;
        ok = false;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok || !g.exec) {
        g.failed = true;   // run this segment directly from now on
        for (int j = j0; j <= j1; ++j) step(j);
        return;
    }
    ++c->graph_captures;
    OSA_HIP(hipGraphLaunch(g.exec, c->st));
    ++c->graph_launches;
}

// y_b = sign(H) x_b for nb internal-layout sources (contiguous, N apart) in
// lockstep: every Arnoldi step applies the stencil, the re-projection, both
// Gram-Schmidt passes and the normalisation to all unfinished sources in one
// launch each; each source keeps its own basis, Hessenberg matrix, check
// history and stopping point, so its result is that of a single-source solve.
void solve_batch(osa_ctx* c, int nb, const cd* xin, cd* yout, double tol,
                 std::vector<SolveResult>& res) {
    res.assign(nb, SolveResult{});
    const int64_t N = c->N();
    const int kmax = c->opts.k_max;
    check_deflation_state(c);
    const bool schur = c->opts.deflation == 1 && c->m_active > 0;   // Eq. 13-19
    // the Schur basis set-up uses m columns of the basis storage as scratch
    // the two-step form keeps up to three columns beyond the Krylov size
    ensure_krylov(c, schur ? std::max(kmax, c->m_active) : (c->opts.orth == 2 ? kmax + 2 : kmax),
                  nb);
    if (c->lay.vec_len < kmax + c->m_alloc + 2 || c->lay.m < c->m_alloc) {
        c->lay = ArenaLayout::make(c->kcap, std::max(c->m_alloc, 1));
        c->arena.ensure(sizeof(cd) * (size_t)c->lay.stride * c->kbatch);
    }
    if (schur) ensure_schur(c);
    const ArenaLayout& L = c->lay;
    const bool fixed = c->opts.check_every < 0;
    const int every = fixed ? kmax : std::max(1, c->opts.check_every);
    // Schur deflation keeps the S coefficients of every H v_j (the block X of
    // Eq. 15), so it projects at every step
    const bool reproj = !c->opts.no_reproject || schur;
    const TsPlan p = ts_plan(N);
    const int64_t VS = (int64_t)(c->kcap + 2) * N;   // basis stride
    // orth 2: two-step blocks (one dot and one update pass per two Arnoldi
    // steps), with LR deflation or none.  Outer step n completes the
    // decomposition of size n + 1, so the checks (at the multiples of
    // check_every and at kmax) can take size n + 1 or n.  Schur deflation takes
    // the delayed one-step form instead.
    const bool blk2 = c->opts.orth == 2 && !schur;
    const bool dcgs = c->opts.orth == 0 || (c->opts.orth == 2 && !blk2);   // delayed reorth.
    const int ldh = L.ldh;
    cd* V = c->V.as<cd>();
    cd* ar = c->arena.as<cd>();
    cd* H = ar + L.H;
    // ds: [0] |b|, [1] beta, [2] |y|, [3] |s - s'| (double), [4] hfro2 (double),
    //     [5] 1/r and [6] c_j of the delayed reorthogonalisation
    cd* ds = ar + L.ds;
    double* hfro2 = (double*)(ds + 4);
    cd* w = c->w.as<cd>();
    cd* x = c->x.as<cd>();
    int* flag = c->flag.as<int>();
    const int m = c->m_active;
    SchurBlock sblk;
    sblk.m = m;
    sblk.T = c->Tsch.as<cd>();
    sblk.X = ar + L.xs;
    sblk.c0 = ar + L.cdef;
    sblk.beta = ds + 1;
    sblk.stride = L.stride;
    const SchurBlock* sbp = schur ? &sblk : nullptr;
    const int ms0 = schur ? m : 0;   // leading S part of the small solution vector
    Batch base;   // strides of the solve workspace
    base.basis = VS;
    base.vec = N;
    base.small = L.stride;
    base.scal = L.stride;
    base.flag = 4;
    base.part = c->normp_stride;
    auto bat = [&](const std::vector<int>& probs) {
        Batch bt = base;
        bt.n = (int)probs.size();
        for (int i = 0; i < bt.n; ++i) bt.idx[i] = (int16_t)probs[i];
        return bt;
    };
    std::vector<int> all(nb);
    for (int b = 0; b < nb; ++b) all[b] = b;
    const Batch ball = bat(all);

    OSA_HIP(hipMemcpyAsync(x, xin, sizeof(cd) * N * nb, hipMemcpyDeviceToDevice, c->st));
    OSA_HIP(hipMemsetAsync(ar, 0, sizeof(cd) * (size_t)L.stride * nb, c->st));
    OSA_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4 * nb, c->st));
    launch_norm_partial(x, false, p, c->normp.as<double>(), c->st, ball);
    launch_normalize(x, nullptr, false, p, c->normp.as<double>(), ds + 0, nullptr, 0.0, nullptr, 0,
                     nullptr, 0, c->st, ball);
    // x <- x_ominus (Eq. 21); craw keeps L^dag b (R^dag b in the adjoint) for the assembly
    if (m > 0) project_out(c, x, ar + L.cdef, ar + L.craw, ball);
    launch_norm_partial(x, false, p, c->normp.as<double>(), c->st, ball);
    launch_normalize(x, nullptr, false, p, c->normp.as<double>(), ds + 1, nullptr, 0.0, nullptr, 0,
                     nullptr, 0, c->st, ball);
    std::vector<cd> hb;
    d2h_strided(c, ds, L.stride * (int64_t)sizeof(cd), 2, all, hb);
    std::vector<double> beta(nb), bnorm(nb);
    std::vector<int> act;
    std::vector<char> done(nb, 0);
    for (int b = 0; b < nb; ++b) {
        bnorm[b] = hb[2 * b].x;
        beta[b] = hb[2 * b + 1].x;
        res[b].bnorm = bnorm[b];
        if (!std::isfinite(bnorm[b]) || !std::isfinite(beta[b])) {
            res[b].st = OSA_ERR_NONFINITE;
            done[b] = 1;
        } else if (beta[b] > 1e-15 * bnorm[b] && beta[b] > 0) {
            act.push_back(b);
        }
    }
    const int64_t scratch_len = (int64_t)(c->upd_scratch.bytes / sizeof(cd));
    if (!act.empty()) {
        Batch b0 = bat(act);
        launch_scale_dev(x, V, false, N, ds + 1, true, c->st, b0);   // v_1 = x_ominus / beta
        if (dcgs) {
            // first column: one pass; u_1 = H v_1 - v_1 h_11 goes to basis column 1
            apply_h(c, V, w, false, c->adj, b0);
            if (reproj && m > 0) project_out(c, w, schur ? ar + L.xs : ar + L.coef2, ar + L.tmp, b0);
            Batch bd = b0, bu = b0;
            bd.part = c->part_stride;
            bu.part = 0;
            int nch = 0;
            timed(c, 0, 2.0 * N * 16.0 * b0.n, [&] {
                nch = launch_dot_partial(V, N, 1, w, false, p, c->partial.as<cd>(), c->st, bd);
            });
            launch_reduce_partial(c->partial.as<cd>(), nch, 1, H, nullptr, nullptr, nullptr, c->st,
                                  bd);
            timed(c, 1, 3.0 * N * 16.0 * b0.n, [&] {
                launch_update(w, V, N, 1, H, false, p, nullptr, nullptr, 0, c->st, bu);
            });
            OSA_HIP(hipMemcpy2DAsync(V + N, sizeof(cd) * VS, w, sizeof(cd) * N, sizeof(cd) * N, nb,
                                     hipMemcpyDeviceToDevice, c->st));
        } else if (blk2) {
            // first two-step block: W = [H v_1, H^2 v_1] in columns 1, 2, one pass
            // against v_1 (U = W - v_1 v_1^H W)
            Batch bv = b0;
            bv.vec = VS;   // the stencil writes into the basis
            apply_h(c, V, V + N, false, c->adj, bv);
            apply_h(c, V + N, V + 2 * N, false, c->adj, bv);
            if (reproj && m > 0) project_out(c, V + N, ar + L.coef2, ar + L.tmp, bv, 2, N);
            Batch bd = bv;
            bd.part = c->part_stride;
            int nch = 0;
            timed(c, 0, 3.0 * N * 16.0 * b0.n, [&] {
                nch = launch_dot2_partial(V, N, 1, V + N, V + 2 * N, false, p, c->partial.as<cd>(),
                                          c->st, bd);
            });
            launch_reduce_partial(c->partial.as<cd>(), nch, 2, ar + L.dc, nullptr, nullptr, nullptr,
                                  c->st, bd);
            launch_blk2_init(ar + L.b2, (int)L.vec_len, ar + L.dc, c->st, b0);
            timed(c, 1, 5.0 * N * 16.0 * b0.n, [&] {
                launch_blk_update(V, N, 3, ar + L.b2 + 4 * L.vec_len, (int)L.vec_len, 1, 2, N,
                                  c->st, b0);
            });
        }
    }
    std::vector<int> kprev(nb, 0);
    // Convergence estimate and check schedule (the paper gives no stopping rule).
    // The change est = beta |s_k - [s_k'; 0]| / |b| since the previous check k'
    // is about the error of check k'.  stop_rule 0 (default): once two changes
    // are known, their ratio gives the per-step rate rho of a geometric error
    // (the slower of the last two rates is used), and the error of the current
    // iterate is estimated by twice the geometric tail est rho^d / (1 - rho^d),
    // d = k - k';
    // the solve stops when that is <= tol (with only one change: when the
    // change is).  stop_rule 1: stop when the change itself is <= tol, i.e. when
    // the previous check was accurate enough.  The rate also predicts where the
    // estimate crosses tol; checks far before that point are skipped (at most 3
    // in a row).
    const bool tail_rule = c->opts.stop_rule == 0;
    std::vector<std::vector<int>> cj(nb);       // performed checks
    std::vector<std::vector<double>> ce(nb);    // ce[i]: change at check i (error of check i-1)
    std::vector<std::vector<double>> crate(nb); // per-step rates from consecutive changes
    std::vector<double> ctail(nb, INFINITY);    // estimated error at the last check
    std::vector<int> hf;
    std::vector<double> hd;
    // Step j: plain CGS2 extends the decomposition to size j + 1; the delayed
    // form (steps 1 .. kmax) completes size j and starts column j.
    // One Arnoldi step j for the problems of bt (no host synchronisation inside).
    auto do_step = [&](int j, const Batch& bt) {
        apply_h(c, V + (size_t)j * N, w, false, c->adj, bt);
        if (reproj && m > 0)   // Schur deflation: column j of X = S^dag H v_j
            project_out(c, w, schur ? ar + L.xs + (size_t)j * m : ar + L.coef2, ar + L.tmp, bt);
        if (dcgs) {
            Batch bd = bt;
            bd.part = c->part_stride;
            int nch = 0;
            timed(c, 0, (j + 3.0) * N * 16.0 * bt.n, [&] {
                nch = launch_dot2_partial(V, N, j + 1, V + (size_t)j * N, w, false, p,
                                          c->partial.as<cd>(), c->st, bd);
            });
            launch_reduce_partial(c->partial.as<cd>(), nch, 2 * (j + 1), ar + L.dc, nullptr,
                                  nullptr, nullptr, c->st, bd);
            launch_dcgs_coef(j, H, ldh, ar + L.dc, ds + 5, hfro2, flag, 1e-14, c->st, bt);
            if (schur) {
                hipLaunchKernelGGL(k_schur_x_fix, dim3((unsigned)m, (unsigned)bt.n), dim3(256), 0,
                                   c->st, m, j, ar + L.xs, (const cd*)(ar + L.dc),
                                   (const cd*)(ds + 5), bt);
                OSA_LAUNCH_CHECK();
            }
            timed(c, 1, (j + 4.0) * N * 16.0 * bt.n, [&] {
                launch_dcgs_update(V, N, j, w, ar + L.dc, ds + 5, false, N,
                                   c->upd_scratch.as<cd>(), scratch_len, c->st, bt);
            });
        } else {
            cgs2(c, w, V, N, j + 1, false, H + (size_t)j * ldh, ar + L.coef, bt);
            launch_normalize(w, V + (size_t)(j + 1) * N, false, p, c->normp.as<double>(),
                             H + (size_t)j * ldh + (j + 1), hfro2, 1e-14, flag, j,
                             H + (size_t)j * ldh, j + 1, c->st, bt);
        }
    };
    // Two-step block, outer step n (odd): the stencil twice on u_b (column n+1)
    // into columns n+2, n+3, one dot pass of columns 0..n+1 with columns n..n+3,
    // the coefficients, one update pass forming columns n..n+3; completes size
    // n + 1 (column n+1 of H stays pending).  The re-projection takes both new
    // columns in one pass over L and R, after the second stencil application:
    // H^2 u_b is formed from the unprojected H u_b, and H commutes with the
    // projector up to the deflated pairs' residual, so this differs from
    // projecting after each application by that residual times the
    // rounding-level component along the deflated directions.
    auto do_step2 = [&](int n, const Batch& bt) {
        Batch bv = bt;
        bv.vec = VS;
        cd* Vn = V + (size_t)n * N;
        apply_h(c, Vn + N, Vn + 2 * N, false, c->adj, bv);
        apply_h(c, Vn + 2 * N, Vn + 3 * N, false, c->adj, bv);
        if (reproj && m > 0) project_out(c, Vn + 2 * N, ar + L.coef2, ar + L.tmp, bv, 2, N);
        Batch bd = bt;
        bd.part = c->part_stride;
        int nch = 0;
        timed(c, 0, (n + 4.0) * N * 16.0 * bt.n, [&] {
            nch = launch_dot4_partial(V, N, n + 2, Vn, N, p, c->partial.as<cd>(), c->st, bd);
        });
        launch_reduce_partial(c->partial.as<cd>(), nch, 4 * (n + 2), ar + L.b2, nullptr, nullptr,
                              nullptr, c->st, bd);
        launch_blk2_coef(n, H, ldh, ar + L.b2, (int)L.vec_len, hfro2, flag, 1e-14, c->st, bt);
        timed(c, 1, (n + 8.0) * N * 16.0 * bt.n, [&] {
            launch_blk_update(V, N, n + 4, ar + L.b2 + 4 * L.vec_len, (int)L.vec_len, n, 4, N,
                              c->st, bt);
        });
    };
    // step index j: the Krylov size it completes; check_size(j) is the size of a
    // check after step j, 0 if none.  A two-step unit j (outer step n = 2j + 1,
    // up to n = kmax) completes size 2j + 2 and can check at 2j + 2 or 2j + 1.
    auto size_of = [&](int j) { return blk2 ? 2 * j + 2 : (dcgs ? j : j + 1); };
    const int jbeg = dcgs ? 1 : 0;
    const int jend = blk2 ? (kmax + 1) / 2 : (dcgs ? kmax + 1 : kmax);
    auto on_grid = [&](int kk) { return kk >= 1 && kk <= kmax && (kk % every == 0 || kk == kmax); };
    auto check_size = [&](int j) {
        const int kk = size_of(j);
        if (on_grid(kk)) return kk;
        if (blk2 && on_grid(kk - 1)) return kk - 1;
        return 0;
    };
    auto is_check = [&](int j) { return check_size(j) > 0; };
    for (int j = jbeg; j < jend && !act.empty(); ++j) {
        // the segment [j, je]: the steps up to and including the next check
        int je = j;
        while (je + 1 < jend && !is_check(je)) ++je;
        run_segment(c, j, je, act, (schur ? 1 : 0) | (reproj ? 2 : 0) | (dcgs ? 4 : 0) |
                                       (c->adj ? 8 : 0) | (fixed ? 16 : 0) | (blk2 ? 32 : 0),
                    [&](int jj) {
                        if (blk2) do_step2(2 * jj + 1, bat(act));
                        else do_step(jj, bat(act));
                    });
        j = je;
        const int kk = check_size(j) > 0 ? check_size(j) : size_of(j);
        if (!is_check(j)) continue;
        // each source follows its own schedule, as it would alone
        std::vector<int> chk, wait;
        for (int b : act) {
            bool want = true;
            if (!fixed && kk != kmax && !crate[b].empty()) {
                const double rho = crate[b].back();
                const double pred = ctail[b] * std::pow(rho, (double)(kk - cj[b].back()));
                const bool near = !(rho < 1.0) || !(pred > 3.0 * tol);
                if (!near && kk - cj[b].back() < 4 * every) want = false;
            }
            (want ? chk : wait).push_back(b);
        }
        if (chk.empty()) continue;
        d2h_strided(c, flag, 4 * (int64_t)sizeof(int), 2, chk, hf);
        // group the sources by the Krylov size of this check
        std::vector<int> kcheck(nb, kk), live;
        for (size_t i = 0; i < chk.size(); ++i) {
            const int b = chk[i];
            if (hf[2 * i] == 2) { res[b].st = OSA_ERR_NONFINITE; done[b] = 1; continue; }
            if (hf[2 * i] == 1) {   // happy breakdown at step hf[1]: K is invariant, result exact
                kcheck[b] = std::min(kk, hf[2 * i + 1] + 1);
                res[b].breakdown = 1;
            }
            live.push_back(b);
        }
        std::vector<int> iters(nb, 0);
        std::vector<char> okv(nb, 0);
        std::vector<int> ks;
        for (int b : live)
            if (std::find(ks.begin(), ks.end(), kcheck[b]) == ks.end()) ks.push_back(kcheck[b]);
        std::vector<int> next;
        for (int kc : ks) {
            std::vector<int> grp;
            for (int b : live)
                if (kcheck[b] == kc) grp.push_back(b);
            small_sign_batch(c, grp, kc, H, ldh, L.stride, ar + L.s_cur, L.stride, iters, okv,
                             sbp);
            std::vector<int> good, withprev;
            for (int b : grp) {
                res[b].newton_iters = iters[b];
                if (iters[b] < 0 || !okv[b]) {
                    res[b].st = OSA_ERR_NEWTON_NOCONV;
                    done[b] = 1;
                    continue;
                }
                res[b].k_used = kc;
                good.push_back(b);
                if (kprev[b] > 0 && !fixed) withprev.push_back(b);
            }
            // est = beta |s - [s_prev; 0]| / |b|, per previous check size
            while (!withprev.empty()) {
                const int kp = kprev[withprev[0]];
                std::vector<int> sub, rest;
                for (int b : withprev) (kprev[b] == kp ? sub : rest).push_back(b);
                Batch bd = bat(sub);
                bd.scal = 2 * L.stride;   // counted in doubles
                launch_diff_norm(ar + L.s_cur, kc + ms0, ar + L.s_prev, kp + ms0, (double*)(ds + 3),
                                 c->st, bd);
                d2h_strided(c, (double*)(ds + 3), L.stride * (int64_t)sizeof(cd), 1, sub, hd);
                for (size_t i = 0; i < sub.size(); ++i) {
                    const int b = sub[i];
                    // s carries beta under Schur deflation (s = sign(H) [c0; beta e_1])
                    res[b].est = (schur ? 1.0 : beta[b]) * hd[i] / bnorm[b];
                }
                withprev.swap(rest);
            }
            std::vector<int> cont;
            for (int b : good) {
                bool stop = res[b].breakdown != 0;
                if (kprev[b] > 0 && !fixed) {
                    const double change = res[b].est;
                    double tail = change;
                    if (ce[b].size() >= 2 && std::isfinite(ce[b].back())) {
                        const int d1 = cj[b].back() - cj[b][cj[b].size() - 2];
                        const int d2 = kc - cj[b].back();
                        const double rho = geometric_rate(ce[b].back(), d1, change, d2);
                        const double rho_use = crate[b].empty() ? rho
                                                                : std::max(rho, crate[b].back());
                        crate[b].push_back(rho);
                        if (tail_rule) {
                            const double q = std::pow(rho_use, (double)d2);
                            // factor 2: margin for a rate that drifts between checks
                            tail = q < 1.0 ? 2.0 * change * q / (1.0 - q) : INFINITY;
                        }
                    }
                    if (tail_rule) res[b].est = tail;
                    ctail[b] = tail;
                    if (res[b].est <= tol) stop = true;
                    ce[b].push_back(change);
                } else {
                    ce[b].push_back(NAN);
                }
                cj[b].push_back(kc);
                if (res[b].breakdown) res[b].est = 0.0;
                if (stop) { done[b] = 1; continue; }
                kprev[b] = kc;
                cont.push_back(b);
            }
            if (!cont.empty()) {   // keep the latest sign in s_prev for the next difference
                Batch bcp = bat(cont);
                bcp.mat = L.stride;
                launch_copy_col0(ar + L.s_cur, kc + ms0, ar + L.s_prev, c->st, bcp);
            }
            next.insert(next.end(), cont.begin(), cont.end());
        }
        next.insert(next.end(), wait.begin(), wait.end());
        std::sort(next.begin(), next.end());
        act.swap(next);
    }
    // assembly (Eq. 22): y = R sgn(Re lambda) c + beta V_k s
    std::vector<int> okp;
    for (int b = 0; b < nb; ++b)
        if (res[b].st >= 0) okp.push_back(b);
    if (schur) {
        // Eq. 19: y = S s[0:m] + V_k s[m:m+k] with s = sign(H) [c0; beta e_1];
        // a source inside Omega_m (no Krylov step) needs sign(T) c0 only
        std::vector<int> z, it0(nb, 0);
        std::vector<char> ok0(nb, 0);
        for (int b : okp)
            if (res[b].k_used == 0) z.push_back(b);
        if (!z.empty()) {
            small_sign_batch(c, z, 0, H, ldh, L.stride, ar + L.s_cur, L.stride, it0, ok0, sbp);
            for (int b : z) {
                res[b].newton_iters = it0[b];
                if (it0[b] < 0 || !ok0[b]) res[b].st = OSA_ERR_NEWTON_NOCONV;
            }
        }
        std::vector<int> ks;
        for (int b : okp)
            if (res[b].st >= 0 && std::find(ks.begin(), ks.end(), res[b].k_used) == ks.end())
                ks.push_back(res[b].k_used);
        for (int ku : ks) {
            std::vector<int> grp;
            for (int b : okp)
                if (res[b].st >= 0 && res[b].k_used == ku) grp.push_back(b);
            const Batch bg = bat(grp);
            Batch bs = bg;
            bs.basis = 0;   // S is shared
            launch_combine(yout, c->Sch.p, N, m, ar + L.s_cur, false, false, N, c->st, bs);
            if (ku > 0) launch_combine(yout, V, N, ku, ar + L.s_cur + m, false, true, N, c->st, bg);
        }
    } else if (!okp.empty()) {
        const Batch bo = bat(okp);
        if (m > 0) {
            if (c->adj)
                hipLaunchKernelGGL(k_adj_sign_coef, dim3(bo.n), dim3(64), 0, c->st, m,
                                   (const cd*)c->lam_dev.p, (const cd*)c->GinvH.p,
                                   (const cd*)(ar + L.craw), ar + L.coef, bo);
            else
                hipLaunchKernelGGL(k_sign_coef, dim3((unsigned)ceil_div(m, 64), bo.n), dim3(64), 0,
                                   c->st, m, (const cd*)c->lam_dev.p, (const cd*)(ar + L.cdef),
                                   ar + L.coef, bo);
            OSA_LAUNCH_CHECK();
            Batch br = bo;
            br.basis = 0;   // R is shared
            launch_combine(yout, c->adj ? c->L.p : c->R.p, N, m, ar + L.coef, false, false, N,
                           c->st, br);
        } else {
            OSA_HIP(hipMemsetAsync(yout, 0, sizeof(cd) * N * nb, c->st));
        }
        std::vector<int> ks;
        for (int b : okp)
            if (res[b].k_used > 0 && std::find(ks.begin(), ks.end(), res[b].k_used) == ks.end())
                ks.push_back(res[b].k_used);
        for (int ku : ks) {
            std::vector<int> grp;
            for (int b : okp)
                if (res[b].k_used == ku) grp.push_back(b);
            Batch bg = bat(grp);
            Batch bsc = bg;   // coef = beta * s  (s read as the "vector", coef as the "basis")
            bsc.vec = L.stride;
            bsc.basis = L.stride;
            launch_scale_dev(ar + L.s_cur, ar + L.coef, false, ku, ds + 1, false, c->st, bsc);
            launch_combine(yout, V, N, ku, ar + L.coef, false, true, N, c->st, bg);
        }
    }
    for (int b = 0; b < nb; ++b) {
        SolveResult& r = res[b];
        if (r.st < 0) continue;
        if (fixed) r.est = NAN;
        if (r.k_used == 0) r.est = 0.0;
        if (!fixed && !(r.est <= tol)) r.st = OSA_NOT_CONVERGED;
    }
    sync(c);
}

// ================================================================ eigensolver
// Krylov-Schur (Stewart) with locking for the nev eigenvalues of A = H^2 of
// smallest modulus, A = H(mu)^2 (right) or H(-mu)^2 (left).  The basis is
// [V_L | V_A | v]: V_L holds locked Schur vectors of converged eigenvalues,
// V_A the active block (at most pa <= 64 vectors), v the next Arnoldi vector,
// with A V_A = V_L C + V_A S_A + v b^H.  Each restart takes the Schur form of
// the active Rayleigh quotient S_A (smallest |theta| first), locks the leading
// converged Schur vectors and keeps a few more.  Because span(V_L) is
// invariant, S_A projects the remaining (block-triangular) part of A, so the
// locked coupling C never enters the small problem.  Output: an orthonormal
// basis X (nev vectors, fp64 internal layout) of the wanted invariant subspace.
// An fp32 search is followed by an fp64 run started from the fp32 subspace.
struct KsStats {
    int64_t matvecs = 0;
    int restarts = 0;
    bool converged = false;
};

// Arnoldi expansion of a Krylov-Schur basis from column kcur (a complete,
// normalised vector) to ptot columns, with A = H^2 and the second Gram-Schmidt
// pass delayed by one step (as in the solve): a single pass for column kcur,
// delayed steps for kcur+1 .. ptot-1, then a last reorthogonalisation that
// completes column ptot-1 and the normalised next vector v_ptot without a
// further product with A.  The Rayleigh quotient S is general (triangular kept
// block, spike row), so the first-pass correction uses all of it.
void expand_delayed(osa_ctx* c, bool adjoint, bool fp32, char* V, int64_t N, cd* S, int ldS,
                    int kcur, int ptot, void* wv, void* tv, cd* d, double* hfro2, int* flag,
                    KsStats& stats) {
    const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
    auto vec = [&](int j) { return V + es * (size_t)N * j; };
    const TsPlan pl = ts_plan(N);
    const int64_t scratch_len = (int64_t)(c->upd_scratch.bytes / sizeof(cd));
    cd* part = c->partial.as<cd>();
    cd* sc = c->dscal.as<cd>() + 10;   // [1/r, c_j]
    const double eb = fp32 ? 8.0 : 16.0;
    auto matvec = [&](int j) {
        apply_h(c, vec(j), tv, fp32, adjoint);
        apply_h(c, tv, wv, fp32, adjoint);
        stats.matvecs += 2;
        c->prof.counters[3] += c->prof_on ? 1 : 0;
    };
    // column kcur: one pass; u_{kcur+1} -> basis column kcur + 1
    matvec(kcur);
    {
        cd* scol = S + (size_t)kcur * ldS;
        int nch = 0;
        timed(c, 0, (kcur + 2.0) * N * eb, [&] {
            nch = launch_dot_partial(V, N, kcur + 1, wv, fp32, pl, part, c->st);
        });
        launch_reduce_partial(part, nch, kcur + 1, scol, nullptr, nullptr, nullptr, c->st);
        timed(c, 1, (kcur + 3.0) * N * eb, [&] {
            launch_update(wv, V, N, kcur + 1, scol, fp32, pl, nullptr, nullptr, 0, c->st);
        });
        OSA_HIP(hipMemcpyAsync(vec(kcur + 1), wv, es * (size_t)N, hipMemcpyDeviceToDevice,
                               c->st));
    }
    for (int j = kcur + 1; j < ptot; ++j) {
        matvec(j);
        int nch = 0;
        timed(c, 0, (j + 3.0) * N * eb, [&] {
            nch = launch_dot2_partial(V, N, j + 1, vec(j), wv, fp32, pl, part, c->st);
        });
        launch_reduce_partial(part, nch, 2 * (j + 1), d, nullptr, nullptr, nullptr, c->st);
        launch_dcgs_coef(j, S, ldS, d, sc, hfro2, flag, 1e-300, c->st, Batch(), false, true);
        timed(c, 1, (j + 4.0) * N * eb, [&] {
            launch_dcgs_update(V, N, j, wv, d, sc, fp32, N, c->upd_scratch.as<cd>(), scratch_len,
                               c->st);
        });
    }
    // last reorthogonalisation: s = V^H u, |u|^2 from one pass over [V_ptot, u]
    {
        int nch = 0;
        timed(c, 0, (ptot + 2.0) * N * eb, [&] {
            nch = launch_dot_partial(V, N, ptot + 1, vec(ptot), fp32, pl, part, c->st);
        });
        launch_reduce_partial(part, nch, ptot + 1, d, nullptr, nullptr, nullptr, c->st);
        launch_dcgs_coef(ptot, S, ldS, d, sc, hfro2, flag, 1e-300, c->st, Batch(), false, false);
        timed(c, 1, (ptot + 2.0) * N * eb, [&] {
            launch_update(vec(ptot), V, N, ptot, d, fp32, pl, nullptr, c->upd_scratch.as<cd>(),
                          scratch_len, c->st);
        });
        launch_scale_dev(vec(ptot), vec(ptot), fp32, N, sc, false, c->st);
    }
}

void ks_run(osa_ctx* c, bool adjoint, int nev, int pa, bool fp32, double tol, int max_restarts,
            const cd* start /* fp64 internal vector or nullptr */, uint64_t seed, cd* Xout,
            KsStats& stats) {
    const int win = pa;   // converge all wanted eigenvalues together (a cluster needs it)
    const int64_t N = c->N();
    const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
    const int P = nev + pa;              // basis capacity (plus the next vector)
    const int ldS = P + 1;
    DevBuf Vb, Vt, wv, tv, S, T, Z, wr, bz, info, Spb, sws, dcb;
    const bool dcgs = c->opts.orth != 1;   // delayed reorthogonalisation, as in the solve
    dcb.ensure(sizeof(cd) * 2 * (size_t)(P + 2));
    Spb.ensure(sizeof(cd) * (size_t)pa * pa);
    if (pa > 64) sws.ensure(schur_ws_bytes(pa));
    Vb.ensure(es * (size_t)N * (P + 1));
    Vt.ensure(es * (size_t)N * pa);
    wv.ensure(es * (size_t)N);
    tv.ensure(es * (size_t)N);
    S.ensure(sizeof(cd) * (size_t)ldS * P);
    T.ensure(sizeof(cd) * (size_t)pa * pa);
    Z.ensure(sizeof(cd) * (size_t)pa * pa);
    wr.ensure(sizeof(cd) * pa);
    bz.ensure(sizeof(cd) * pa);
    info.ensure(sizeof(int) * 4);
    char* V = (char*)Vb.p;
    auto vec = [&](int j) { return V + es * (size_t)N * j; };
    const TsPlan pl = ts_plan(N);
    double* hfro2 = (double*)(c->dscal.as<cd>() + 8);
    int* flag = c->flag.as<int>();
    OSA_HIP(hipMemsetAsync(S.p, 0, sizeof(cd) * (size_t)ldS * P, c->st));
    if (start) launch_convert(start, false, vec(0), fp32, N, c->st);
    else launch_random_vector(vec(0), fp32, c->g, seed, c->st);
    launch_norm_partial(vec(0), fp32, pl, c->normp.as<double>(), c->st);
    launch_normalize(vec(0), vec(0), fp32, pl, c->normp.as<double>(), c->dscal.as<cd>() + 9,
                     nullptr, 0.0, nullptr, 0, nullptr, 0, c->st);
    OSA_HIP(hipMemsetAsync(hfro2, 0, sizeof(double), c->st));
    int nlock = 0, kcur = 0;
    std::vector<cd> th(pa), bzh(pa);
    double anorm = 0;
    for (int rs = 0; rs <= max_restarts; ++rs) {
        OSA_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, c->st));
        const int ptot = nlock + pa;
        if (dcgs) {
            expand_delayed(c, adjoint, fp32, V, N, S.as<cd>(), ldS, kcur, ptot, wv.p, tv.p,
                           dcb.as<cd>(), hfro2, flag, stats);
        } else {
            for (int j = kcur; j < ptot; ++j) {
                apply_h(c, vec(j), tv.p, fp32, adjoint);
                apply_h(c, tv.p, wv.p, fp32, adjoint);
                stats.matvecs += 2;
                c->prof.counters[3] += c->prof_on ? 1 : 0;
                cd* scol = S.as<cd>() + (size_t)j * ldS;
                cgs2(c, wv.p, V, N, j + 1, fp32, scol, c->coef.as<cd>());
                launch_normalize(wv.p, vec(j + 1), fp32, pl, c->normp.as<double>(),
                                 scol + (j + 1), hfro2, 1e-300, flag, j, scol, j + 1, c->st);
            }
        }
        // Schur form of the active Rayleigh quotient, smallest |theta| first
        const double tr0 = now_ms();
        const int na = pa;
        cd* Sp = Spb.as<cd>();
        OSA_HIP(hipMemcpy2DAsync(Sp, sizeof(cd) * na, S.as<cd>() + nlock + (size_t)nlock * ldS,
                                 sizeof(cd) * ldS, sizeof(cd) * na, na, hipMemcpyDeviceToDevice,
                                 c->st));
        timed(c, 4, 0.0, [&] {
            small_schur(Sp, na, T.as<cd>(), Z.as<cd>(), wr.as<cd>(), 0, info.as<int>(), sws.p,
                        c->st);
        });
        // spike in the Schur basis: b^H Z with b^H = S[ptot, nlock:ptot]
        launch_zgemm(0, 0, 1, na, na, mk(1.0, 0.0), S.as<cd>() + ptot + (size_t)nlock * ldS, ldS,
                     Z.as<cd>(), na, mk(0.0, 0.0), bz.as<cd>(), 1, c->st);
        int hinfo2[2] = {0, 0};
        d2h(c, info.p, 2, hinfo2);
        const int hinfo = hinfo2[0];
        if (c->prof_on && hinfo >= 0) {
            c->prof.counters[0] += hinfo;
            c->prof.counters[1] += hinfo2[1];
        }
        if (hinfo < 0)
            throw OsaError{OSA_ERR_EIG_NOCONV, "small Schur QR did not converge (active block " +
                                                   std::to_string(na) + ", restart " +
                                                   std::to_string(rs) + ")"};
        d2h(c, wr.p, na, th.data());
        d2h(c, bz.p, na, bzh.data());
        for (int i = 0; i < na; ++i) anorm = std::max(anorm, cabsd(th[i]));
        const int want = nev - nlock;
        int nc = 0;
        while (nc < want && cabsd(bzh[nc]) <= tol * anorm) ++nc;
        stats.restarts = rs;
        if (nc >= want || rs == max_restarts) {
            stats.converged = (nc >= want);
            if (nlock > 0) launch_convert(V, fp32, Xout, false, N * nlock, c->st);
            launch_rotate(vec(nlock), N, na, Z.as<cd>(), na, want, Vt.p, N, fp32, N, c->st);
            launch_convert(Vt.p, fp32, Xout + (size_t)nlock * N, false, N * want, c->st);
            sync(c);
            return;
        }
        // restart: lock nc vectors; keep the wanted Schur vectors plus up to half the
        // surplus, and never less than half of the active block (with few wanted
        // left, a thin restart would discard the cluster around them)
        const int wa = std::min(want, win);
        int keep = std::max(wa + std::min(nc, (na - wa) / 2), na / 2);
        if (keep > na - 4) keep = na - 4;
        if (keep < wa) keep = wa;
        launch_rotate(vec(nlock), N, na, Z.as<cd>(), na, keep, Vt.p, N, fp32, N, c->st);
        OSA_HIP(hipMemcpyAsync(vec(nlock), Vt.p, es * (size_t)N * keep, hipMemcpyDeviceToDevice,
                               c->st));
        OSA_HIP(hipMemcpyAsync(vec(nlock + keep), vec(ptot), es * (size_t)N,
                               hipMemcpyDeviceToDevice, c->st));
        OSA_HIP(hipMemsetAsync(S.p, 0, sizeof(cd) * (size_t)ldS * P, c->st));
        const int nl2 = nlock + nc, na2 = keep - nc;
        // active block: T[nc:keep, nc:keep]; spike row at index nlock + keep
        OSA_HIP(hipMemcpy2DAsync(S.as<cd>() + nl2 + (size_t)nl2 * ldS, sizeof(cd) * ldS,
                                 T.as<cd>() + nc + (size_t)nc * na, sizeof(cd) * na,
                                 sizeof(cd) * na2, na2, hipMemcpyDeviceToDevice, c->st));
        OSA_HIP(hipMemcpy2DAsync(S.as<cd>() + (nlock + keep) + (size_t)nl2 * ldS, sizeof(cd) * ldS,
                                 bz.as<cd>() + nc, sizeof(cd), sizeof(cd), na2,
                                 hipMemcpyDeviceToDevice, c->st));
        kcur = nlock + keep;
        nlock = nl2;
        if (c->prof_on && c->prof.calls[5]++ % c->prof_every == 0) {
            sync(c);
            c->prof.ms[5] += now_ms() - tr0;
            c->prof.launches[5] += 1;
        }
    }
}

// ------------------------------------------------ filtered subspace iteration
// out = alpha ay + beta y + gamma yp over n complex entries (real coefficients);
// out may be yp.
__global__ __launch_bounds__(256) void k_cheb_step(cd* out, const cd* __restrict__ ay,
                                                   const cd* __restrict__ y, const cd* yp,
                                                   int64_t n, double alpha, double beta,
                                                   double gamma) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cd a = ay[i], v = y[i];
    cd r = mk(fma(alpha, a.x, beta * v.x), fma(alpha, a.y, beta * v.y));
    if (yp) {
        const cd q = yp[i];
        r.x = fma(gamma, q.x, r.x);
        r.y = fma(gamma, q.y, r.y);
    }
    out[i] = r;
}

void launch_cheb_step(cd* out, const cd* ay, const cd* y, const cd* yp, int64_t n, double alpha,
                      double beta, double gamma, hipStream_t st) {
    hipLaunchKernelGGL(k_cheb_step, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, out, ay, y,
                       yp, n, alpha, beta, gamma);
    OSA_LAUNCH_CHECK();
}

// Chebyshev-filtered subspace iteration for the nev eigenvalues of A = H^2 of
// smallest modulus (A = H(mu)^2, or H(-mu)^2 for the left vectors), an
// alternative to Krylov-Schur for the search of the critical eigenpairs.  A
// block of s orthonormal vectors is replaced each iteration by p(A) X, where p
// is the degree-deg Chebyshev polynomial of the first kind mapped from [a, b]
// to [-1, 1] (so |p| <= 1 on the damped part of the spectrum and grows fast
// below a), in the three-term recurrence scaled so that p(0) stays of order
// one.  The filtered block is orthonormalised (CGS2, column by column) and
// rotated by the Schur vectors of its Rayleigh quotient X^H A X, smallest
// |theta| first.  b = 1.01 hnorm_bound^2 bounds |lambda(A)|; a is the largest
// |theta| of the block, which for Hermitian A is at least the s-th smallest
// eigenvalue (Courant-Fischer), so the wanted ones stay below it.  Converged
// when the Schur residuals |A x_i - X t_i| of the first nev columns are all at
// most tol * b; the output is then those nev columns, an orthonormal basis of
// the wanted invariant subspace, as from ks_run.  Returns false if max_it
// iterations do not converge.
constexpr int kFilterMaxIt = 80;   // iterations before falling back to Krylov-Schur

bool chfsi_run(osa_ctx* c, bool adjoint, int nev, int s, int deg, double tol, int max_it,
               uint64_t seed, cd* Xout, KsStats& stats) {
    const int64_t N = c->N();
    ensure_exec(c, 2 * s + 2);
    const size_t blk = sizeof(cd) * (size_t)N * s;
    DevBuf buf[4], G, T, Z, wr, info, sws, hc, co, hs;
    for (auto& b : buf) b.ensure(blk);
    G.ensure(sizeof(cd) * (size_t)s * s);
    T.ensure(sizeof(cd) * (size_t)s * s);
    Z.ensure(sizeof(cd) * (size_t)s * s);
    wr.ensure(sizeof(cd) * s);
    info.ensure(sizeof(int) * 4);
    hc.ensure(sizeof(cd) * s);
    co.ensure(sizeof(cd) * s);
    hs.ensure(sizeof(cd) * s);
    if (s > 64) sws.ensure(schur_ws_bytes(s));
    cd* X = buf[0].as<cd>();    // current orthonormal block
    cd* Q = buf[1].as<cd>();    // rotated block / recurrence
    cd* W = buf[2].as<cd>();    // A applied to a block
    cd* Tm = buf[3].as<cd>();   // H applied to a block, residuals
    auto col = [&](cd* base, int j) { return base + (size_t)N * j; };
    const TsPlan pl = ts_plan(N);
    const int64_t scratch_len = (int64_t)(c->upd_scratch.bytes / sizeof(cd));
    cd* part = c->partial.as<cd>();
    const double b = 1.01 * c->hnorm_bound * c->hnorm_bound;
    auto apply_a = [&](const cd* in, cd* out) {
        apply_h_contig(c, in, Tm, false, adjoint, s);
        apply_h_contig(c, Tm, out, false, adjoint, s);
        stats.matvecs += 2 * s;
    };
    auto orthonormalize = [&](cd* Y) {
        for (int j = 0; j < s; ++j) {
            if (j > 0) cgs2(c, col(Y, j), Y, N, j, false, hc.as<cd>(), co.as<cd>());
            else launch_norm_partial(col(Y, 0), false, pl, c->normp.as<double>(), c->st);
            launch_normalize(col(Y, j), col(Y, j), false, pl, c->normp.as<double>(),
                             hs.as<cd>(), nullptr, 0.0, nullptr, 0, nullptr, 0, c->st);
        }
    };
    for (int j = 0; j < s; ++j)
        launch_random_vector(col(X, j), false, c->g, seed + 104729ULL * (uint64_t)j, c->st);
    orthonormalize(X);
    std::vector<cd> th(s), thp(s, mk(0.0, 0.0)), rn(nev);
    for (int it = 0; it <= max_it; ++it) {
        // Rayleigh quotient G = X^H A X (two columns per pass over X), Schur form
        apply_a(X, W);
        for (int j = 0; j < s; j += 2) {
            int nch = 0;
            if (j + 1 < s) {
                timed(c, 0, (s + 2.0) * N * 16.0, [&] {
                    nch = launch_dot2_partial(X, N, s, col(W, j), col(W, j + 1), false, pl, part,
                                              c->st);
                });
                launch_reduce_partial(part, nch, 2 * s, G.as<cd>() + (size_t)j * s, nullptr,
                                      nullptr, nullptr, c->st);
            } else {
                timed(c, 0, (s + 1.0) * N * 16.0, [&] {
                    nch = launch_dot_partial(X, N, s, col(W, j), false, pl, part, c->st);
                });
                launch_reduce_partial(part, nch, s, G.as<cd>() + (size_t)j * s, nullptr, nullptr,
                                      nullptr, c->st);
            }
        }
        timed(c, 4, 0.0, [&] {
            small_schur(G.as<cd>(), s, T.as<cd>(), Z.as<cd>(), wr.as<cd>(), 0, info.as<int>(),
                        sws.p, c->st);
        });
        int hinfo[2] = {0, 0};
        d2h(c, info.p, 2, hinfo);
        if (hinfo[0] < 0) return false;
        if (c->prof_on) {
            c->prof.counters[0] += hinfo[0];
            c->prof.counters[1] += hinfo[1];
        }
        d2h(c, wr.p, s, th.data());
        stats.restarts = it;
        // Schur residuals once the leading |theta| have settled (moduli: members of
        // a pair of equal modulus may trade places between iterations), and at
        // least every fourth iteration
        double dth = 0;
        for (int i = 0; i < nev; ++i)
            dth = std::max(dth, std::fabs(cabsd(th[i]) - cabsd(thp[i])) /
                                    std::max(cabsd(th[i]), 1e-300));
        thp = th;
        const bool check = (it > 0 && dth < 1e-7) || it % 4 == 3 || it == max_it;
        // Schur basis Q = X Z (the filter runs on it: its most amplified columns
        // come first, which keeps the column-wise orthonormalisation accurate)
        // and A Q = W Z (into Tm)
        launch_rotate(X, N, s, Z.as<cd>(), s, s, Q, N, false, N, c->st);
        launch_rotate(W, N, s, Z.as<cd>(), s, s, Tm, N, false, N, c->st);
        if (check) {
            // residuals A q_i - Q t_i of the first nev columns, in W
            OSA_HIP(hipMemcpyAsync(W, Tm, sizeof(cd) * (size_t)N * nev, hipMemcpyDeviceToDevice,
                                   c->st));
            for (int i = 0; i < nev; ++i) {
                timed(c, 1, (i + 3.0) * N * 16.0, [&] {
                    launch_update(col(W, i), Q, N, i + 1, T.as<cd>() + (size_t)i * s, false, pl,
                                  c->normp.as<double>(), c->upd_scratch.as<cd>(), scratch_len,
                                  c->st);
                });
                launch_normalize(col(W, i), nullptr, false, pl, c->normp.as<double>(),
                                 hs.as<cd>() + i, nullptr, 0.0, nullptr, 0, nullptr, 0, c->st);
            }
            d2h(c, hs.p, nev, rn.data());
            int nc = 0;
            while (nc < nev && rn[nc].x <= tol * b) ++nc;
            if (nc >= nev) {
                OSA_HIP(hipMemcpyAsync(Xout, Q, sizeof(cd) * (size_t)N * nev,
                                       hipMemcpyDeviceToDevice, c->st));
                sync(c);
                stats.converged = true;
                return true;
            }
        }
        if (it == max_it) break;
        // filter interval [a, b]: a = the largest |theta| of the block
        double a = 0;
        for (int i = 0; i < s; ++i) a = std::max(a, cabsd(th[i]));
        a = std::min(a, 0.95 * b);
        const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
        const double s1 = e / (0.0 - cc);   // scaling at the wanted end, 0
        // y0 = Q, y1 = (s1/e)(A - cc) y0 (A y0 in Tm),
        // y_{n+1} = 2(sn/e)(A - cc) y_n - s sn y_{n-1}
        cd* prev = Q;
        cd* cur = X;
        const int64_t nn = N * (int64_t)s;
        launch_cheb_step(cur, Tm, prev, nullptr, nn, s1 / e, -s1 * cc / e, 0.0, c->st);
        double sg = s1;
        for (int n = 2; n <= deg; ++n) {
            const double sn = 1.0 / (2.0 / s1 - sg);
            apply_a(cur, W);
            launch_cheb_step(prev, W, cur, prev, nn, 2.0 * sn / e, -2.0 * sn * cc / e, -sg * sn,
                             c->st);
            std::swap(prev, cur);
            sg = sn;
        }
        orthonormalize(cur);
        if (cur != X) std::swap(buf[0].p, buf[1].p);   // X <- filtered block
        X = buf[0].as<cd>();
        Q = buf[1].as<cd>();
    }
    sync(c);
    return false;
}

// max_i |H v_i - lam_i v_i| over the columns cols of V (unit vectors, ld N)
double eig_resid(osa_ctx* c, bool adjoint, const cd* V, const std::vector<cd>& lam,
                 const std::vector<int>& cols) {
    const int64_t N = c->N();
    DevBuf hv;
    hv.ensure(sizeof(cd) * (size_t)N);
    double mx = 0;
    for (int i : cols) {
        apply_h(c, V + (size_t)i * N, hv.p, false, adjoint);
        cd negl = mk(-lam[i].x, -lam[i].y);
        h2d(c, c->coef.p, &negl, 1);
        launch_combine(hv.p, V + (size_t)i * N, N, 1, c->coef.as<cd>(), false, true, N, c->st);
        vec_norm(c, hv.p, false, c->dscal.as<cd>() + 12);
        cd hn;
        d2h(c, c->dscal.as<cd>() + 12, 1, &hn);
        mx = std::max(mx, hn.x);
    }
    return mx;
}

// Rayleigh-Ritz with H in span(X): M = X^H H X, Schur form sorted by |Re|,
// eigenvectors Y; Rv = X Y[:, :m], lam = diag.  Residuals |H r - lam r| of the
// first mres of them (all m when mres < 0).
void rayleigh_ritz(osa_ctx* c, bool adjoint, int nev, int m, cd* X, cd* Rout,
                   std::vector<cd>& lam, double& max_res, int mres = -1) {
    if (mres < 0) mres = m;
    const int64_t N = c->N();
    DevBuf W, Mb, T, Z, Y, wr, info, HR, res;
    W.ensure(sizeof(cd) * (size_t)N * nev);
    Mb.ensure(sizeof(cd) * nev * nev);
    T.ensure(sizeof(cd) * nev * nev);
    Z.ensure(sizeof(cd) * nev * nev);
    Y.ensure(sizeof(cd) * nev * nev);
    wr.ensure(sizeof(cd) * nev);
    info.ensure(sizeof(int) * 4);
    HR.ensure(sizeof(cd) * (size_t)N * m);
    apply_h_contig(c, X, W.p, false, adjoint, nev);
    const TsPlan p = ts_plan(N);
    for (int j = 0; j < nev; ++j) {
        const int nch = launch_dot_partial(X, N, nev, W.as<cd>() + (size_t)j * N, false, p,
                                           c->partial.as<cd>(), c->st);
        launch_reduce_partial(c->partial.as<cd>(), nch, nev, Mb.as<cd>() + (size_t)j * nev,
                              nullptr, nullptr, nullptr, c->st);
    }
    DevBuf sws;
    if (nev > 64) sws.ensure(schur_ws_bytes(nev));
    small_schur(Mb.as<cd>(), nev, T.as<cd>(), Z.as<cd>(), wr.as<cd>(), 1, info.as<int>(), sws.p,
                c->st);
    small_eigvecs(T.as<cd>(), Z.as<cd>(), nev, Y.as<cd>(), c->st);
    int hinfo = 0;
    d2h(c, info.p, 1, &hinfo);
    if (hinfo < 0) throw OsaError{OSA_ERR_EIG_NOCONV};
    std::vector<cd> allw(nev);
    d2h(c, wr.p, nev, allw.data());
    lam.assign(allw.begin(), allw.begin() + m);
    launch_rotate(X, N, nev, Y.as<cd>(), nev, m, Rout, N, false, N, c->st);
    launch_rotate(W.p, N, nev, Y.as<cd>(), nev, m, HR.p, N, false, N, c->st);
    // residuals: |HR_i - lam_i R_i| (R_i unit)
    max_res = 0;
    for (int i = 0; i < mres; ++i) {
        cd* hr = HR.as<cd>() + (size_t)i * N;
        cd negl = mk(-lam[i].x, -lam[i].y);
        h2d(c, c->coef.p, &negl, 1);
        launch_combine(hr, Rout + (size_t)i * N, N, 1, c->coef.as<cd>(), false, true, N, c->st);
        vec_norm(c, hr, false, c->dscal.as<cd>() + 12);
        cd hn;
        d2h(c, c->dscal.as<cd>() + 12, 1, &hn);
        max_res = std::max(max_res, hn.x);
    }
}

// ncv_req / maxr_req > 0 override the active block and the restart cap;
// t0: start of the whole initialisation (a retry keeps counting from it)
void deflate(osa_ctx* c, int m, osa_info* info, int ncv_req = 0, int maxr_req = 0,
             double t0 = -1.0) {
    if (t0 < 0) t0 = now_ms();
    if (m == 0) {
        c->m_alloc = c->m_active = 0;
        c->lambda.clear();
        c->t_init_ms = 0;
        return;
    }
    const int64_t N = c->N();
    ensure_krylov(c, std::max(c->kcap, std::max(c->opts.k_max, 64)));
    const int extra = std::max(4, m / 5);
    const int nev = m + extra;
    // active block of the Krylov-Schur basis (the small Schur kernels take up
    // to 96); the whole basis must fit in the 12 V dimensional space
    const int64_t dim = 12LL * c->g.V;
    // default active block nev + 16 within [64, 96]: at 8^4 with nev = 48, 64 beats 56,
    // 72, 80 and 96 (the Schur cost per restart grows as the cube of the block);
    // smaller blocks failed to converge on hard instances (m_w near -1.9)
    int ncv = ncv_req > 0 ? ncv_req
                          : (c->opts.eig_ncv > 0 ? c->opts.eig_ncv
                                                 : std::min(96, std::max(64, nev + 16)));
    if (ncv > 96) ncv = 96;
    if ((int64_t)nev + ncv + 1 > dim) ncv = (int)std::max<int64_t>(8, dim - nev - 1);
    if (ncv < nev + 4 || (int64_t)nev + ncv + 1 > dim) throw OsaError{OSA_ERR_ARG};
    const double tol = c->opts.eig_tol > 0 ? c->opts.eig_tol : 1e-12;
    // FP64 search with eig_filter = d > 0: Chebyshev-filtered subspace iteration of
    // degree d (block nev + 48 within [64, 96] unless eig_ncv is set)
    const int filter_deg = c->opts.eig_filter > 0 ? c->opts.eig_filter : 0;
    int fblock = (ncv_req > 0 || c->opts.eig_ncv > 0) ? ncv : std::min(96, std::max(64, nev + 48));
    if ((int64_t)fblock > dim) fblock = (int)dim;
    const int maxr = maxr_req > 0 ? maxr_req
                                  : (c->opts.eig_max_restarts > 0 ? c->opts.eig_max_restarts : 2000);
    const bool fp32 = (c->opts.eig_prec == OSA_FP32);
    if (fp32) ensure_links32(c);
    // Schur deflation needs the right eigenvectors only
    const bool right_only = c->opts.deflation == 1;
    DevBuf X, Rn, Ln, Xs;
    X.ensure(sizeof(cd) * (size_t)N * nev);
    Xs.ensure(sizeof(cd) * N);
    Rn.ensure(sizeof(cd) * (size_t)N * m);
    // the left search returns all nev Ritz pairs of H(-mu), for the pairing below
    if (!right_only) Ln.ensure(sizeof(cd) * (size_t)N * nev);
    KsStats st;
    std::vector<cd> lam_r, lam_l;
    double res_r = 0, res_l = 0;
    // One side of the eigenproblem: right vectors of H(mu) (adj = false) or of
    // H(-mu) = H(mu)^dag, i.e. left vectors of H(mu) (adj = true).
    auto side = [&](osa_ctx* e, bool adj, cd* Xb, cd* Xs, cd* out, std::vector<cd>& lam,
                    double& res, KsStats& sst) {
        const uint64_t seed = 0x5eedULL + 7919ULL * (adj ? 1 : 0);
        if (fp32) {
            KsStats s32;
            ks_run(e, adj, nev, ncv, true, std::max(tol, 1e-6), maxr, nullptr, seed, Xb, s32);
            sst.matvecs += s32.matvecs;
            sst.restarts += s32.restarts;
            // fp64 refinement from the fp32 subspace: start vector = sum of its basis
            std::vector<cd> ones(nev, mk(1.0, 0.0));
            h2d(e, e->coef.p, ones.data(), nev);
            launch_combine(Xs, Xb, N, nev, e->coef.as<cd>(), false, false, N, e->st);
            KsStats s64;
            ks_run(e, adj, nev, ncv, false, tol, maxr, Xs, seed, Xb, s64);
            sst.matvecs += s64.matvecs;
            sst.restarts += s64.restarts;
            if (!s64.converged)
                throw OsaError{OSA_ERR_EIG_NOCONV, "fp64 refinement hit the restart cap"};
        } else {
            bool done = false;
            if (filter_deg > 0) {   // filtered subspace iteration, Krylov-Schur if it fails
                KsStats sf;
                done = chfsi_run(e, adj, nev, fblock, filter_deg, tol, kFilterMaxIt, seed, Xb, sf);
                sst.matvecs += sf.matvecs;
                sst.restarts += sf.restarts;
            }
            if (!done) {
                KsStats s64;
                ks_run(e, adj, nev, ncv, false, tol, maxr, nullptr, seed, Xb, s64);
                sst.matvecs += s64.matvecs;
                sst.restarts += s64.restarts;
                if (!s64.converged)
                    throw OsaError{OSA_ERR_EIG_NOCONV, "Krylov-Schur hit the restart cap (" +
                                                           std::to_string(maxr) + ")"};
            }
        }
        sst.matvecs += nev;
        // the left side keeps all nev pairs; their residuals follow the pairing
        rayleigh_ritz(e, adj, nev, adj ? nev : m, Xb, out, lam, res, adj ? 0 : m);
    };
    // the left side runs on a worker clone: own non-blocking stream and work
    // buffers, the parent's links; ordered after everything queued so far
    std::unique_ptr<osa_ctx> w(new osa_ctx());
    w->g = c->g;
    w->links_fp32 = c->links_fp32;
    w->mu = c->mu; w->m_w = c->m_w; w->kappa = c->kappa; w->hnorm_bound = c->hnorm_bound;
    w->hc = c->hc; w->hc_adj = c->hc_adj; w->opts = c->opts;
    w->u_ext = c->U.p;
    w->u32_ext = c->U32.p;
    w->prof_on = c->prof_on;
    w->prof_every = c->prof_every;
    OSA_HIP(hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking));
    w->own_stream = true;
    ensure_exec(w.get(), nev + ncv + 1);
    {
        hipEvent_t ready;
        OSA_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        OSA_HIP(hipEventRecord(ready, c->st));
        OSA_HIP(hipStreamWaitEvent(w->st, ready, 0));
        OSA_HIP(hipEventSynchronize(ready));
        (void)hipEventDestroy(ready);
    }
    DevBuf X2, Xs2;
    if (!right_only) {
        X2.ensure(sizeof(cd) * (size_t)N * nev);
        Xs2.ensure(sizeof(cd) * N);
    }
    KsStats st_l;
    std::exception_ptr werr;
    std::thread worker([&] {
        if (right_only) return;
        try {
            side(w.get(), true, X2.as<cd>(), Xs2.as<cd>(), Ln.as<cd>(), lam_l, res_l, st_l);
        } catch (...) {
            werr = std::current_exception();
        }
    });
    std::exception_ptr merr;
    try {
        side(c, false, X.as<cd>(), Xs.as<cd>(), Rn.as<cd>(), lam_r, res_r, st);
    } catch (...) {
        merr = std::current_exception();
    }
    worker.join();
    if (c->prof_on) {
        for (int i = 0; i < OSA_PROFILE_CLASSES; ++i) {
            c->prof.ms[i] += w->prof.ms[i];
            c->prof.bytes[i] += w->prof.bytes[i];
            c->prof.flops[i] += w->prof.flops[i];
            c->prof.launches[i] += w->prof.launches[i];
            c->prof.calls[i] += w->prof.calls[i];
        }
        for (int i = 0; i < 4; ++i) c->prof.counters[i] += w->prof.counters[i];
    }
    if (merr) std::rethrow_exception(merr);
    if (werr) std::rethrow_exception(werr);
    st.matvecs += st_l.matvecs;
    st.restarts += st_l.restarts;
    // Pair the left vectors with the right ones.  Right eigenvalue lam_r[i] takes
    // the unused left Ritz pair (of H(-mu)) whose conjugate eigenvalue is nearest,
    // so L comes in R's order and G = L^dag R is nearly diagonal.  A swap inside a
    // cluster of close eigenvalues is harmless: the projector R G^-1 L^dag of
    // Eq. 20-21 and the adjoint's deflated part only need the same invariant
    // subspace on both sides.  What must hold is that every right eigenvalue has a
    // left partner; the tolerance, 1e-6 |H|, allows for ill-conditioned
    // eigenvalues, whose error is the residual times the condition number
    // 1 / |l^dag r|.  Two searches that found different eigenvalues closer than
    // that leave G singular, which build_ginv reports.
    std::vector<int> pick(m, -1);
    if (!right_only) {
        const double hn = c->hnorm_bound;
        std::vector<char> used(lam_l.size(), 0);
        double worst = 0;
        for (int i = 0; i < m; ++i) {
            int best = -1;
            double bd = INFINITY;
            for (size_t j = 0; j < lam_l.size(); ++j) {
                if (used[j]) continue;
                const double d = cabsd(csub(cconj(lam_l[j]), lam_r[i]));
                if (d < bd) { bd = d; best = (int)j; }
            }
            if (best < 0) {
                c->m_alloc = c->m_active = 0;
                throw OsaError{OSA_ERR_EIG_NOCONV, "fewer left than right critical pairs"};
            }
            used[best] = 1;
            pick[i] = best;
            worst = std::max(worst, bd);
        }
        res_l = eig_resid(w.get(), true, Ln.as<cd>(), lam_l, pick);
        if (!(worst <= 1e-6 * hn)) {
            c->m_alloc = c->m_active = 0;
            char b[200];
            snprintf(b, sizeof b, "left and right searches disagree: a critical eigenvalue has "
                     "no left partner within %.1e (nearest %.3e; residuals %.1e / %.1e)",
                     1e-6 * hn, worst, res_r, res_l);
            throw OsaError{OSA_ERR_EIG_NOCONV, b};
        }
    }
    // install
    c->R.ensure(sizeof(cd) * (size_t)N * m);
    OSA_HIP(hipMemcpyAsync(c->R.p, Rn.p, sizeof(cd) * (size_t)N * m, hipMemcpyDeviceToDevice, c->st));
    if (!right_only) {
        c->L.ensure(sizeof(cd) * (size_t)N * m);
        for (int i = 0; i < m; ++i)
            OSA_HIP(hipMemcpyAsync(c->L.as<cd>() + (size_t)i * N, Ln.as<cd>() + (size_t)pick[i] * N,
                                   sizeof(cd) * (size_t)N, hipMemcpyDeviceToDevice, c->st));
    }
    c->have_left = !right_only;
    c->schur_m = 0;
    c->lambda = lam_r;
    c->lam_dev.ensure(sizeof(cd) * m);
    h2d(c, c->lam_dev.p, c->lambda.data(), m);
    c->m_alloc = m;
    double hn = c->hnorm_bound;
    c->min_abs_re = INFINITY;
    for (auto& l : c->lambda) c->min_abs_re = std::min(c->min_abs_re, std::fabs(l.x));
    c->max_eig_resid = std::max(res_r, res_l);
    c->eig_matvecs = st.matvecs;
    c->eig_restarts = st.restarts;
    if (c->min_abs_re < 1e-12 * hn) {
        c->m_alloc = c->m_active = 0;   // no half-installed deflation data stays active
        throw OsaError{OSA_ERR_IMAG_AXIS};
    }
    // the Krylov-Schur test is on H^2; the pairs used are checked on H itself
    if (!(c->max_eig_resid <= 1e-8 * hn)) {
        c->m_alloc = c->m_active = 0;
        char b[160];
        snprintf(b, sizeof b, "eigenpair residual %.3e (right %.3e, left %.3e) above 1e-8 |H|",
                 c->max_eig_resid, res_r, res_l);
        throw OsaError{OSA_ERR_EIG_NOCONV, b};
    }
    set_active(c, m);
    sync(c);
    c->t_init_ms = now_ms() - t0;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->n_defl = m;
        info->min_abs_re_lambda = c->min_abs_re;
        info->max_eig_resid = c->max_eig_resid;
        info->t_init_ms = c->t_init_ms;
        info->eig_matvecs = c->eig_matvecs;
        info->eig_restarts = c->eig_restarts;
        info->status = OSA_OK;
    }
}

void fill_defaults(osa_opts& o) {
    // orth: 0 delayed reorthogonalisation (default), 1 plain CGS2
    if (o.max_batch <= 0) o.max_batch = 16;
    if (o.k_max <= 0) o.k_max = 600;
    if (o.check_every == 0) o.check_every = 50;
}

osa_status validate_lattice(const osa_lattice* lat) {
    if (!lat) return OSA_ERR_ARG;
    for (int i = 0; i < 4; ++i)
        if (lat->dims[i] < 2 || lat->dims[i] > 4096) return OSA_ERR_ARG;
    const int64_t v = (int64_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    if (v > (1LL << 28)) return OSA_ERR_ARG;
    return OSA_OK;
}

template <typename F>
osa_status guard(F&& f, std::string* msg = nullptr) {
    if (msg) msg->clear();
    try {
        return f();
    } catch (const OsaError& e) {
        if (msg) *msg = e.why;
        return e.s;
    } catch (const HipError& e) {
        if (msg) *msg = std::string(e.where) + ": " + hipGetErrorString(e.e);
        (void)hipGetLastError();
        return OSA_ERR_HIP;
    } catch (const std::bad_alloc&) {
        if (msg) *msg = "device allocation failed";
        return OSA_ERR_OOM;
    } catch (const std::length_error& e) {
        if (msg) *msg = e.what();
        return OSA_ERR_ARG;
    } catch (...) {
        return OSA_ERR_HIP;
    }
}

// What an apply call computes from the sign: sign(H) B, sign(H)^dag B, or the
// overlap operator B + gamma_5 sign(H) B.
enum class ApplyMode { kSign, kAdjoint, kOverlap };

// GinvH = (G^{-1})^H, m x m column-major
__global__ void k_conj_transpose(int m, const cd* __restrict__ A, cd* __restrict__ B) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * m) return;
    const int i = e % m, j = e / m;
    B[e] = cconj(A[j + (int64_t)i * m]);
}

// Y = B + gamma_5 Y in the boundary layout (index (site*4 + spin)*3 + color;
// chiral basis, gamma_5 = diag(1, 1, -1, -1) in spin)
__global__ void k_overlap_finish(const cd* __restrict__ B, cd* Y, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int spin = (int)((e / 3) % 4);
    const cd b = B[e], y = Y[e];
    Y[e] = spin < 2 ? cadd(b, y) : csub(b, y);
}

// ================================================================ block Krylov
// A multi-source variant that is not the paper's method: one Krylov space is
// built from all s sources together, the block full orthogonalisation
// approximation of sign(H) B (Eq. 11 per block of sources; with s = 1 it is
// Eq. 22), with the same LR deflation (Eq. 21-22):
//   B_ominus = V_1 R_0 (the projected sources, QR by Gram-Schmidt),
//   H V_j re-projected and orthogonalised against all blocks by classical
//   Gram-Schmidt applied twice (the shared basis is read once per pass for all
//   s vectors), then its QR gives V_{j+1} and the subdiagonal block,
//   sign(H) B ~ R sgn(Lambda) G^{-1} L^dag B + V_K sign(H_K) E_1 R_0,
// with H_K the K s x K s block upper Hessenberg matrix.  The convergence
// estimate is the largest change of a column of sign(H_K) E_1 R_0 between
// checks relative to its source's norm, with the geometric-tail rule of the
// single-source solve.
struct BlockResult {
    osa_status st = OSA_OK;
    int dim = 0;          // K s
    int blocks = 0;
    double est = NAN;
    int newton_iters = 0;
    int breakdown = 0;
};

void solve_block(osa_ctx* c, int s, const cd* xin, cd* yout, double tol, int kb_max,
                 BlockResult& out, std::vector<double>& est_src) {
    const int64_t N = c->N();
    const int m = c->m_active;
    check_deflation_state(c);
    if (c->opts.deflation == 1 && m > 0)
        throw OsaError{OSA_ERR_STATE, "the block variant uses LR deflation (deflation = 0)"};
    const int D = (kb_max + 1) * s;     // basis columns
    const int64_t ldh = D;
    const int kdim = kb_max * s;        // largest small problem
    ensure_exec(c, D + s, s);
    c->Vblk.ensure(sizeof(cd) * (size_t)N * D);
    c->Hblk.ensure(sizeof(cd) * (size_t)ldh * kdim);
    c->Wblk.ensure(sizeof(cd) * (size_t)N * s);
    c->cblk2.ensure(sizeof(cd) * (size_t)ldh * s);
    const int mm = std::max(m, 1);
    c->cdefb.ensure(sizeof(cd) * (size_t)mm * s);
    c->ctmpb.ensure(sizeof(cd) * (size_t)mm * s);
    c->ccoefb.ensure(sizeof(cd) * (size_t)mm * s);
    c->r0b.ensure(sizeof(cd) * (size_t)s * s);
    c->ysmb.ensure(sizeof(cd) * (size_t)kdim * s);
    // small-sign workspace for one problem of size up to kdim
    if (c->scap < kdim || c->kbatch < 1) {
        c->scap = std::max(c->scap, kdim);
        const int scap = c->scap;
        const int nb = std::max(c->kbatch, 1);
        c->kbatch = nb;
        c->red_stride = newton_red_len(scap) + 16;
        c->red.ensure(sizeof(double) * (size_t)c->red_stride * nb);
        c->sX.ensure(sizeof(cd) * (size_t)scap * scap * nb);
        c->sM.ensure(sizeof(cd) * (size_t)scap * scap * nb);
        c->sY.ensure(sizeof(cd) * (size_t)scap * scap * nb);
        c->logpiv.ensure(sizeof(double) * (size_t)scap * nb);
        c->gj_stride = (int64_t)ceil_div((int64_t)gj_ws_bytes(scap), 256) * 256;
        c->gjws.ensure((size_t)c->gj_stride * nb);
        c->nflag.ensure(sizeof(int) * 4 * nb);
        c->dscal.ensure(sizeof(cd) * 16);
    }
    const TsPlan p = ts_plan(N);
    cd* Vb = c->Vblk.as<cd>();
    cd* Hb = c->Hblk.as<cd>();
    cd* W = c->Wblk.as<cd>();
    cd* r0 = c->r0b.as<cd>();
    int* flag = c->flag.as<int>();
    double* hfro2 = (double*)(c->dscal.as<cd>() + 14);
    const bool fixed = c->opts.check_every < 0;
    const int cb = fixed ? kb_max : std::max(1, (int)ceil_div(std::max(1, c->opts.check_every), s));
    Batch bs;   // the s sources: consecutive vectors
    bs.n = s;
    bs.basis = N;
    bs.vec = N;
    Batch bp = bs;   // projection coefficients: m per source
    bp.small = mm;
    Batch bd = bs;   // block Gram-Schmidt: coefficients are columns of H (stride ldh)
    bd.part = c->part_stride;
    bd.small = ldh;
    Batch bu = bs;
    bu.small = ldh;
    OSA_HIP(hipMemsetAsync(Hb, 0, sizeof(cd) * (size_t)ldh * kdim, c->st));
    OSA_HIP(hipMemsetAsync(r0, 0, sizeof(cd) * (size_t)s * s, c->st));
    OSA_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, c->st));
    OSA_HIP(hipMemsetAsync(hfro2, 0, sizeof(double), c->st));
    OSA_HIP(hipMemcpyAsync(W, xin, sizeof(cd) * (size_t)N * s, hipMemcpyDeviceToDevice, c->st));
    // |b| of every source (host) for the relative estimate
    std::vector<double> bnorm(s);
    for (int i = 0; i < s; ++i) {
        vec_norm(c, W + (size_t)i * N, false, c->dscal.as<cd>() + 12);
        cd hn;
        d2h(c, c->dscal.as<cd>() + 12, 1, &hn);
        bnorm[i] = hn.x;
        if (!std::isfinite(bnorm[i])) throw OsaError{OSA_ERR_NONFINITE, "source"};
    }
    // B_ominus = B - R G^{-1} L^dag B (Eq. 21); cdefb keeps G^{-1} L^dag B
    if (m > 0) project_out(c, W, c->cdefb.as<cd>(), c->ctmpb.as<cd>(), bp);
    // thin QR B_ominus = V_1 R_0 by Gram-Schmidt (applied twice) column by column
    auto block_qr = [&](cd* src, cd* dst, cd* rcol0, int64_t ldr, int step, bool track) {
        for (int i = 0; i < s; ++i) {
            cd* wcol = src + (size_t)i * N;
            cd* rc = rcol0 + (size_t)i * ldr;   // column i of the R factor (rows 0..i)
            if (i > 0)
                cgs2(c, wcol, dst, N, i, false, rc, c->coef2.as<cd>());
            else
                launch_norm_partial(wcol, false, p, c->normp.as<double>(), c->st);
            launch_normalize(wcol, dst + (size_t)i * N, false, p, c->normp.as<double>(), rc + i,
                             track ? hfro2 : nullptr, track ? 1e-14 : 0.0, track ? flag : nullptr,
                             step, track ? rc : nullptr, track ? i : 0, c->st);
        }
    };
    block_qr(W, Vb, r0, s, 0, false);
    std::vector<cd> ysm_prev, ysm_cur;
    std::vector<double> changes, rates, kprev_list;
    int kprev = 0, skipped = 0;
    double tail = INFINITY;
    for (int j = 0; j < kb_max; ++j) {
        const int ncol = (j + 1) * s;
        // W = H V_j, re-projected (Eq. 21)
        apply_h(c, Vb + (size_t)j * s * N, W, false, false, bs);
        if (m > 0) project_out(c, W, c->ctmpb.as<cd>(), c->ccoefb.as<cd>(), bp);
        cd* hcol = Hb + (size_t)j * s * ldh;   // columns js .. js+s-1 of H
        // block classical Gram-Schmidt, twice; the shared basis is read once per pass
        int nch = 0;
        timed(c, 0, (ncol + s) * (double)N * 16.0, [&] {
            nch = launch_mdot_partial(Vb, N, ncol, W, p, c->partial.as<cd>(), c->st, bd);
        });
        launch_reduce_partial(c->partial.as<cd>(), nch, ncol, hcol, nullptr, nullptr, nullptr,
                              c->st, bd);
        timed(c, 1, (ncol + 2.0 * s) * (double)N * 16.0, [&] {
            launch_mcombine(W, Vb, N, ncol, hcol, N, 1.0, -1.0, c->st, bu);
        });
        timed(c, 0, (ncol + s) * (double)N * 16.0, [&] {
            nch = launch_mdot_partial(Vb, N, ncol, W, p, c->partial.as<cd>(), c->st, bd);
        });
        launch_reduce_partial(c->partial.as<cd>(), nch, ncol, c->cblk2.as<cd>(), hcol, nullptr,
                              nullptr, c->st, bd);
        timed(c, 1, (ncol + 2.0 * s) * (double)N * 16.0, [&] {
            launch_mcombine(W, Vb, N, ncol, c->cblk2.as<cd>(), N, 1.0, -1.0, c->st, bu);
        });
        // QR of the new block: V_{j+1} and the subdiagonal block H[ncol:ncol+s, js:js+s]
        block_qr(W, Vb + (size_t)ncol * N, hcol + ncol, ldh, j, true);
        const int kb = j + 1;
        const bool last = kb == kb_max;
        if (!last && (fixed || kb % cb != 0)) continue;
        int hf[2] = {0, 0};
        d2h(c, flag, 2, hf);
        if (hf[0] == 2) throw OsaError{OSA_ERR_NONFINITE, "block Arnoldi"};
        const bool brk = hf[0] == 1;   // rank-deficient new block: the space is invariant
        if (!last && !brk && !fixed && !changes.empty() && std::isfinite(tail)) {
            // skip checks far before the predicted crossing (at most 3 in a row)
            const double rho = rates.empty() ? 1.0 : rates.back();
            const double pred = tail * std::pow(rho, (double)(kb * s - kprev));
            if (rho < 1.0 && pred > 3.0 * tol && skipped < 3) { ++skipped; continue; }
        }
        skipped = 0;
        const int dim = kb * s;
        std::vector<int> iters(std::max(c->kbatch, 1), 0);
        std::vector<char> okv(std::max(c->kbatch, 1), 0);
        small_sign_batch(c, std::vector<int>{0}, dim, Hb, (int)ldh, 0, c->ysmb.as<cd>(), 0, iters,
                         okv);
        out.newton_iters = iters[0];
        if (iters[0] < 0 || !okv[0]) throw OsaError{OSA_ERR_NEWTON_NOCONV, "block small sign"};
        // F E_1 R_0: the first s columns of sign(H_K) times R_0
        launch_zgemm(0, 0, dim, s, s, mk(1.0, 0.0), c->sX.as<cd>(), dim, r0, s, mk(0.0, 0.0),
                     c->ysmb.as<cd>(), dim, c->st);
        ysm_cur.resize((size_t)dim * s);
        d2h(c, c->ysmb.p, (size_t)dim * s, ysm_cur.data());
        out.blocks = kb;
        out.dim = dim;
        bool stop = brk || last;
        if (brk) out.breakdown = 1;
        if (kprev > 0 && !fixed) {
            double change = 0;
            for (int b = 0; b < s; ++b) {
                double d2 = 0;
                for (int i = 0; i < dim; ++i) {
                    cd d = ysm_cur[(size_t)b * dim + i];
                    if (i < kprev) d = csub(d, ysm_prev[(size_t)b * kprev + i]);
                    d2 += cabs2(d);
                }
                const double e = std::sqrt(d2) / bnorm[b];
                est_src[b] = e;
                change = std::max(change, e);
            }
            tail = change;
            if (!changes.empty()) {
                const int d1 = kprev - (int)kprev_list.back();
                const int d2 = dim - kprev;
                const double rho = geometric_rate(changes.back(), d1, change, d2);
                const double rho_use = rates.empty() ? rho : std::max(rho, rates.back());
                rates.push_back(rho);
                if (c->opts.stop_rule == 0) {
                    const double q = std::pow(rho_use, (double)d2);
                    tail = q < 1.0 ? 2.0 * change * q / (1.0 - q) : INFINITY;
                    for (int b = 0; b < s; ++b)
                        est_src[b] = q < 1.0 ? 2.0 * est_src[b] * q / (1.0 - q) : INFINITY;
                }
            }
            changes.push_back(change);
            kprev_list.push_back(kprev);
            out.est = tail;
            if (tail <= tol) stop = true;
        }
        if (brk) {
            out.est = 0.0;
            for (auto& e : est_src) e = 0.0;
        }
        ysm_prev.swap(ysm_cur);
        kprev = dim;
        if (stop) break;
    }
    // Y = R sgn(Re lambda) G^{-1} L^dag B + V_K (F E_1 R_0)  (Eq. 22 per block)
    const int dim = out.dim;
    Batch by = bs;
    if (m > 0) {
        Batch bo = bs;
        bo.small = mm;
        hipLaunchKernelGGL(k_sign_coef, dim3((unsigned)ceil_div(m, 64), s), dim3(64), 0, c->st, m,
                           (const cd*)c->lam_dev.p, (const cd*)c->cdefb.p, c->ccoefb.as<cd>(), bo);
        OSA_LAUNCH_CHECK();
        by.small = mm;
        launch_mcombine(yout, c->R.as<cd>(), N, m, c->ccoefb.as<cd>(), N, 0.0, 1.0, c->st, by);
    }
    by.small = dim;
    launch_mcombine(yout, Vb, N, dim, c->ysmb.as<cd>(), N, m > 0 ? 1.0 : 0.0, 1.0, c->st, by);
    if (!fixed && !(out.est <= tol)) out.st = OSA_NOT_CONVERGED;
    if (fixed) out.est = NAN;
    sync(c);
}

osa_status apply_impl(osa_ctx* c, int32_t nrhs, const void* B, void* Y, double tol,
                      osa_info* infos, ApplyMode mode) {
    if (!c || nrhs < 1 || !B || !Y) return OSA_ERR_ARG;
    const bool fixed = c->opts.check_every < 0;
    if (!fixed && !(tol > 0)) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        struct AdjScope {   // the adjoint flag holds for this call only
            osa_ctx* c;
            ~AdjScope() { c->adj = false; }
        } scope{c};
        c->adj = (mode == ApplyMode::kAdjoint);
        check_deflation_state(c);
        if (c->adj && c->m_active > 0) {
            const int m = c->m_active;
            c->GinvH.ensure(sizeof(cd) * (size_t)m * m + 16);
            hipLaunchKernelGGL(k_conj_transpose, dim3((unsigned)ceil_div((int64_t)m * m, 256)),
                               dim3(256), 0, c->st, m, c->Ginv.as<cd>(), c->GinvH.as<cd>());
            OSA_LAUNCH_CHECK();
        }
        const int64_t N = c->N();
        const int64_t nbnd = 12LL * c->g.V;
        const int maxb = std::max(1, std::min(c->opts.max_batch, kMaxBatch));
        const int gmax = std::min<int>(nrhs, maxb);
        osa_status first_err = OSA_OK, worst = OSA_OK;
        // kept in the context: a per-call allocation would make hipFree wait for
        // the whole device, serialising concurrent contexts
        DevBuf& xin = c->xio;
        DevBuf& yint = c->yio;
        xin.ensure(sizeof(cd) * N * gmax);
        yint.ensure(sizeof(cd) * N * gmax);
        std::vector<SolveResult> res;
        for (int r0 = 0; r0 < nrhs; r0 += maxb) {
            const int nb = std::min(maxb, nrhs - r0);
            const double t0 = now_ms();
            launch_vec_to_internal((const cd*)B + r0 * nbnd, xin.p, false, c->g, nb, c->st);
            solve_batch(c, nb, xin.as<cd>(), yint.as<cd>(), tol, res);
            // |y| of each result, for the relative estimate
            std::vector<int> okp;
            for (int b = 0; b < nb; ++b)
                if (res[b].st == OSA_OK || res[b].st == OSA_NOT_CONVERGED) okp.push_back(b);
            std::vector<cd> yn;
            if (!okp.empty()) {
                Batch bt = batch_of(okp);
                bt.vec = N;
                bt.part = c->normp_stride;
                bt.scal = c->lay.stride;
                const TsPlan p = ts_plan(N);
                cd* slot = c->arena.as<cd>() + c->lay.ds + 2;
                launch_norm_partial(yint.p, false, p, c->normp.as<double>(), c->st, bt);
                launch_normalize(yint.p, nullptr, false, p, c->normp.as<double>(), slot, nullptr,
                                 0.0, nullptr, 0, nullptr, 0, c->st, bt);
                for (int b : okp) {
                    launch_vec_from_internal(yint.as<cd>() + (size_t)b * N, false,
                                             (cd*)Y + (r0 + b) * nbnd, c->g, 1, c->st);
                    if (mode == ApplyMode::kOverlap) {
                        hipLaunchKernelGGL(k_overlap_finish, dim3((unsigned)ceil_div(nbnd, 256)),
                                           dim3(256), 0, c->st, (const cd*)B + (r0 + b) * nbnd,
                                           (cd*)Y + (r0 + b) * nbnd, nbnd);
                        OSA_LAUNCH_CHECK();
                    }
                }
                d2h_strided(c, slot, c->lay.stride * (int64_t)sizeof(cd), 1, okp, yn);
            }
            sync(c);
            const double t1 = now_ms();
            for (int b = 0; b < nb; ++b) {
                const SolveResult& sr = res[b];
                double ynorm = 1.0;
                for (size_t i = 0; i < okp.size(); ++i)
                    if (okp[i] == b) ynorm = yn[i].x;
                if (infos) {
                    osa_info& in = infos[r0 + b];
                    std::memset(&in, 0, sizeof(in));
                    in.resid_est = std::isnan(sr.est) ? sr.est
                                                      : sr.est * sr.bnorm / std::max(ynorm, 1e-300);
                    in.k_used = sr.k_used;
                    in.n_defl = c->m_active;
                    in.status = sr.st;
                    in.newton_iters = sr.newton_iters;
                    in.breakdown = sr.breakdown;
                    in.min_abs_re_lambda = c->m_active ? c->min_abs_re : NAN;
                    in.max_eig_resid = c->max_eig_resid;
                    in.t_init_ms = c->t_init_ms;
                    in.t_solve_ms = t1 - t0;
                    in.eig_matvecs = c->eig_matvecs;
                    in.eig_restarts = c->eig_restarts;
                    in.batch = nb;
                }
                if (sr.st < 0 && first_err == OSA_OK) first_err = sr.st;
                if (sr.st > worst) worst = sr.st;
            }
        }
        return first_err != OSA_OK ? first_err : worst;
    });
}

}  // namespace

// ====================================================== allocation-free scratch
// Workspace of osa_small_sign_noalloc: one file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  Its size
// covers the small sign of one k x k problem for k <= OSA_NOALLOC_MAX_K: three
// k x k matrices, the pivot logs, the Gauss-Jordan work arrays, the flags and
// the reduction slots, each rounded up to 256 bytes.
static constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
static constexpr size_t kNoallocScratchBytes =
    3 * round256(16ull * OSA_NOALLOC_MAX_K * OSA_NOALLOC_MAX_K) +   // X, M, Y
    round256(8ull * OSA_NOALLOC_MAX_K) +                            // log |pivot|
    round256(92ull * OSA_NOALLOC_MAX_K + 256) +                     // Gauss-Jordan (gj_ws_bytes)
    256 +                                                           // flags
    round256(8ull * (2 + 2 * ((OSA_NOALLOC_MAX_K * OSA_NOALLOC_MAX_K + 255) / 256) + 16));
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[64] = {};   // device address of scratch per device ordinal

// The device address of `scratch` on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in, so kernels get this address, never the name.
static void* noalloc_scratch() {
    int dev = 0;
    OSA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw OsaError{OSA_ERR_HIP, "device ordinal beyond 63"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        OSA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw OsaError{OSA_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL"};
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

// ================================================================ C ABI
extern "C" {

const char* osa_version(void) { return "osa 0.1 (gfx950)"; }

osa_status osa_set_allocator(void* (*alloc)(size_t, void*, void*),
                             void (*dealloc)(void*, void*, void*), void* user) {
    if ((alloc == nullptr) != (dealloc == nullptr)) return OSA_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.dealloc = dealloc;
    g_alloc.user = alloc ? user : nullptr;
    return OSA_OK;
}

const char* osa_last_message(const osa_ctx* c) { return c ? c->msg.c_str() : ""; }

osa_status osa_set_autotune(int32_t on) {
    set_autotune(on != 0);
    return OSA_OK;
}

int32_t osa_autotune_table(int64_t* n, int32_t* bucket, int32_t* chunks, int32_t cap) {
    if (cap < 0) cap = 0;
    std::vector<int> b(cap), w(cap);
    const int total = autotune_entries(n, b.data(), w.data(), cap);
    for (int i = 0; i < std::min(total, (int)cap); ++i) {
        if (bucket) bucket[i] = b[i];
        if (chunks) chunks[i] = w[i];
    }
    return total;
}

osa_status osa_graph_stats(const osa_ctx* c, int64_t* captures, int64_t* launches) {
    if (!c) return OSA_ERR_ARG;
    if (captures) *captures = c->graph_captures;
    if (launches) *launches = c->graph_launches;
    return OSA_OK;
}

const char* osa_status_string(osa_status s) {
    switch (s) {
        case OSA_OK: return "ok";
        case OSA_NOT_CONVERGED: return "not converged (result usable)";
        case OSA_ERR_ARG: return "invalid argument";
        case OSA_ERR_HIP: return "HIP runtime error";
        case OSA_ERR_OOM: return "out of device memory";
        case OSA_ERR_NONFINITE: return "non-finite input or intermediate";
        case OSA_ERR_IMAG_AXIS: return "deflated eigenvalue on the imaginary axis";
        case OSA_ERR_EIG_NOCONV: return "eigensolver did not converge";
        case OSA_ERR_NEWTON_NOCONV: return "small sign iteration did not converge";
        case OSA_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

osa_status osa_set_opts(osa_ctx* c, const osa_opts* opts) {
    if (!c) return OSA_ERR_ARG;
    osa_opts o{};
    if (opts) o = *opts;
    if (o.k_max < 0 || o.k_max > 4000 || o.eig_ncv < 0 || o.eig_ncv > 96 || o.eig_tol < 0 ||
        o.eig_max_restarts < 0 || (o.eig_prec != OSA_FP64 && o.eig_prec != OSA_FP32) ||
        o.max_batch < 0 || o.max_batch > 64 || o.orth < 0 || o.orth > 2 || o.stop_rule < 0 ||
        o.stop_rule > 1 || o.no_graphs < 0 || o.no_graphs > 1 || o.eig_filter < 0 ||
        o.eig_filter > 200)
        return OSA_ERR_ARG;
    fill_defaults(o);
    c->opts = o;
    c->clear_graphs();
    return OSA_OK;
}

osa_status osa_create(osa_ctx** out, const osa_lattice* lat, const void* links, osa_prec link_prec,
                      double mu, double m_w, const osa_opts* opts, void* stream) {
    if (!out || !links) return OSA_ERR_ARG;
    *out = nullptr;
    if (validate_lattice(lat) != OSA_OK) return OSA_ERR_ARG;
    if (!(m_w > -2.0 && m_w < 0.0) || !std::isfinite(mu) || std::fabs(mu) > 50.0) return OSA_ERR_ARG;
    if (link_prec != OSA_FP64 && link_prec != OSA_FP32) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        std::unique_ptr<osa_ctx> c(new osa_ctx());
        c->st = (hipStream_t)stream;
        osa_status s = osa_set_opts(c.get(), opts);
        if (s != OSA_OK) return s;
        Geom& g = c->g;
        g.lx = lat->dims[0]; g.ly = lat->dims[1]; g.lz = lat->dims[2]; g.lt = lat->dims[3];
        g.V = g.lx * g.ly * g.lz * g.lt;
        g.Vp = (int)(ceil_div(g.V, 64) * 64);
        g.apt = lat->antiperiodic_t ? 1 : 0;
        c->links_fp32 = (link_prec == OSA_FP32);
        c->mu = mu;
        c->m_w = m_w;
        c->kappa = 1.0 / (8.0 + 2.0 * m_w);
        for (int nu = 0; nu < 3; ++nu) {
            c->hc.fwd[nu] = c->hc.bwd[nu] = -c->kappa;
            c->hc_adj.fwd[nu] = c->hc_adj.bwd[nu] = -c->kappa;
        }
        c->hc.fwd[3] = -c->kappa * std::exp(mu);
        c->hc.bwd[3] = -c->kappa * std::exp(-mu);
        c->hc_adj.fwd[3] = -c->kappa * std::exp(-mu);
        c->hc_adj.bwd[3] = -c->kappa * std::exp(mu);
        c->hnorm_bound = 1.0 + 2.0 * c->kappa * (3.0 + std::cosh(mu));
        const size_t lb = (size_t)g.Vp * 36 * (c->links_fp32 ? sizeof(cf) : sizeof(cd));
        c->U.ensure(lb);
        launch_links_to_internal(links, c->links_fp32, c->U.p, c->links_fp32, g, c->st);
        ensure_krylov(c.get(), c->opts.k_max);
        c->host.ensure(1 << 16);
        sync(c.get());
        *out = c.release();
        return OSA_OK;
    });
}

void osa_destroy(osa_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    delete c;
}

osa_status osa_deflate(osa_ctx* c, int32_t n_defl, osa_info* info) {
    if (!c) return OSA_ERR_ARG;
    if (n_defl < 0 || n_defl > 48 || (int64_t)n_defl >= 12LL * c->g.V) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        const double t0 = now_ms();
        try {
            deflate(c, n_defl, info, 0, 0, t0);
        } catch (const OsaError& e) {
            // with the default block, a hard spectrum gets one more run with the
            // largest block and twice the restart cap
            if (e.s != OSA_ERR_EIG_NOCONV || c->opts.eig_ncv > 0) throw;
            const int cap = c->opts.eig_max_restarts > 0 ? c->opts.eig_max_restarts : 2000;
            deflate(c, n_defl, info, 96, 2 * cap, t0);
        }
        return OSA_OK;
    }, &c->msg);
}

osa_status osa_set_deflation(osa_ctx* c, int32_t m, const void* R, const void* L,
                             const double* lambda) {
    if (!c || m < 0 || m > 64 || (int64_t)m >= 12LL * c->g.V) return OSA_ERR_ARG;
    if (m > 0 && (!R || !lambda || (!L && c->opts.deflation != 1))) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        const int64_t N = c->N();
        if (m == 0) { c->m_alloc = c->m_active = 0; c->lambda.clear(); return OSA_OK; }
        c->R.ensure(sizeof(cd) * (size_t)N * m);
        launch_vec_to_internal((const cd*)R, c->R.p, false, c->g, m, c->st);
        if (L) {
            c->L.ensure(sizeof(cd) * (size_t)N * m);
            launch_vec_to_internal((const cd*)L, c->L.p, false, c->g, m, c->st);
        }
        c->have_left = L != nullptr;
        c->schur_m = 0;
        c->lambda.resize(m);
        for (int i = 0; i < m; ++i) c->lambda[i] = mk(lambda[2 * i], lambda[2 * i + 1]);
        c->lam_dev.ensure(sizeof(cd) * m);
        h2d(c, c->lam_dev.p, c->lambda.data(), m);
        c->m_alloc = m;
        c->min_abs_re = INFINITY;
        for (auto& l : c->lambda) c->min_abs_re = std::min(c->min_abs_re, std::fabs(l.x));
        if (c->min_abs_re < 1e-12 * c->hnorm_bound) {
            c->m_alloc = c->m_active = 0;   // the solve then runs without deflation
            return OSA_ERR_IMAG_AXIS;
        }
        c->max_eig_resid = NAN;
        set_active(c, m);
        return OSA_OK;
    });
}

osa_status osa_get_deflation(const osa_ctx* cc, int32_t* m_out, void* R, void* L, double* lambda) {
    osa_ctx* c = const_cast<osa_ctx*>(cc);
    if (!c) return OSA_ERR_ARG;
    if (m_out) *m_out = c->m_alloc;
    return guard([&]() -> osa_status {
        const int m = c->m_alloc;
        if (m == 0) return OSA_OK;
        if (R) launch_vec_from_internal(c->R.p, false, (cd*)R, c->g, m, c->st);
        if (L && !c->have_left) return OSA_ERR_STATE;
        if (L) launch_vec_from_internal(c->L.p, false, (cd*)L, c->g, m, c->st);
        if (lambda)
            for (int i = 0; i < m; ++i) { lambda[2 * i] = c->lambda[i].x; lambda[2 * i + 1] = c->lambda[i].y; }
        sync(c);
        return OSA_OK;
    });
}

osa_status osa_set_active_deflation(osa_ctx* c, int32_t m) {
    if (!c || m < 0 || m > c->m_alloc) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        set_active(c, m);
        return OSA_OK;
    });
}

osa_status osa_apply(osa_ctx* c, int32_t nrhs, const void* B, void* Y, double tol,
                     osa_info* infos) {
    return apply_impl(c, nrhs, B, Y, tol, infos, ApplyMode::kSign);
}

osa_status osa_apply_adjoint(osa_ctx* c, int32_t nrhs, const void* B, void* Y, double tol,
                             osa_info* infos) {
    return apply_impl(c, nrhs, B, Y, tol, infos, ApplyMode::kAdjoint);
}

osa_status osa_apply_overlap(osa_ctx* c, int32_t nrhs, const void* B, void* Y, double tol,
                             osa_info* infos) {
    return apply_impl(c, nrhs, B, Y, tol, infos, ApplyMode::kOverlap);
}

osa_status osa_apply_block(osa_ctx* c, int32_t s, const void* B, void* Y, double tol,
                           int32_t k_blocks, osa_info* infos) {
    if (!c || s < 1 || s > kMaxBatch || !B || !Y || k_blocks < 0) return OSA_ERR_ARG;
    const bool fixed = c->opts.check_every < 0;
    if (!fixed && !(tol > 0)) return OSA_ERR_ARG;
    const int kb = k_blocks > 0 ? k_blocks : std::max(1, (int)ceil_div(4LL * c->opts.k_max, s));
    if ((int64_t)kb * s > 6000 || (int64_t)(kb + 1) * s > 12LL * c->g.V) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        const int64_t N = c->N();
        const int64_t nbnd = 12LL * c->g.V;
        const double t0 = now_ms();
        c->xio.ensure(sizeof(cd) * N * s);
        c->yio.ensure(sizeof(cd) * N * s);
        launch_vec_to_internal((const cd*)B, c->xio.p, false, c->g, s, c->st);
        BlockResult r;
        std::vector<double> est(s, NAN);
        solve_block(c, s, c->xio.as<cd>(), c->yio.as<cd>(), tol, kb, r, est);
        launch_vec_from_internal(c->yio.p, false, (cd*)Y, c->g, s, c->st);
        sync(c);
        const double t1 = now_ms();
        if (infos) {
            for (int b = 0; b < s; ++b) {
                osa_info& in = infos[b];
                std::memset(&in, 0, sizeof(in));
                in.resid_est = fixed ? NAN : est[b];
                in.k_used = r.dim;
                in.n_defl = c->m_active;
                in.status = r.st;
                in.newton_iters = r.newton_iters;
                in.breakdown = r.breakdown;
                in.min_abs_re_lambda = c->m_active ? c->min_abs_re : NAN;
                in.max_eig_resid = c->max_eig_resid;
                in.t_init_ms = c->t_init_ms;
                in.t_solve_ms = t1 - t0;
                in.batch = s;
            }
        }
        (void)nbnd;
        return r.st;
    }, &c->msg);
}

osa_status osa_batch_apply(int32_t n, osa_ctx* const* ctxs, const void* const* B, void* const* Y,
                           double tol, osa_info* infos) {
    if (n < 1 || !ctxs || !B || !Y) return OSA_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !B[i] || !Y[i]) return OSA_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return OSA_ERR_ARG;   // one context cannot run twice at once
    }
    // Independent instances (each its own operator, lattice and deflation data)
    // run concurrently: a pool of host workers, each driving one context at a
    // time on a stream of its own that first waits for the work queued on the
    // context's stream.  Every instance computes exactly what osa_apply computes.
    const int nw = std::min<int>(n, kBatchWorkers);
    std::vector<hipStream_t> streams(nw, nullptr);
    std::vector<osa_status> st(n, OSA_OK);
    std::atomic<int> next{0};
    osa_status setup = OSA_OK;
    for (int w = 0; w < nw && setup == OSA_OK; ++w)
        if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            setup = OSA_ERR_HIP;
        }
    if (setup == OSA_OK) {
        auto work = [&](int w) {
            hipEvent_t ev = nullptr;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                ev = nullptr;
            }
            for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
                osa_ctx* c = ctxs[i];
                if (!ev || hipEventRecord(ev, c->st) != hipSuccess ||
                    hipStreamWaitEvent(streams[w], ev, 0) != hipSuccess) {
                    (void)hipGetLastError();
                    st[i] = OSA_ERR_HIP;
                    continue;
                }
                hipStream_t own = c->st;
                c->st = streams[w];
                st[i] = osa_apply(c, 1, B[i], Y[i], tol, infos ? infos + i : nullptr);
                c->st = own;   // osa_apply has synchronised the worker stream
            }
            if (ev) (void)hipEventDestroy(ev);
        };
        std::vector<std::thread> pool;
        for (int w = 1; w < nw; ++w) pool.emplace_back(work, w);
        work(0);
        for (auto& t : pool) t.join();
    }
    for (auto s2 : streams)
        if (s2) (void)hipStreamDestroy(s2);
    if (setup != OSA_OK) return setup;
    osa_status worst = OSA_OK;
    for (int i = 0; i < n; ++i) {
        if (st[i] < 0) return st[i];
        if (st[i] > worst) worst = st[i];
    }
    return worst;
}

osa_status osa_set_links(osa_ctx* c, const void* links) {
    if (!c || !links) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        launch_links_to_internal(links, c->links_fp32, c->U.p, c->links_fp32, c->g, c->st);
        if (c->U32.p) launch_convert(c->U.p, false, c->U32.p, true, (int64_t)c->g.Vp * 36, c->st);
        c->m_alloc = c->m_active = 0;
        c->lambda.clear();
        sync(c);
        return OSA_OK;
    });
}

osa_status osa_profile_enable(osa_ctx* c, int32_t every) {
    if (!c) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        sync(c);
        c->prof = osa_profile{};
        c->prof_on = every > 0;
        c->prof_every = every > 0 ? every : 1;
        return OSA_OK;
    });
}

osa_status osa_profile_read(osa_ctx* c, osa_profile* out) {
    if (!c || !out) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        sync(c);
        *out = c->prof;
        return OSA_OK;
    });
}

osa_status osa_apply_hw(osa_ctx* c, int32_t nrhs, const void* X, void* Y) {
    if (!c || nrhs < 1 || !X || !Y) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        const int64_t N = c->N();
        DevBuf a, b;
        a.ensure(sizeof(cd) * N * nrhs);
        b.ensure(sizeof(cd) * N * nrhs);
        launch_vec_to_internal((const cd*)X, a.p, false, c->g, nrhs, c->st);
        apply_h_contig(c, a.p, b.p, false, false, nrhs);
        launch_vec_from_internal(b.p, false, (cd*)Y, c->g, nrhs, c->st);
        sync(c);
        return OSA_OK;
    });
}

osa_status osa_apply_hw32(osa_ctx* c, int32_t nrhs, const void* X, void* Y) {
    if (!c || nrhs < 1 || !X || !Y) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        if (!c->links()) throw OsaError{OSA_ERR_STATE, "no links set"};
        const int64_t N = c->N();
        const int64_t nb = 12LL * c->g.V * nrhs;   // boundary-layout entries
        ensure_links32(c);
        DevBuf t, a, b;
        t.ensure(sizeof(cd) * (size_t)nb);
        a.ensure(sizeof(cf) * (size_t)N * nrhs);
        b.ensure(sizeof(cf) * (size_t)N * nrhs);
        // complex64 -> complex128 (exact) -> internal complex64 (exact)
        launch_convert(X, true, t.p, false, nb, c->st);
        launch_vec_to_internal(t.as<cd>(), a.p, true, c->g, nrhs, c->st);
        apply_h_contig(c, a.p, b.p, true, false, nrhs);
        launch_vec_from_internal(b.p, true, t.as<cd>(), c->g, nrhs, c->st);
        launch_convert(t.p, false, Y, true, nb, c->st);
        sync(c);
        return OSA_OK;
    });
}

osa_status osa_krylov_h2(osa_ctx* c, int32_t prec, int32_t adjoint, int32_t k, const void* x,
                         void* Vout, void* Sout) {
    if (!c || (prec != OSA_FP64 && prec != OSA_FP32) || k < 1 || k > 64 || !x || !Vout ||
        !Sout)
        return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        if (!c->links()) throw OsaError{OSA_ERR_STATE, "no links set"};
        if ((int64_t)k + 1 > 12LL * c->g.V) throw OsaError{OSA_ERR_ARG, "k + 1 exceeds N"};
        const bool fp32 = prec == OSA_FP32;
        const int64_t N = c->N();
        const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
        if (fp32) ensure_links32(c);
        ensure_exec(c, k + 2);
        const int ldS = k + 1;
        DevBuf Vb, wv, tv, S, d;
        Vb.ensure(es * (size_t)N * (k + 1));
        wv.ensure(es * (size_t)N);
        tv.ensure(es * (size_t)N);
        S.ensure(sizeof(cd) * (size_t)ldS * (k + 1));
        d.ensure(sizeof(cd) * 2 * (size_t)(k + 2));
        launch_fill_zero(S.p, sizeof(cd) * (size_t)ldS * (k + 1), c->st);
        double* hfro2 = (double*)(c->dscal.as<cd>() + 8);
        launch_fill_zero(hfro2, sizeof(double), c->st);
        launch_fill_zero(c->flag.p, sizeof(int) * 4, c->st);
        const TsPlan pl = ts_plan(N);
        launch_vec_to_internal((const cd*)x, Vb.p, fp32, c->g, 1, c->st);
        launch_norm_partial(Vb.p, fp32, pl, c->normp.as<double>(), c->st);
        launch_normalize(Vb.p, Vb.p, fp32, pl, c->normp.as<double>(), c->dscal.as<cd>() + 9,
                         nullptr, 0.0, nullptr, 0, nullptr, 0, c->st);
        KsStats st;
        expand_delayed(c, adjoint != 0, fp32, (char*)Vb.p, N, S.as<cd>(), ldS, 0, k, wv.p, tv.p,
                       d.as<cd>(), hfro2, c->flag.as<int>(), st);
        launch_vec_from_internal(Vb.p, fp32, (cd*)Vout, c->g, k + 1, c->st);
        OSA_HIP(hipMemcpyAsync(Sout, S.p, sizeof(cd) * (size_t)ldS * k, hipMemcpyDeviceToDevice,
                               c->st));
        int hf = 0;
        d2h(c, c->flag.p, 1, &hf);
        if (hf == 2) throw OsaError{OSA_ERR_NONFINITE, "non-finite Arnoldi vector"};
        return OSA_OK;
    });
}

osa_status osa_small_sign(int32_t k, const void* A, void* s, int32_t* iters, void* stream) {
    if (k < 1 || k > 4000 || !A || !s) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        osa_ctx c;
        c.st = (hipStream_t)stream;
        c.g.lx = c.g.ly = c.g.lz = c.g.lt = 2;
        c.g.V = 16;
        c.g.Vp = 64;
        c.host.ensure(1 << 16);
        c.kcap = k;
        c.scap = k;
        c.kbatch = 1;
        c.sX.ensure(sizeof(cd) * (size_t)k * k);
        c.sM.ensure(sizeof(cd) * (size_t)k * k);
        c.sY.ensure(sizeof(cd) * (size_t)k * k);
        c.logpiv.ensure(sizeof(double) * k);
        c.gj_stride = (int64_t)ceil_div((int64_t)gj_ws_bytes(k), 256) * 256;
        c.gjws.ensure((size_t)c.gj_stride);
        c.nflag.ensure(sizeof(int) * 4);
        c.red_stride = newton_red_len(k) + 16;
        c.red.ensure(sizeof(double) * (size_t)c.red_stride);
        std::vector<int> its(1, 0);
        std::vector<char> ok(1, 0);
        small_sign_batch(&c, std::vector<int>{0}, k, (const cd*)A, k, 0, (cd*)s, 0, its, ok);
        sync(&c);
        if (iters) *iters = its[0];
        if (its[0] < 0 || !ok[0]) return OSA_ERR_NEWTON_NOCONV;
        return OSA_OK;
    });
}

osa_status osa_small_gemm(int32_t n, int32_t nb, const void* A, const void* B, void* C,
                          void* stream) {
    if (n < 1 || n > 4000 || nb < 1 || nb > kMaxBatch || !A || !B || !C) return OSA_ERR_ARG;
    const size_t bytes = sizeof(cd) * (size_t)n * n * nb;
    auto overlap = [&](const void* p, const void* q) {
        return (const char*)p < (const char*)q + bytes && (const char*)q < (const char*)p + bytes;
    };
    if (overlap(C, A) || overlap(C, B)) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        Batch bt;
        bt.n = nb;
        bt.mat = (int64_t)n * n;
        launch_zgemm_sq(n, mk(1.0, 0.0), (const cd*)A, (const cd*)B, 0.0, nullptr, 0.0, (cd*)C,
                        nullptr, nullptr, (hipStream_t)stream, bt);
        OSA_HIP(hipStreamSynchronize((hipStream_t)stream));
        return OSA_OK;
    });
}

osa_status osa_small_sign_noalloc(int32_t k, const void* A, void* s, int32_t* iters,
                                  void* stream) {
    if (k < 1 || !A || !s) return OSA_ERR_ARG;
    if (k > OSA_NOALLOC_MAX_K) return OSA_ERR_ARG;   // the scratch array holds k <= 256
    return guard([&]() -> osa_status {
        char* base = (char*)noalloc_scratch();
        // carve the workspace of one problem of size k, with the strides
        // osa_small_sign uses, so both run the same launches on the same layout
        const size_t mat = sizeof(cd) * (size_t)k * k;
        const int64_t gj_stride = (int64_t)ceil_div((int64_t)gj_ws_bytes(k), 256) * 256;
        const int64_t red_stride = newton_red_len(k) + 16;
        size_t off = 0;
        auto take = [&](size_t b) {
            char* q = base + off;
            off += (size_t)ceil_div((int64_t)b, 256) * 256;
            return q;
        };
        osa_ctx c;
        c.st = (hipStream_t)stream;
        c.g.lx = c.g.ly = c.g.lz = c.g.lt = 2;
        c.g.V = 16;
        c.g.Vp = 64;
        c.kcap = k;
        c.scap = k;
        c.kbatch = 1;
        c.gj_stride = gj_stride;
        c.red_stride = red_stride;
        c.sX.borrow(take(mat), mat);
        c.sM.borrow(take(mat), mat);
        c.sY.borrow(take(mat), mat);
        c.logpiv.borrow(take(sizeof(double) * k), sizeof(double) * k);
        c.gjws.borrow(take((size_t)gj_stride), (size_t)gj_stride);
        c.nflag.borrow(take(sizeof(int) * 4), sizeof(int) * 4);
        c.red.borrow(take(sizeof(double) * (size_t)red_stride), sizeof(double) * (size_t)red_stride);
        if (off > kNoallocScratchBytes) throw OsaError{OSA_ERR_ARG, "scratch too small"};
        thread_local char staging[1 << 12];   // ordinary host memory for the read-backs
        c.host.borrow(staging, sizeof staging);
        std::vector<int> its(1, 0);
        std::vector<char> ok(1, 0);
        small_sign_batch(&c, std::vector<int>{0}, k, (const cd*)A, k, 0, (cd*)s, 0, its, ok);
        sync(&c);
        if (iters) *iters = its[0];
        if (its[0] < 0 || !ok[0]) return OSA_ERR_NEWTON_NOCONV;
        return OSA_OK;
    });
}

osa_status osa_small_schur(int32_t p, const void* A, void* T, void* Z, void* w, int32_t mode,
                           void* stream) {
    if (p < 1 || p > 96 || !A || !T || !Z || !w || (mode != 0 && mode != 1)) return OSA_ERR_ARG;
    return guard([&]() -> osa_status {
        hipStream_t st = (hipStream_t)stream;
        DevBuf info, ws;
        info.ensure(sizeof(int) * 4);
        if (p > 64) ws.ensure(schur_ws_bytes(p));
        small_schur((const cd*)A, p, (cd*)T, (cd*)Z, (cd*)w, mode, info.as<int>(), ws.p, st);
        int h = 0;
        OSA_HIP(hipMemcpyAsync(&h, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
        OSA_HIP(hipStreamSynchronize(st));
        return h < 0 ? OSA_ERR_EIG_NOCONV : OSA_OK;
    });
}

osa_status overlap_sign_apply(const osa_lattice* lat, const void* links, osa_prec link_prec,
                              double mu, double m_w, const void* source, double tol,
                              int32_t n_defl, void* result, double* resid_est, void* stream) {
    if (!source || !result || !(tol > 0) || n_defl < 0 || source == result) return OSA_ERR_ARG;
    osa_ctx* c = nullptr;
    osa_status s = osa_create(&c, lat, links, link_prec, mu, m_w, nullptr, stream);
    if (s != OSA_OK) return s;
    s = osa_deflate(c, n_defl, nullptr);
    osa_info info{};
    if (s == OSA_OK) s = osa_apply(c, 1, source, result, tol, &info);
    if (resid_est) *resid_est = info.resid_est;
    osa_destroy(c);
    return s;
}

}  // extern "C"
