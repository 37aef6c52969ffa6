// Tall-skinny complex kernels for the Arnoldi recurrence (Eq. 7), the LR
// projection (Eq. 21) and the final assembly (Eq. 22).
//
// All reductions are two-stage with a fixed order (per-block partial sums, then
// one sequential sum per output), so results are bitwise reproducible run to
// run.  Vectors are stored as complex128 (double2) or complex64 (float2);
// every accumulation is in double.
//
// Every kernel takes a Batch: one grid axis runs over the problems of the
// batch, and each array argument is offset by the problem's stride.  The
// arithmetic of one problem does not depend on the batch it runs in.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace osa {

static constexpr int kBlock = 256;
static constexpr int kWaves = kBlock / 64;
// Workgroups of a launch are dealt to the 8 XCDs (each with its own L2) in turn.
static constexpr int kXcds = 8;

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV doubles over the block; results valid in sm_out[0..NV) after return.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sm /* kWaves*NV */,
                                          double* sm_out /* NV */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = wave_sum(v[i]);
        if (lane == 0) sm[wave * NV + i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NV; i += kBlock) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += sm[w * NV + i];
        sm_out[i] = s;
    }
    __syncthreads();
}

// Row chunks of a dot launch: 64 chunks while that gives at least 1024 blocks
// of (chunk x 8 columns); beyond about 128 columns, fewer and longer chunks so
// the launch stays near 1024 blocks (measured at 8^4: more rows per thread
// helps the long bases of the solve, 64 chunks suit the short eigensolver
// ones).  Depends on n and ncols only (never on a batch), so a problem's
// summation order is fixed.
static TsPlan dot_plan(int64_t n, int ncols, int C) {
    const int64_t groups = ceil_div(ncols > 0 ? ncols : 1, C);
    int64_t want = ceil_div(1024, groups);
    if (want > 64) want = 64;
    if (want < 8) want = 8;
    TsPlan p;
    p.n = n;
    int64_t rpc = ceil_div(ceil_div(n, want), kBlock) * kBlock;
    if (rpc < kBlock) rpc = kBlock;
    p.rows_per_chunk = (int)rpc;
    p.nchunks = (int)ceil_div(n, rpc);
    return p;
}

// ----------------------------------------------------------------- autotuner
// The row chunking of the dot kernels (k_dot_partial, k_dot2_partial,
// k_mdot_partial) is picked by measurement: at the first launch with a given
// length n and column bucket ceil(ncols / 32) the launcher times each candidate
// chunk count (8 ... 128 chunks, and the built-in choice) on the call's own
// operands (the dot kernels only read them), keeps the fastest, and every later
// launch with that (n, bucket), by any dot kernel, any batch and any thread of
// the process, uses it.  A problem's summation order therefore depends on
// (n, ncols) alone within a process, which keeps batched results bitwise those
// of single-source solves.  Off (osa_set_autotune(0)), or while the stream is
// being captured into a graph, the built-in choice is used for new keys.
namespace {
struct TuneKey {
    int64_t n;
    int bucket;
    bool operator<(const TuneKey& o) const { return n < o.n || (n == o.n && bucket < o.bucket); }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;          // (n, bucket) -> chunk count target
std::atomic<int> g_tune_on{1};
}  // namespace

void set_autotune(bool on) { g_tune_on.store(on ? 1 : 0); }
bool autotune_enabled() { return g_tune_on.load() != 0; }

int autotune_entries(int64_t* n, int* bucket, int* want, int cap) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int i = 0;
    for (const auto& kv : g_tune) {
        if (i < cap) {
            if (n) n[i] = kv.first.n;
            if (bucket) bucket[i] = kv.first.bucket;
            if (want) want[i] = kv.second;
        }
        ++i;
    }
    return i;
}

static TsPlan plan_for_want(int64_t n, int64_t want) {
    TsPlan p;
    p.n = n;
    int64_t rpc = ceil_div(ceil_div(n, want), kBlock) * kBlock;
    if (rpc < kBlock) rpc = kBlock;
    p.rows_per_chunk = (int)rpc;
    p.nchunks = (int)ceil_div(n, rpc);
    return p;
}

// The plan of a dot launch; with the autotuner on and a new (n, bucket), first
// times launch(candidate plan) for every candidate on stream st.
template <typename F>
static TsPlan tuned_plan(int64_t n, int ncols, int C, hipStream_t st, F&& launch) {
    const TsPlan def = dot_plan(n, ncols, C);
    const TuneKey key{n, (int)ceil_div(ncols > 0 ? ncols : 1, 32)};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return plan_for_want(n, it->second);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!g_tune_on.load() || hipStreamIsCapturing(st, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return def;
    }
    // at most kMaxChunks / 2 chunks, as the built-in choice: the two-vector dot
    // writes 2 ncols partials per chunk into buffers sized ncols x kMaxChunks
    std::vector<int> cands = {def.nchunks};
    for (int w : {8, 16, 32, 48, 64})
        if (std::find(cands.begin(), cands.end(), w) == cands.end()) cands.push_back(w);
    hipEvent_t e0, e1;
    OSA_HIP(hipEventCreate(&e0));
    OSA_HIP(hipEventCreate(&e1));
    int best = def.nchunks;
    float best_ms = 1e30f;
    for (int w : cands) {
        const TsPlan p = plan_for_want(n, w);
        if (p.nchunks > kMaxChunks / 2) continue;
        launch(p);   // warm
        OSA_HIP(hipEventRecord(e0, st));
        launch(p);
        launch(p);
        OSA_HIP(hipEventRecord(e1, st));
        OSA_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        OSA_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; best = w; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_tune[key] = best;
    return plan_for_want(n, best);
}

TsPlan ts_plan(int64_t n) {
    TsPlan p;
    p.n = n;
    // about 64 chunks, each a multiple of the block size
    int64_t rpc = ceil_div(ceil_div(n, 64), kBlock) * kBlock;
    if (rpc < kBlock) rpc = kBlock;
    p.rows_per_chunk = (int)rpc;
    p.nchunks = (int)ceil_div(n, rpc);
    return p;
}

// ---------------------------------------------------------------- dot
template <typename T, int C>
__global__ __launch_bounds__(kBlock) void k_dot_partial(const T* __restrict__ B, int64_t ldb,
                                                        int ncols, const T* __restrict__ w,
                                                        int64_t n, int rpc, int nchunks,
                                                        cd* __restrict__ partial, Batch bt) {
    __shared__ double sm[kWaves * 2 * C];
    __shared__ double so[2 * C];
    const int pb = bt.idx[blockIdx.z];
    B += pb * bt.basis;
    w += pb * bt.vec;
    partial += pb * bt.part;
    const int q = blockIdx.x;
    const int c0 = blockIdx.y * C;
    const int64_t r0 = (int64_t)q * rpc;
    const int64_t r1 = (r0 + rpc < n) ? r0 + rpc : n;
    double acc[2 * C];
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) acc[i] = 0.0;
    const int nc = (ncols - c0 < C) ? ncols - c0 : C;
    if (nc == C) {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            const cd wi = tod(w[i]);
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                const cd b = tod(B[(int64_t)(c0 + cc) * ldb + i]);
                acc[2 * cc] = fma(b.x, wi.x, fma(b.y, wi.y, acc[2 * cc]));
                acc[2 * cc + 1] = fma(b.x, wi.y, fma(-b.y, wi.x, acc[2 * cc + 1]));
            }
        }
    } else {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            const cd wi = tod(w[i]);
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                if (cc < nc) {
                    const cd b = tod(B[(int64_t)(c0 + cc) * ldb + i]);
                    acc[2 * cc] = fma(b.x, wi.x, fma(b.y, wi.y, acc[2 * cc]));
                    acc[2 * cc + 1] = fma(b.x, wi.y, fma(-b.y, wi.x, acc[2 * cc + 1]));
                }
            }
        }
    }
    block_sum<2 * C>(acc, sm, so);
    if (threadIdx.x < nc) partial[(int64_t)(c0 + threadIdx.x) * nchunks + q] =
        mk(so[2 * threadIdx.x], so[2 * threadIdx.x + 1]);
}

int launch_dot_partial(const void* B, int64_t ldb, int ncols, const void* w, bool fp32,
                       const TsPlan& pn, cd* partial, hipStream_t st, const Batch& bt) {
    constexpr int C = 8;
    if (ncols <= 0 || bt.n <= 0) return dot_plan(pn.n, ncols, C).nchunks;
    auto go = [&](const TsPlan& p) {
        dim3 grid((unsigned)p.nchunks, (unsigned)ceil_div(ncols, C), (unsigned)bt.n), blk(kBlock);
        if (fp32)
            hipLaunchKernelGGL((k_dot_partial<cf, C>), grid, blk, 0, st, (const cf*)B, ldb, ncols,
                               (const cf*)w, p.n, p.rows_per_chunk, p.nchunks, partial, bt);
        else
            hipLaunchKernelGGL((k_dot_partial<cd, C>), grid, blk, 0, st, (const cd*)B, ldb, ncols,
                               (const cd*)w, p.n, p.rows_per_chunk, p.nchunks, partial, bt);
        OSA_LAUNCH_CHECK();
    };
    const TsPlan p = tuned_plan(pn.n, ncols, C, st, go);
    go(p);
    return p.nchunks;
}

// Two vectors against the same columns (one read of B): partial[c*nchunks + q]
// for w1 and partial[(ncols + c)*nchunks + q] for w2.  The chunk's rows of w1,
// w2 are read by every column group: XCD x takes a contiguous run of (chunk,
// column group) items, column group fastest, so those re-reads stay in its L2.
template <typename T, int C>
__global__ __launch_bounds__(kBlock) void k_dot2_partial(const T* __restrict__ B, int64_t ldb,
                                                         int ncols, const T* __restrict__ w1,
                                                         const T* __restrict__ w2, int64_t n,
                                                         int rpc, int nchunks, int ngroups,
                                                         int per_xcd, cd* __restrict__ partial,
                                                         Batch bt) {
    __shared__ double sm[kWaves * 4 * C];
    __shared__ double so[4 * C];
    const int item = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    if (item >= nchunks * ngroups) return;   // whole block: before any barrier
    const int pb = bt.idx[blockIdx.z];
    B += pb * bt.basis;
    w1 += pb * bt.basis;
    w2 += pb * bt.vec;
    partial += pb * bt.part;
    const int q = item / ngroups;
    const int c0 = (item % ngroups) * C;
    const int64_t r0 = (int64_t)q * rpc;
    const int64_t r1 = (r0 + rpc < n) ? r0 + rpc : n;
    double acc[4 * C];
#pragma unroll
    for (int i = 0; i < 4 * C; ++i) acc[i] = 0.0;
    const int nc = (ncols - c0 < C) ? ncols - c0 : C;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const cd a = tod(w1[i]), b2 = tod(w2[i]);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
            if (cc < nc) {
                const cd v = tod(B[(int64_t)(c0 + cc) * ldb + i]);
                acc[4 * cc] = fma(v.x, a.x, fma(v.y, a.y, acc[4 * cc]));
                acc[4 * cc + 1] = fma(v.x, a.y, fma(-v.y, a.x, acc[4 * cc + 1]));
                acc[4 * cc + 2] = fma(v.x, b2.x, fma(v.y, b2.y, acc[4 * cc + 2]));
                acc[4 * cc + 3] = fma(v.x, b2.y, fma(-v.y, b2.x, acc[4 * cc + 3]));
            }
        }
    }
    block_sum<4 * C>(acc, sm, so);
    if (threadIdx.x < nc) {
        const int c = c0 + threadIdx.x;
        partial[(int64_t)c * nchunks + q] = mk(so[4 * threadIdx.x], so[4 * threadIdx.x + 1]);
        partial[(int64_t)(ncols + c) * nchunks + q] =
            mk(so[4 * threadIdx.x + 2], so[4 * threadIdx.x + 3]);
    }
}

int launch_dot2_partial(const void* B, int64_t ldb, int ncols, const void* w1, const void* w2,
                        bool fp32, const TsPlan& pn, cd* partial, hipStream_t st, const Batch& bt) {
    constexpr int C = 8;
    if (ncols <= 0 || bt.n <= 0) return dot_plan(pn.n, ncols, C).nchunks;
    auto go = [&](const TsPlan& p) {
        const int ngroups = (int)ceil_div(ncols, C);
        const int per_xcd = (int)ceil_div((int64_t)p.nchunks * ngroups, kXcds);
        dim3 grid((unsigned)(kXcds * per_xcd), 1, (unsigned)bt.n), blk(kBlock);
        if (fp32)
            hipLaunchKernelGGL((k_dot2_partial<cf, C>), grid, blk, 0, st, (const cf*)B, ldb, ncols,
                               (const cf*)w1, (const cf*)w2, p.n, p.rows_per_chunk, p.nchunks,
                               ngroups, per_xcd, partial, bt);
        else
            hipLaunchKernelGGL((k_dot2_partial<cd, C>), grid, blk, 0, st, (const cd*)B, ldb, ncols,
                               (const cd*)w1, (const cd*)w2, p.n, p.rows_per_chunk, p.nchunks,
                               ngroups, per_xcd, partial, bt);
        OSA_LAUNCH_CHECK();
    };
    const TsPlan p = tuned_plan(pn.n, ncols, C, st, go);
    go(p);
    return p.nchunks;
}

// ---------------------------------------------------------------- reduce
// val[c] = sum_q partial[c*nchunks + q], one wavefront per column (lane q holds
// chunk q, q + 64, ...; fixed shuffle tree, so the order never changes).
// out[c] = val (set); accum[c] += val when accum != nullptr.
__global__ __launch_bounds__(256) void k_reduce_cols(const cd* __restrict__ partial, int nchunks,
                                                     int ncols, cd* __restrict__ out,
                                                     cd* __restrict__ accum, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    partial += pb * bt.part;
    out += pb * bt.small;
    if (accum) accum += pb * bt.small;
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= ncols) return;
    double re = 0, im = 0;
    for (int q = lane; q < nchunks; q += 64) {
        const cd v = partial[(int64_t)c * nchunks + q];
        re += v.x;
        im += v.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        out[c] = mk(re, im);
        if (accum) accum[c] = mk(accum[c].x + re, accum[c].y + im);
    }
}

// One block per problem: val = sum over chunks, then out = M val (M: ncols x
// ncols, used for G^{-1} L^dag w with the small m x m matrix G^{-1}).
__global__ __launch_bounds__(kBlock) void k_reduce_apply(const cd* __restrict__ partial,
                                                         int nchunks, int ncols, cd* out,
                                                         const cd* __restrict__ M, cd* tmp,
                                                         Batch bt) {
    const int pb = bt.idx[blockIdx.x];
    partial += pb * bt.part;
    out += pb * bt.small;
    tmp += pb * bt.small;
    // a wave per column: lane l sums chunks l, l + 64, ..., then a butterfly
    // over the lanes (an order fixed by nchunks)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = wave; c < ncols; c += kWaves) {
        double sr = 0.0, si = 0.0;
        for (int q = lane; q < nchunks; q += 64) {
            const cd v = partial[(int64_t)c * nchunks + q];
            sr += v.x;
            si += v.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) tmp[c] = mk(sr, si);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncols; c += kBlock) {
        cd s = mk(0.0, 0.0);
        for (int d = 0; d < ncols; ++d) cfma(s, M[c + (int64_t)d * ncols], tmp[d]);
        out[c] = s;
    }
}

void launch_reduce_partial(const cd* partial, int nchunks, int ncols, cd* out, cd* accum,
                           const cd* M, cd* tmp, hipStream_t st, const Batch& bt) {
    if (ncols <= 0 || bt.n <= 0) return;
    if (M) {
        hipLaunchKernelGGL(k_reduce_apply, dim3((unsigned)bt.n), dim3(kBlock), 0, st, partial,
                           nchunks, ncols, out, M, tmp, bt);
    } else {
        hipLaunchKernelGGL(k_reduce_cols, dim3((unsigned)ceil_div(ncols, 4), (unsigned)bt.n),
                           dim3(256), 0, st, partial, nchunks, ncols, out, accum, bt);
    }
    OSA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- update
// w[i] = alpha*w[i] - sum_{c in group} B[c][i] coef[c]; the column loop is split
// into G groups writing to scratch when the row count alone cannot fill the GPU.
static constexpr int kCoefTile = 256;

template <typename T>
__device__ __forceinline__ cd gemv_rows(const T* __restrict__ B, int64_t ldb, int cbeg, int cend,
                                        const cd* __restrict__ coef, int64_t i, cd* scoef) {
    cd acc = mk(0.0, 0.0);
    for (int cb = cbeg; cb < cend; cb += kCoefTile) {
        const int ce = (cb + kCoefTile < cend) ? cb + kCoefTile : cend;
        __syncthreads();
        for (int c = cb + (int)threadIdx.x; c < ce; c += kBlock) scoef[c - cb] = coef[c];
        __syncthreads();
        int c = cb;
        for (; c + 4 <= ce; c += 4) {
            const cd b0 = tod(B[(int64_t)(c + 0) * ldb + i]);
            const cd b1 = tod(B[(int64_t)(c + 1) * ldb + i]);
            const cd b2 = tod(B[(int64_t)(c + 2) * ldb + i]);
            const cd b3 = tod(B[(int64_t)(c + 3) * ldb + i]);
            cfma(acc, b0, scoef[c - cb + 0]);
            cfma(acc, b1, scoef[c - cb + 1]);
            cfma(acc, b2, scoef[c - cb + 2]);
            cfma(acc, b3, scoef[c - cb + 3]);
        }
        for (; c < ce; ++c) cfma(acc, tod(B[(int64_t)c * ldb + i]), scoef[c - cb]);
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_direct(T* w, const T* __restrict__ B,
                                                          int64_t ldb, int ncols,
                                                          const cd* __restrict__ coef, int64_t n,
                                                          double alpha, double sgn,
                                                          double* normp, Batch bt) {
    __shared__ cd scoef[kCoefTile];
    __shared__ double sm[kWaves];
    __shared__ double so[1];
    const int pb = bt.idx[blockIdx.y];
    w += pb * bt.vec;
    B += pb * bt.basis;
    coef += pb * bt.small;
    if (normp) normp += pb * bt.part;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ii = (i < n) ? i : n - 1;   // keep every thread in the barriers
    cd acc = gemv_rows(B, ldb, 0, ncols, coef, ii, scoef);
    cd v = mk(0.0, 0.0);
    if (i < n) {
        cd base = (alpha != 0.0) ? cscale(tod(w[i]), alpha) : mk(0.0, 0.0);
        v = mk(base.x + sgn * acc.x, base.y + sgn * acc.y);
        w[i] = fromd<T>(v);
    }
    if (normp) {
        cd vr = tod(fromd<T>(v));
        double nv[1] = {(i < n) ? cabs2(vr) : 0.0};
        block_sum<1>(nv, sm, so);
        if (threadIdx.x == 0) normp[blockIdx.x] = so[0];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_split(const T* __restrict__ B, int64_t ldb,
                                                         int ncols, const cd* __restrict__ coef,
                                                         int64_t n, int cpg,
                                                         cd* __restrict__ scratch, int G,
                                                         Batch bt) {
    __shared__ cd scoef[kCoefTile];
    const int pb = bt.idx[blockIdx.z];
    B += pb * bt.basis;
    coef += pb * bt.small;
    scratch += (int64_t)blockIdx.z * G * n;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ii = (i < n) ? i : n - 1;
    const int g = blockIdx.y;
    const int cb = g * cpg;
    const int ce = (cb + cpg < ncols) ? cb + cpg : ncols;
    cd acc = gemv_rows(B, ldb, cb, ce, coef, ii, scoef);
    if (i < n) scratch[(int64_t)g * n + i] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_finish(T* w, const cd* __restrict__ scratch,
                                                          int G, int64_t n, double alpha,
                                                          double sgn, double* normp, Batch bt) {
    __shared__ double sm[kWaves];
    __shared__ double so[1];
    const int pb = bt.idx[blockIdx.y];
    w += pb * bt.vec;
    if (normp) normp += pb * bt.part;
    scratch += (int64_t)blockIdx.y * G * n;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    cd v = mk(0.0, 0.0);
    if (i < n) {
        cd acc = mk(0.0, 0.0);
        for (int g = 0; g < G; ++g) acc = cadd(acc, scratch[(int64_t)g * n + i]);
        cd base = (alpha != 0.0) ? cscale(tod(w[i]), alpha) : mk(0.0, 0.0);
        v = mk(base.x + sgn * acc.x, base.y + sgn * acc.y);
        w[i] = fromd<T>(v);
    }
    if (normp) {
        cd vr = tod(fromd<T>(v));
        double nv[1] = {(i < n) ? cabs2(vr) : 0.0};
        block_sum<1>(nv, sm, so);
        if (threadIdx.x == 0) normp[blockIdx.x] = so[0];
    }
}

template <typename T>
static void update_impl(T* w, const T* B, int64_t ldb, int ncols, const cd* coef, int64_t n,
                        double alpha, double sgn, double* normp, cd* scratch,
                        int64_t scratch_len, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const int rb = (int)ceil_div(n, kBlock);
    // The split depends on the row count and the column count only, not on the
    // batch, so a problem gets the same summation order in any batch (the
    // caller sizes scratch to 8 n per problem).
    int G = 1;
    if (ncols > 32 && rb < 1024 && scratch) {
        G = (int)ceil_div(1024, rb);
        int gmax = ncols / 16;
        if (G > gmax) G = gmax;
        if (G > 8) G = 8;
        while (G > 1 && (int64_t)G * n * bt.n > scratch_len) --G;
    }
    if (G <= 1) {
        hipLaunchKernelGGL((k_update_direct<T>), dim3(rb, bt.n), dim3(kBlock), 0, st, w, B, ldb,
                           ncols, coef, n, alpha, sgn, normp, bt);
    } else {
        const int cpg = (int)ceil_div(ncols, G);
        G = (int)ceil_div(ncols, cpg);
        hipLaunchKernelGGL((k_update_split<T>), dim3(rb, G, bt.n), dim3(kBlock), 0, st, B, ldb,
                           ncols, coef, n, cpg, scratch, G, bt);
        hipLaunchKernelGGL((k_update_finish<T>), dim3(rb, bt.n), dim3(kBlock), 0, st, w,
                           (const cd*)scratch, G, n, alpha, sgn, normp, bt);
    }
    OSA_LAUNCH_CHECK();
}

// Norm partials from the update kernels are per 256-row block, the layout
// launch_normalize reads.
void launch_update(void* w, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                   const TsPlan& p, double* normp, cd* scratch, int64_t scratch_len,
                   hipStream_t st, const Batch& bt) {
    if (ncols <= 0 && !normp) return;
    if (fp32)
        update_impl<cf>((cf*)w, (const cf*)B, ldb, ncols, coef, p.n, 1.0, -1.0, normp, scratch,
                        scratch_len, st, bt);
    else
        update_impl<cd>((cd*)w, (const cd*)B, ldb, ncols, coef, p.n, 1.0, -1.0, normp, scratch,
                        scratch_len, st, bt);
}

void launch_combine(void* y, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                    bool add, int64_t n, hipStream_t st, const Batch& bt) {
    if (fp32)
        update_impl<cf>((cf*)y, (const cf*)B, ldb, ncols, coef, n, add ? 1.0 : 0.0, 1.0, nullptr,
                        nullptr, 0, st, bt);
    else
        update_impl<cd>((cd*)y, (const cd*)B, ldb, ncols, coef, n, add ? 1.0 : 0.0, 1.0, nullptr,
                        nullptr, 0, st, bt);
}

// ------------------------------------------- shared basis, several vectors
// The LR projection of a lockstep batch applies the same R, L (m columns) to
// every source's vector.  These kernels read the shared columns once for a
// group of sources instead of once per source, and give every source exactly
// the arithmetic of the one-source kernels above (same row chunks, the same
// fma sequence per (column, source), the same block reduction), so batched
// results stay bitwise those of single-source solves.

// Dots of C shared columns with R sources' vectors per block (chunk q, column
// group, source group); partial of problem b, column c at
// b*bt.part + c*nchunks + q.  Up to 12 sources per group with 2 columns per block (all 12 sources of a
// lockstep batch read the shared columns once), else 4 sources with 8 columns.
// The sources' rows are re-read by every column group: XCD x takes a
// contiguous run of (chunk, column group) items, column group fastest.
template <int C, int R>
__global__ __launch_bounds__(kBlock) void k_mdot_partial(const cd* __restrict__ B, int64_t ldb,
                                                         int ncols, const cd* __restrict__ w,
                                                         int64_t n, int rpc, int nchunks,
                                                         int ngroups, int per_xcd,
                                                         cd* __restrict__ partial, Batch bt) {
    constexpr int NV = 2 * C * R;
    __shared__ double sm[kWaves * NV];
    __shared__ double so[NV];
    const int item = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    if (item >= nchunks * ngroups) return;   // whole block: before any barrier
    const int q = item / ngroups;
    const int c0 = (item % ngroups) * C;
    const int g0 = blockIdx.z * R;
    const int nr = (bt.n - g0 < R) ? bt.n - g0 : R;
    const int nc = (ncols - c0 < C) ? ncols - c0 : C;
    const int64_t r0 = (int64_t)q * rpc;
    const int64_t r1 = (r0 + rpc < n) ? r0 + rpc : n;
    const cd* wv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) wv[r] = w + (int64_t)bt.idx[g0 + (r < nr ? r : 0)] * bt.vec;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        cd wi[R];
#pragma unroll
        for (int r = 0; r < R; ++r) wi[r] = wv[r][i];
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
            if (cc < nc) {
                const cd b = B[(int64_t)(c0 + cc) * ldb + i];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double* a = acc + 2 * (r * C + cc);
                    a[0] = fma(b.x, wi[r].x, fma(b.y, wi[r].y, a[0]));
                    a[1] = fma(b.x, wi[r].y, fma(-b.y, wi[r].x, a[1]));
                }
            }
        }
    }
    block_sum<NV>(acc, sm, so);
    if (threadIdx.x < nc * R) {
        const int r = threadIdx.x / nc, cc = threadIdx.x % nc;
        if (r < nr) {
            const int pb = bt.idx[g0 + r];
            partial[pb * bt.part + (int64_t)(c0 + cc) * nchunks + q] =
                mk(so[2 * (r * C + cc)], so[2 * (r * C + cc) + 1]);
        }
    }
}

int launch_mdot_partial(const cd* B, int64_t ldb, int ncols, const cd* w, const TsPlan& pn,
                        cd* partial, hipStream_t st, const Batch& bt) {
    constexpr int C = 8;   // the one-source kernel's column group: its chunk plan
    if (ncols <= 0 || bt.n <= 0) return dot_plan(pn.n, ncols, C).nchunks;
    const bool wide = bt.n > 4;
    auto go = [&](const TsPlan& p) {
        const int cg = wide ? 2 : 8, rg = wide ? 12 : 4;
        const int ngroups = (int)ceil_div(ncols, cg);
        const int per_xcd = (int)ceil_div((int64_t)p.nchunks * ngroups, kXcds);
        dim3 grid((unsigned)(kXcds * per_xcd), 1, (unsigned)ceil_div(bt.n, rg));
        if (wide)
            hipLaunchKernelGGL((k_mdot_partial<2, 12>), grid, dim3(kBlock), 0, st, B, ldb, ncols, w,
                               p.n, p.rows_per_chunk, p.nchunks, ngroups, per_xcd, partial, bt);
        else
            hipLaunchKernelGGL((k_mdot_partial<8, 4>), grid, dim3(kBlock), 0, st, B, ldb, ncols, w,
                               p.n, p.rows_per_chunk, p.nchunks, ngroups, per_xcd, partial, bt);
        OSA_LAUNCH_CHECK();
    };
    const TsPlan p = tuned_plan(pn.n, ncols, C, st, go);   // the one-source plan: same chunks
    go(p);
    return p.nchunks;
}

// w_v[i] -= sum_c B[c][i] coef_v[c] for nv vectors per problem (vector t of
// problem b at w + b*bt.vec + t*off2, its coefficients at coef + b*bt.small +
// t*coff2), NR vectors per launch entry (at most kMupdV), B read once per entry:
// the arithmetic of k_update_direct (alpha = 1, no norm partials) for every
// vector.  The coefficients are uniform over the block and are read with
// uniform addresses (scalar loads), not staged through LDS.
static constexpr int kMupdR = 16;
static constexpr int kMupdV = 24;
static constexpr int kMupdCols = 64;

template <int NR>
__global__ __launch_bounds__(kBlock) void k_mupdate(cd* w, int64_t off2, int nv,
                                                    const cd* __restrict__ B, int64_t ldb,
                                                    int ncols, const cd* __restrict__ coef,
                                                    int64_t coff2, int64_t n, int v0, Batch bt) {
    const cd* cp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int v = v0 + r;
        cp[r] = coef + (int64_t)bt.idx[v / nv] * bt.small + (int64_t)(v % nv) * coff2;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    cd acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = mk(0.0, 0.0);
    for (int c = 0; c < ncols; ++c) {
        const cd b = B[(int64_t)c * ldb + i];
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma(acc[r], b, cp[r][c]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int v = v0 + r;
        cd* wp = w + (int64_t)bt.idx[v / nv] * bt.vec + (int64_t)(v % nv) * off2 + i;
        const cd base = *wp;
        *wp = mk(base.x + -1.0 * acc[r].x, base.y + -1.0 * acc[r].y);
    }
}

bool mupdate_matches_single(int64_t n, int ncols) {
    // k_update_direct is the one-source kernel exactly when update_impl does not
    // split the columns: at most 32 columns, or rows enough to fill the GPU
    return ncols <= kMupdCols && (ncols <= 32 || ceil_div(n, kBlock) >= 1024);
}

template <int NR>
static void mupdate_go(cd* w, int64_t off2, int nv, const cd* B, int64_t ldb, int ncols,
                       const cd* coef, int64_t coff2, int64_t n, int v0, hipStream_t st,
                       const Batch& bt) {
    hipLaunchKernelGGL(k_mupdate<NR>, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, w,
                       off2, nv, B, ldb, ncols, coef, coff2, n, v0, bt);
}

void launch_mupdate(cd* w, const cd* B, int64_t ldb, int ncols, const cd* coef, int64_t n,
                    hipStream_t st, const Batch& bt, int nv, int64_t off2, int64_t coff2) {
    if (bt.n <= 0 || ncols <= 0) return;
    if (ncols > kMupdCols) throw HipError{hipErrorInvalidValue, "launch_mupdate: ncols > 64"};
    if (nv < 1 || nv > 2) throw HipError{hipErrorInvalidValue, "launch_mupdate: nv not 1 or 2"};
    const int nvec = bt.n * nv;
    for (int v0 = 0; v0 < nvec; v0 += kMupdV) {
        const int nr = std::min(kMupdV, nvec - v0);
#define OSA_MUPD(NR) \
    case NR: mupdate_go<NR>(w, off2, nv, B, ldb, ncols, coef, coff2, n, v0, st, bt); break;
        switch (nr) {
            OSA_MUPD(1) OSA_MUPD(2) OSA_MUPD(3) OSA_MUPD(4) OSA_MUPD(5) OSA_MUPD(6)
            OSA_MUPD(7) OSA_MUPD(8) OSA_MUPD(9) OSA_MUPD(10) OSA_MUPD(11) OSA_MUPD(12)
            OSA_MUPD(13) OSA_MUPD(14) OSA_MUPD(15) OSA_MUPD(16) OSA_MUPD(17) OSA_MUPD(18)
            OSA_MUPD(19) OSA_MUPD(20) OSA_MUPD(21) OSA_MUPD(22) OSA_MUPD(23)
            default: mupdate_go<24>(w, off2, nv, B, ldb, ncols, coef, coff2, n, v0, st, bt); break;
        }
#undef OSA_MUPD
        OSA_LAUNCH_CHECK();
    }
}

// ------------------------------------------- projection dots, LDS tiles
// Dots of the m shared columns L (m <= kPdMaxM) with the vectors of the batch,
// nv per problem (vector t of problem b at w + b*bt.vec + t*off2): partial
// [b*bt.part + (t*m + c)*nchunks + q] = sum over chunk q of conj(L[c][i]) w[i].
// One block per row chunk and group of up to kPdMaxV vectors.  Tiles of kPdKT
// rows of L and of the vectors are staged through LDS (double-buffered,
// column-major with a one-row pad, the next tile's loads in flight during the
// current tile's products), so L and the vectors are each read once from HBM.
// Wave g of the block owns the rows r of its chunk with (r - r0) % 8 == g, in
// increasing order; lane l owns the TC x TV (column, vector) pairs of column
// group l % 8 and vector group l / 8.  A pair's dot is therefore the same fma
// chain over the same rows whatever the batch or the lane split, and the eight
// wave sums are added in the order 0..7: results depend on (n, m) only (the
// chunk plan, pdot_plan), so a batched projection is bitwise that of one source.
static constexpr int kPdSlices = 8;                 // waves per block
static constexpr int kPdThreads = 64 * kPdSlices;
static constexpr int kPdLanes = 8;                  // column groups (= vector groups)
static constexpr int kPdKT = 16;                    // rows per tile
static constexpr int kPdMaxV = 3 * kPdLanes;        // vectors per block

template <int TC, int TV>
__global__ __launch_bounds__(kPdThreads) void k_pdot_partial(
    const cd* __restrict__ L, int64_t ldl, int m, const cd* __restrict__ w, int64_t off2, int nv,
    int v0, int S, int64_t n, int rpc, int nchunks, cd* __restrict__ partial, Batch bt) {
    extern __shared__ cd pd_sh[];
    constexpr int KT = kPdKT, KTP = KT + 1;
    constexpr int NLD = (kPdMaxM * KT + kPdThreads - 1) / kPdThreads;
    constexpr int NWD = (kPdLanes * TV * KT + kPdThreads - 1) / kPdThreads;
    const int bufsz = (m + S) * KTP;
    cd* const sL0 = pd_sh;
    cd* const sW0 = pd_sh + m * KTP;
    const int q = blockIdx.x;
    const int64_t r0 = (int64_t)q * rpc;
    const int64_t r1 = (r0 + rpc < n) ? r0 + rpc : n;
    const int tid = threadIdx.x, lane = tid & 63;
    const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cb = (lane % kPdLanes) * TC, vb = (lane / kPdLanes) * TV;
    // the tile loads: element e of the L tile is (column e / KT, row e % KT),
    // clamped into range (the surplus loads repeat a valid address and are
    // never stored), so every prefetch register is always written
    const int ntile = (int)((r1 - r0 + KT - 1) / KT);
    double2 rl[NLD], rw[NWD];
    const int nle = m * KT, nwe = S * KT;
    auto vec_ptr = [&](int v) {
        const int gv = v0 + v;
        return w + (int64_t)bt.idx[gv / nv] * bt.vec + (int64_t)(gv % nv) * off2;
    };
#define OSA_PD_LOAD(T)                                                                       \
    {                                                                                        \
        const int64_t t0n = r0 + (int64_t)(T) * KT;                                          \
        _Pragma("unroll") for (int k = 0; k < NLD; ++k) {                                    \
            int e = tid + k * kPdThreads;                                                    \
            e = (e < nle) ? e : nle - 1;                                                     \
            const int64_t rr = (t0n + e % KT < r1) ? t0n + e % KT : r1 - 1;                  \
            rl[k] = *(const double2*)(L + (int64_t)(e / KT) * ldl + rr);                     \
        }                                                                                    \
        _Pragma("unroll") for (int k = 0; k < NWD; ++k) {                                    \
            int e = tid + k * kPdThreads;                                                    \
            e = (e < nwe) ? e : nwe - 1;                                                     \
            const int64_t rr = (t0n + e % KT < r1) ? t0n + e % KT : r1 - 1;                  \
            rw[k] = *(const double2*)(vec_ptr(e / KT) + rr);                                 \
        }                                                                                    \
    }
#define OSA_PD_STORE(BUF)                                                                    \
    {                                                                                        \
        cd* sl_ = sL0 + (BUF) * bufsz;                                                       \
        cd* sw_ = sW0 + (BUF) * bufsz;                                                       \
        _Pragma("unroll") for (int k = 0; k < NLD; ++k) {                                    \
            const int e = tid + k * kPdThreads;                                              \
            if (e < nle) sl_[(e / KT) * KTP + e % KT] = mk(rl[k].x, rl[k].y);                \
        }                                                                                    \
        _Pragma("unroll") for (int k = 0; k < NWD; ++k) {                                    \
            const int e = tid + k * kPdThreads;                                              \
            if (e < nwe) sw_[(e / KT) * KTP + e % KT] = mk(rw[k].x, rw[k].y);                \
        }                                                                                    \
    }
    double acc[TC][TV][2];
#pragma unroll
    for (int i = 0; i < TC; ++i)
#pragma unroll
        for (int k = 0; k < TV; ++k) acc[i][k][0] = acc[i][k][1] = 0.0;
    int ci[TC], vi[TV];
#pragma unroll
    for (int i = 0; i < TC; ++i) ci[i] = (cb + i < m) ? cb + i : m - 1;
#pragma unroll
    for (int k = 0; k < TV; ++k) vi[k] = (vb + k < S) ? vb + k : S - 1;
    if (ntile > 0) {
        OSA_PD_LOAD(0)
        OSA_PD_STORE(0)
    }
    __syncthreads();
    for (int t = 0; t < ntile; ++t) {
        if (t + 1 < ntile) OSA_PD_LOAD(t + 1)
        const cd* sl = sL0 + (t & 1) * bufsz + g;
        const cd* sw = sW0 + (t & 1) * bufsz + g;
        const cd* pl[TC];
        const cd* pw[TV];
#pragma unroll
        for (int i = 0; i < TC; ++i) pl[i] = sl + ci[i] * KTP;
#pragma unroll
        for (int k = 0; k < TV; ++k) pw[k] = sw + vi[k] * KTP;
        const int64_t t0 = r0 + (int64_t)t * KT;
        const int nrow = (r1 - t0 < KT) ? (int)(r1 - t0) : KT;
#pragma unroll
        for (int j = 0; j < KT / kPdSlices; ++j) {
            if (g + kPdSlices * j < nrow) {
                cd wv[TV];
#pragma unroll
                for (int k = 0; k < TV; ++k) wv[k] = pw[k][kPdSlices * j];
#pragma unroll
                for (int i = 0; i < TC; ++i) {
                    const cd l = pl[i][kPdSlices * j];
#pragma unroll
                    for (int k = 0; k < TV; ++k) {   // conj(l) w
                        acc[i][k][0] = fma(l.x, wv[k].x, fma(l.y, wv[k].y, acc[i][k][0]));
                        acc[i][k][1] = fma(l.x, wv[k].y, fma(-l.y, wv[k].x, acc[i][k][1]));
                    }
                }
            }
        }
        if (t + 1 < ntile) OSA_PD_STORE((t + 1) & 1)
        __syncthreads();
    }
#undef OSA_PD_LOAD
#undef OSA_PD_STORE
    // the eight waves' sums, added in wave order
    cd* red = pd_sh;
    for (int s = 0; s < kPdSlices; ++s) {
        if (g == s) {
#pragma unroll
            for (int i = 0; i < TC; ++i)
#pragma unroll
                for (int k = 0; k < TV; ++k)
                    if (cb + i < m && vb + k < S) {
                        cd* r = red + (cb + i) * S + vb + k;
                        *r = (s == 0) ? mk(acc[i][k][0], acc[i][k][1])
                                      : mk(r->x + acc[i][k][0], r->y + acc[i][k][1]);
                    }
        }
        __syncthreads();
    }
    for (int e = tid; e < m * S; e += kPdThreads) {
        const int c = e % m, v = e / m, gv = v0 + v;
        partial[(int64_t)bt.idx[gv / nv] * bt.part + (int64_t)((gv % nv) * m + c) * nchunks + q] =
            red[c * S + v];
    }
}

TsPlan pdot_plan(int64_t n, int m) {
    // up to 512 chunks, at least 256 rows each, and 2 m chunks within the
    // partial buffer's 160 kMaxChunks entries per problem (two vectors)
    int64_t want = ceil_div(n, 256);
    want = std::min<int64_t>(want, 512);
    want = std::min<int64_t>(want, (int64_t)(160 * kMaxChunks) / (2 * std::max(m, 1)));
    if (want < 1) want = 1;
    TsPlan p;
    p.n = n;
    p.rows_per_chunk = (int)(ceil_div(ceil_div(n, want), kPdSlices) * kPdSlices);
    p.nchunks = (int)ceil_div(n, p.rows_per_chunk);
    return p;
}

template <int TC, int TV>
static void pdot_go(const cd* L, int64_t ldl, int m, const cd* w, int64_t off2, int nv, int v0,
                    int S, const TsPlan& p, cd* partial, hipStream_t st, const Batch& bt) {
    const size_t lds = sizeof(cd) * std::max<size_t>((size_t)2 * (m + S) * (kPdKT + 1),
                                                     (size_t)m * S);
    hipLaunchKernelGGL((k_pdot_partial<TC, TV>), dim3((unsigned)p.nchunks), dim3(kPdThreads), lds,
                       st, L, ldl, m, w, off2, nv, v0, S, p.n, p.rows_per_chunk, p.nchunks, partial,
                       bt);
}

template <int TC>
static void pdot_tv(int tv, const cd* L, int64_t ldl, int m, const cd* w, int64_t off2, int nv,
                    int v0, int S, const TsPlan& p, cd* partial, hipStream_t st, const Batch& bt) {
    if (tv == 1) pdot_go<TC, 1>(L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt);
    else if (tv == 2) pdot_go<TC, 2>(L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt);
    else pdot_go<TC, 3>(L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt);
}

int launch_pdot_partial(const cd* L, int64_t ldl, int m, const cd* w, int64_t off2, int nv,
                        int64_t n, cd* partial, hipStream_t st, const Batch& bt) {
    const TsPlan p = pdot_plan(n, m);
    if (m <= 0 || bt.n <= 0) return p.nchunks;
    if (m > kPdMaxM) throw HipError{hipErrorInvalidValue, "launch_pdot_partial: m > 64"};
    if (nv < 1 || nv > 2) throw HipError{hipErrorInvalidValue, "launch_pdot_partial: nv"};
    if ((int64_t)2 * m * p.nchunks > (int64_t)160 * kMaxChunks)
        throw HipError{hipErrorInvalidValue, "launch_pdot_partial: partial buffer"};
    const int tc = (int)ceil_div(m, kPdLanes);
    const int nvec = bt.n * nv;
    for (int v0 = 0; v0 < nvec; v0 += kPdMaxV) {
        const int S = std::min(kPdMaxV, nvec - v0);
        const int tv = (int)ceil_div(S, kPdLanes);
        switch (tc) {
            case 1: pdot_tv<1>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 2: pdot_tv<2>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 3: pdot_tv<3>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 4: pdot_tv<4>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 5: pdot_tv<5>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 6: pdot_tv<6>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            case 7: pdot_tv<7>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
            default: pdot_tv<8>(tv, L, ldl, m, w, off2, nv, v0, S, p, partial, st, bt); break;
        }
        OSA_LAUNCH_CHECK();
    }
    return p.nchunks;
}

// out_b[i] = a w_b[i] + sg sum_{c < ncols} B[c][i] coef_b[c] for every problem b
// of the batch, the shared columns B read once per group of kMupdR problems and
// the coefficients staged through LDS in tiles of kMupdCols: the block
// Gram-Schmidt update W -= Q h and the block assembly Y += V (F E_1 R_0) of the
// block Krylov variant.  Batch strides: vec (w), small (coef).
__global__ __launch_bounds__(kBlock) void k_mcombine(cd* w, const cd* __restrict__ B, int64_t ldb,
                                                     int ncols, const cd* __restrict__ coef,
                                                     int64_t n, double a, double sg, Batch bt) {
    __shared__ cd scoef[kMupdR][kMupdCols];
    const int g0 = blockIdx.y * kMupdR;
    const int nr = (bt.n - g0 < kMupdR) ? bt.n - g0 : kMupdR;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n;
    cd acc[kMupdR];
#pragma unroll
    for (int r = 0; r < kMupdR; ++r) acc[r] = mk(0.0, 0.0);
    for (int cb = 0; cb < ncols; cb += kMupdCols) {
        const int nc = (ncols - cb < kMupdCols) ? ncols - cb : kMupdCols;
        __syncthreads();
        for (int e = threadIdx.x; e < nr * nc; e += kBlock) {
            const int r = e / nc, cc = e - r * nc;
            scoef[r][cc] = coef[(int64_t)bt.idx[g0 + r] * bt.small + cb + cc];
        }
        __syncthreads();
        if (valid) {
            for (int c = 0; c < nc; ++c) {
                const cd b = B[(int64_t)(cb + c) * ldb + i];
#pragma unroll
                for (int r = 0; r < kMupdR; ++r)
                    if (r < nr) cfma(acc[r], b, scoef[r][c]);
            }
        }
    }
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < kMupdR; ++r) {
        if (r < nr) {
            cd* wp = w + (int64_t)bt.idx[g0 + r] * bt.vec + i;
            cd v = mk(sg * acc[r].x, sg * acc[r].y);
            if (a != 0.0) {
                const cd base = *wp;
                v = mk(fma(a, base.x, v.x), fma(a, base.y, v.y));
            }
            *wp = v;
        }
    }
}

void launch_mcombine(cd* w, const cd* B, int64_t ldb, int ncols, const cd* coef, int64_t n,
                     double a, double sg, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0 || ncols <= 0) return;
    dim3 grid((unsigned)ceil_div(n, kBlock), (unsigned)ceil_div(bt.n, kMupdR));
    hipLaunchKernelGGL(k_mcombine, grid, dim3(kBlock), 0, st, w, B, ldb, ncols, coef, n, a, sg,
                       bt);
    OSA_LAUNCH_CHECK();
}

// ------------------------------------------------ delayed reorthogonalisation
// Step j (>= 1) of the Arnoldi recurrence with delayed reorthogonalisation.
// Column j of the basis holds u_j, orthogonalised once and not normalised; z =
// H u_j (re-projected).  With s = V_j^H u_j, t = V_j^H z, r = |u_j - V_j s| and
// c_j = v_j^H z (all from one dot pass over [V_j, u_j] with [u_j, z]):
//   v_j     = (u_j - V_j s) / r
//   u_{j+1} = (z - V_j t - c_j v_j) / r
// one pass over V_j computes both.  coef: s at [0, j), t at [j+1, 2j+1);
// sc: [0] = 1/r (0 after a breakdown), [1] = c_j.
template <typename T>
__device__ __forceinline__ void gemv2_rows(const T* __restrict__ B, int64_t ldb, int cbeg, int cend,
                                           const cd* __restrict__ cs, const cd* __restrict__ ct,
                                           int64_t i, cd* s1, cd* s2, cd& as, cd& at) {
    as = mk(0.0, 0.0);
    at = mk(0.0, 0.0);
    for (int cb = cbeg; cb < cend; cb += kCoefTile) {
        const int ce = (cb + kCoefTile < cend) ? cb + kCoefTile : cend;
        __syncthreads();
        for (int c = cb + (int)threadIdx.x; c < ce; c += kBlock) {
            s1[c - cb] = cs[c];
            s2[c - cb] = ct[c];
        }
        __syncthreads();
        int c = cb;
        for (; c + 2 <= ce; c += 2) {
            const cd b0 = tod(B[(int64_t)(c + 0) * ldb + i]);
            const cd b1 = tod(B[(int64_t)(c + 1) * ldb + i]);
            cfma(as, b0, s1[c - cb + 0]);
            cfma(at, b0, s2[c - cb + 0]);
            cfma(as, b1, s1[c - cb + 1]);
            cfma(at, b1, s2[c - cb + 1]);
        }
        for (; c < ce; ++c) {
            const cd b0 = tod(B[(int64_t)c * ldb + i]);
            cfma(as, b0, s1[c - cb]);
            cfma(at, b0, s2[c - cb]);
        }
    }
}

template <typename T>
__device__ __forceinline__ void dcgs_finish_row(T* __restrict__ V, int64_t ldb, int j,
                                                const T* __restrict__ z, const cd* sc, int64_t i,
                                                cd as, cd at) {
    const double ir = sc[0].x;
    const cd cj = sc[1];
    const cd u = tod(V[(int64_t)j * ldb + i]);
    const cd v = cscale(csub(u, as), ir);
    const cd v_st = tod(fromd<T>(v));
    cd un = csub(csub(tod(z[i]), at), cmul(cj, v_st));
    un = cscale(un, ir);
    V[(int64_t)j * ldb + i] = fromd<T>(v);
    V[(int64_t)(j + 1) * ldb + i] = fromd<T>(un);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dcgs_update(T* V, int64_t ldb, int j,
                                                        const T* __restrict__ z,
                                                        const cd* __restrict__ coef,
                                                        const cd* __restrict__ sc, int64_t n,
                                                        Batch bt) {
    __shared__ cd s1[kCoefTile], s2[kCoefTile];
    const int pb = bt.idx[blockIdx.y];
    V += pb * bt.basis;
    z += pb * bt.vec;
    coef += pb * bt.small;
    sc += pb * bt.scal;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ii = (i < n) ? i : n - 1;
    cd as, at;
    gemv2_rows(V, ldb, 0, j, coef, coef + j + 1, ii, s1, s2, as, at);
    if (i < n) dcgs_finish_row(V, ldb, j, z, sc, i, as, at);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dcgs_split(const T* __restrict__ V, int64_t ldb, int j,
                                                       const cd* __restrict__ coef, int64_t n,
                                                       int cpg, cd* __restrict__ scratch, int G,
                                                       Batch bt) {
    __shared__ cd s1[kCoefTile], s2[kCoefTile];
    const int pb = bt.idx[blockIdx.z];
    V += pb * bt.basis;
    coef += pb * bt.small;
    scratch += (int64_t)blockIdx.z * 2 * G * n;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ii = (i < n) ? i : n - 1;
    const int g = blockIdx.y;
    const int cb = g * cpg;
    const int ce = (cb + cpg < j) ? cb + cpg : j;
    cd as, at;
    gemv2_rows(V, ldb, cb, ce, coef, coef + j + 1, ii, s1, s2, as, at);
    if (i < n) {
        scratch[(int64_t)(2 * g) * n + i] = as;
        scratch[(int64_t)(2 * g + 1) * n + i] = at;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dcgs_finish(T* V, int64_t ldb, int j,
                                                        const T* __restrict__ z,
                                                        const cd* __restrict__ scratch, int G,
                                                        const cd* __restrict__ sc, int64_t n,
                                                        Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    V += pb * bt.basis;
    z += pb * bt.vec;
    sc += pb * bt.scal;
    scratch += (int64_t)blockIdx.y * 2 * G * n;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    cd as = mk(0.0, 0.0), at = mk(0.0, 0.0);
    for (int g = 0; g < G; ++g) {
        as = cadd(as, scratch[(int64_t)(2 * g) * n + i]);
        at = cadd(at, scratch[(int64_t)(2 * g + 1) * n + i]);
    }
    dcgs_finish_row(V, ldb, j, z, sc, i, as, at);
}

template <typename T>
static void dcgs_impl(T* V, int64_t ldb, int j, const T* z, const cd* coef, const cd* sc,
                      int64_t n, cd* scratch, int64_t scratch_len, hipStream_t st,
                      const Batch& bt) {
    if (bt.n <= 0) return;
    const int rb = (int)ceil_div(n, kBlock);
    // the same split rule as the plain update: it depends on rows and columns only
    int G = 1;
    if (j > 32 && rb < 1024 && scratch) {
        G = (int)ceil_div(1024, rb);
        int gmax = j / 16;
        if (G > gmax) G = gmax;
        if (G > 8) G = 8;
        while (G > 1 && (int64_t)2 * G * n * bt.n > scratch_len) --G;
    }
    if (G <= 1) {
        hipLaunchKernelGGL((k_dcgs_update<T>), dim3(rb, bt.n), dim3(kBlock), 0, st, V, ldb, j, z,
                           coef, sc, n, bt);
    } else {
        const int cpg = (int)ceil_div(j, G);
        G = (int)ceil_div(j, cpg);
        hipLaunchKernelGGL((k_dcgs_split<T>), dim3(rb, G, bt.n), dim3(kBlock), 0, st,
                           (const T*)V, ldb, j, coef, n, cpg, scratch, G, bt);
        hipLaunchKernelGGL((k_dcgs_finish<T>), dim3(rb, bt.n), dim3(kBlock), 0, st, V, ldb, j, z,
                           (const cd*)scratch, G, sc, n, bt);
    }
    OSA_LAUNCH_CHECK();
}

void launch_dcgs_update(void* V, int64_t ldb, int j, const void* z, const cd* coef, const cd* sc,
                        bool fp32, int64_t n, cd* scratch, int64_t scratch_len, hipStream_t st,
                        const Batch& bt) {
    if (fp32)
        dcgs_impl<cf>((cf*)V, ldb, j, (const cf*)z, coef, sc, n, scratch, scratch_len, st, bt);
    else
        dcgs_impl<cd>((cd*)V, ldb, j, (const cd*)z, coef, sc, n, scratch, scratch_len, st, bt);
}

// Small per-problem part of step j.  k_dcgs_coef (one block per problem), from
// the reduced dot products d = [s (j), u^H u, t (j), u^H z], completes column
// j-1 of H (H[0:j, j-1] += s, H[j, j-1] = r, with the breakdown test of the
// plain recurrence) and sets sc = [1/r, c_j]; k_dcgs_col (one wavefront per
// row) then writes the first-pass column j,
//   H[0:j+1, j] = ([t; c_j] - H[0:j+1, 0:j] s) / r,
// using the Hessenberg band of H (hess) or all of it (a Krylov-Schur Rayleigh
// quotient after a restart).  Without the first pass (the last step before a
// restart: d = [s, u^H u] only) just column j-1 and 1/r are set.
__global__ __launch_bounds__(256) void k_dcgs_coef(int j, cd* H, int ldh, const cd* __restrict__ d,
                                                   cd* sc, double* hfro2, int* flag, double rel,
                                                   int with_t, Batch bt) {
    __shared__ double sred[4 * 4];
    const int pb = bt.idx[blockIdx.x];
    H += pb * bt.small;
    d += pb * bt.small;
    sc += pb * bt.scal;
    hfro2 += 2 * pb * bt.scal;
    flag += pb * bt.flag;
    const cd* s = d;
    const cd* t = d + j + 1;
    double ss = 0, stx = 0, sty = 0, col2 = 0;
    for (int c = threadIdx.x; c < j; c += 256) {
        const cd sv = s[c], tv = with_t ? t[c] : mk(0.0, 0.0);
        ss += cabs2(sv);
        stx += sv.x * tv.x + sv.y * tv.y;   // conj(s) t
        sty += sv.x * tv.y - sv.y * tv.x;
        const cd hc = cadd(H[c + (int64_t)(j - 1) * ldh], sv);
        H[c + (int64_t)(j - 1) * ldh] = hc;
        col2 += cabs2(hc);
    }
    double v4[4] = {ss, stx, sty, col2};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double x = wave_sum(v4[q]);
        if (lane == 0) sred[wave * 4 + q] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[4] = {0, 0, 0, 0};
        for (int w = 0; w < 4; ++w)
            for (int q = 0; q < 4; ++q) tot[q] += sred[w * 4 + q];
        const double alpha = d[j].x;
        const double r = sqrt(fmax(alpha - tot[0], 0.0));
        *hfro2 += tot[3];
        const double scale = sqrt(*hfro2 + r * r);
        int bd = (r <= rel * scale) ? 1 : 0;
        if (!(r == r) || r > 1e300 || !(alpha == alpha)) bd = 2;   // non-finite
        if (bd) {
            if (flag[0] == 0) flag[1] = j - 1;
            if (bd > flag[0]) flag[0] = bd;
        }
        H[j + (int64_t)(j - 1) * ldh] = mk(r, 0.0);
        const double ir = flag[0] ? 0.0 : 1.0 / r;
        const cd g = with_t ? d[2 * j + 1] : mk(0.0, 0.0);
        const cd cj = cscale(mk(g.x - tot[1], g.y - tot[2]), ir);
        sc[0] = mk(ir, 0.0);
        sc[1] = cj;
    }
}

// row = 4*blockIdx.x + wave: lanes take columns in order, then a fixed shuffle tree
__global__ __launch_bounds__(256) void k_dcgs_col(int j, cd* H, int ldh, const cd* __restrict__ d,
                                                  const cd* __restrict__ sc, int hess, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    H += pb * bt.small;
    d += pb * bt.small;
    sc += pb * bt.scal;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row > j) return;
    double hx = 0, hy = 0;
    for (int col = (hess && row > 0 ? row - 1 : 0) + lane; col < j; col += 64) {
        const cd hv = H[row + (int64_t)col * ldh], sv = d[col];
        hx += hv.x * sv.x - hv.y * sv.y;
        hy += hv.x * sv.y + hv.y * sv.x;
    }
    hx = wave_sum(hx);
    hy = wave_sum(hy);
    if (lane == 0) {
        const cd base = (row < j) ? d[j + 1 + row] : sc[1];
        H[row + (int64_t)j * ldh] = cscale(mk(base.x - hx, base.y - hy), sc[0].x);
    }
}

void launch_dcgs_coef(int j, cd* H, int ldh, const cd* d, cd* sc, double* hfro2, int* flag,
                      double rel, hipStream_t st, const Batch& bt, bool hess, bool first_pass) {
    if (bt.n <= 0) return;
    hipLaunchKernelGGL(k_dcgs_coef, dim3((unsigned)bt.n), dim3(256), 0, st, j, H, ldh, d, sc,
                       hfro2, flag, rel, first_pass ? 1 : 0, bt);
    if (first_pass)
        hipLaunchKernelGGL(k_dcgs_col, dim3((unsigned)ceil_div(j + 1, 4), (unsigned)bt.n),
                           dim3(256), 0, st, j, H, ldh, d, (const cd*)sc, hess ? 1 : 0, bt);
    OSA_LAUNCH_CHECK();
}

// ------------------------------------------- two-step block Arnoldi
// The two-step form of the Arnoldi recurrence (Eq. 7) extends the basis by two
// vectors per outer step with one dot pass and one update pass over the basis:
// columns n, n+1 hold the block U = [u_a, u_b] (orthogonalised once against
// v_0..v_{n-1}, not yet against each other), columns n+2, n+3 the new block
// W = [H u_b, H^2 u_b].  One dot pass gives [V_n, U]^H [U, W]; the coefficient
// kernel finishes U into v_n, v_{n+1} (second Gram-Schmidt pass and a 2x2
// Cholesky factor R), orthogonalises W once against v_0..v_{n+1}, recovers the
// Hessenberg columns n-1 and n and the pending part of column n+1, and the
// update pass forms all four columns from one read of the basis.  Same
// decomposition as the one-vector recurrence in exact arithmetic.

// Dots of ncols columns of B with the four vectors W + v*ldw (v < 4), all in the
// problem's basis: partial[(v*ncols + c)*nchunks + q].  A block takes C columns
// over one chunk of rows; the chunk's rows of the four vectors are read by all
// ncols / C column groups, so the blocks are ordered for the L2 caches:
// workgroups are dealt to the 8 XCDs in turn, and XCD x takes a contiguous run
// of (chunk, column group) items with the column group varying fastest, so the
// re-reads of a chunk's vector rows follow each other in one L2.  (8 columns
// per block, or the vectors split over two half-blocks, measured slower.)
static constexpr int kDot4Cols = 4;

template <int C>
__global__ __launch_bounds__(kBlock) void k_dot4_partial(const cd* __restrict__ B, int64_t ldb,
                                                         int ncols, const cd* __restrict__ W,
                                                         int64_t ldw, int64_t n, int rpc,
                                                         int nchunks, int ngroups, int per_xcd,
                                                         cd* __restrict__ partial, Batch bt) {
    __shared__ double sm[kWaves * 8 * C];
    __shared__ double so[8 * C];
    const int item = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    if (item >= nchunks * ngroups) return;   // whole block: before any barrier
    const int q = item / ngroups;
    const int c0 = (item % ngroups) * C;
    const int pb = bt.idx[blockIdx.z];
    B += pb * bt.basis;
    W += pb * bt.basis;
    partial += pb * bt.part;
    const int64_t r0 = (int64_t)q * rpc;
    const int64_t r1 = (r0 + rpc < n) ? r0 + rpc : n;
    double acc[8 * C];
#pragma unroll
    for (int i = 0; i < 8 * C; ++i) acc[i] = 0.0;
    const int nc = (ncols - c0 < C) ? ncols - c0 : C;
    // columns past ncols (the last group) read column c0 again and their sums
    // are dropped, so every load of a row is issued before its products
    const cd* bp[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) bp[cc] = B + (int64_t)(c0 + (cc < nc ? cc : 0)) * ldb;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        cd w[4], bb[C];
#pragma unroll
        for (int v = 0; v < 4; ++v) w[v] = W[v * ldw + i];
#pragma unroll
        for (int cc = 0; cc < C; ++cc) bb[cc] = bp[cc][i];
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
            const cd b = bb[cc];
#pragma unroll
            for (int v = 0; v < 4; ++v) {   // conj(b) w_v
                acc[8 * cc + 2 * v] = fma(b.x, w[v].x, fma(b.y, w[v].y, acc[8 * cc + 2 * v]));
                acc[8 * cc + 2 * v + 1] =
                    fma(b.x, w[v].y, fma(-b.y, w[v].x, acc[8 * cc + 2 * v + 1]));
            }
        }
    }
    block_sum<8 * C>(acc, sm, so);
    if (threadIdx.x < nc) {
        const int c = c0 + threadIdx.x;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            partial[(int64_t)(v * ncols + c) * nchunks + q] =
                mk(so[8 * threadIdx.x + 2 * v], so[8 * threadIdx.x + 2 * v + 1]);
    }
}

int launch_dot4_partial(const cd* B, int64_t ldb, int ncols, const cd* W, int64_t ldw,
                        const TsPlan& pn, cd* partial, hipStream_t st, const Batch& bt) {
    constexpr int C = kDot4Cols;
    if (ncols <= 0 || bt.n <= 0) return dot_plan(pn.n, ncols, C).nchunks;
    auto go = [&](const TsPlan& p) {
        const int ngroups = (int)ceil_div(ncols, C);
        const int per_xcd = (int)ceil_div((int64_t)p.nchunks * ngroups, kXcds);
        dim3 grid((unsigned)(kXcds * per_xcd), 1, (unsigned)bt.n), blk(kBlock);
        hipLaunchKernelGGL((k_dot4_partial<C>), grid, blk, 0, st, B, ldb, ncols, W, ldw, p.n,
                           p.rows_per_chunk, p.nchunks, ngroups, per_xcd, partial, bt);
        OSA_LAUNCH_CHECK();
    };
    const TsPlan p = tuned_plan(pn.n, ncols, C, st, go);
    go(p);
    return p.nchunks;
}

// Columns o0 .. o0+NO-1 of the problem's basis become X M, X = columns 0 .. nin-1
// (which include the output columns: each row is read whole before it is
// written), M[o*ldm + c] the problem's coefficients.
template <int NO>
__global__ __launch_bounds__(kBlock) void k_blk_update(cd* V, int64_t ldb, int nin,
                                                       const cd* __restrict__ M, int ldm, int o0,
                                                       int64_t n, Batch bt) {
    __shared__ cd sc[kCoefTile * NO];
    const int pb = bt.idx[blockIdx.y];
    V += pb * bt.basis;
    M += pb * bt.small;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ii = (i < n) ? i : n - 1;   // keep every thread in the barriers
    cd acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = mk(0.0, 0.0);
    for (int cb = 0; cb < nin; cb += kCoefTile) {
        const int ce = (cb + kCoefTile < nin) ? cb + kCoefTile : nin;
        __syncthreads();
        for (int e = threadIdx.x; e < (ce - cb) * NO; e += kBlock)
            sc[e] = M[(int64_t)(e % NO) * ldm + cb + e / NO];
        __syncthreads();
        int c = cb;
        for (; c + 4 <= ce; c += 4) {
            cd x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = V[(int64_t)(c + u) * ldb + ii];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int o = 0; o < NO; ++o) cfma(acc[o], x[u], sc[(c + u - cb) * NO + o]);
        }
        for (; c < ce; ++c) {
            const cd x = V[(int64_t)c * ldb + ii];
#pragma unroll
            for (int o = 0; o < NO; ++o) cfma(acc[o], x, sc[(c - cb) * NO + o]);
        }
    }
    if (i < n) {
#pragma unroll
        for (int o = 0; o < NO; ++o) V[(int64_t)(o0 + o) * ldb + i] = acc[o];
    }
}

void launch_blk_update(cd* V, int64_t ldb, int nin, const cd* M, int ldm, int o0, int nout,
                       int64_t n, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const dim3 grid((unsigned)ceil_div(n, kBlock), (unsigned)bt.n);
    if (nout == 4)
        hipLaunchKernelGGL((k_blk_update<4>), grid, dim3(kBlock), 0, st, V, ldb, nin, M, ldm, o0,
                           n, bt);
    else if (nout == 2)
        hipLaunchKernelGGL((k_blk_update<2>), grid, dim3(kBlock), 0, st, V, ldb, nin, M, ldm, o0,
                           n, bt);
    else
        throw std::invalid_argument("launch_blk_update: nout must be 2 or 4");
    OSA_LAUNCH_CHECK();
}

// Per-problem workspace of the two-step form (entries from b2, vl = slot length):
//   D  [0, 4 vl)     dots, D[v*(n+2) + c] = column c ^H vector v
//   M  [4 vl, 8 vl)  update coefficients, M[o*vl + c]
//   a  [8 vl, 9 vl)  pending column: H v_{n-1} = V_n a + t0 u_a
//   Cp [9 vl, 11 vl) first-pass coefficients of the block, Cp[o*vl + c]
//   Y  [11 vl, 13 vl) Hessenberg products
//   sc [13 vl, ...)  sc[0].x = t0
// The first outer step: v_0 is column 0, W = [H v_0, H^2 v_0] columns 1, 2 and
// d = v_0^H W (two entries).  U = W - v_0 d, H v_0 = d_0 v_0 + u_a.
__global__ void k_blk2_init(cd* b2, int vl, const cd* __restrict__ d, Batch bt) {
    const int pb = bt.idx[blockIdx.x];
    b2 += pb * bt.small;
    d += pb * bt.small;
    if (threadIdx.x != 0) return;
    cd* M = b2 + 4 * (int64_t)vl;
    cd* a = b2 + 8 * (int64_t)vl;
    cd* Cp = b2 + 9 * (int64_t)vl;
    cd* sc = b2 + 13 * (int64_t)vl;
    const cd zero = mk(0.0, 0.0), one = mk(1.0, 0.0);
    const cd d0 = d[0], d1 = d[1];
    a[0] = d0;
    Cp[0] = d0;
    Cp[vl] = d1;
    sc[0] = one;
    M[0] = mk(-d0.x, -d0.y);
    M[1] = one;
    M[2] = zero;
    M[vl + 0] = mk(-d1.x, -d1.y);
    M[vl + 1] = zero;
    M[vl + 2] = one;
}

// Outer step n >= 1 (one block per problem).  With S = V_n^H U, G = U^H U,
// CV = V_n^H W, E = U^H W from the dot pass:
//   R^H R = G - S^H S (2x2 Cholesky),  [v_n, v_{n+1}] = (U - V_n S) R^{-1},
//   CQ = R^{-H} (E - S^H CV),  U' = W - V_n CV - [v_n, v_{n+1}] CQ,
//   column n-1:  H[0:n, n-1] = a + t0 S[:, 0],  H[n, n-1] = t0 R00,
//   column n:    H[0:n+2, n] = ([Cp_b + S_b; R01; R11] - [H_n (Cp_a + S_a); 0]) / R00,
//   pending n+1: a' = ([CV_a; CQ_a] - [H_n S_b; 0] - H[0:n+2, n] R01) / R11,
//                t0' = 1 / R11,
// where H_n = H[0:n+1, 0:n] (column n-1 included) and Cp the previous block's
// first-pass coefficients (H u_a = V Cp_b + u_b - H V Cp_a).  A subdiagonal
// entry (t0 R00, then R11 / R00) at most rel * |H|_F is a breakdown (flag[0] = 1,
// flag[1] = the column); the reciprocals are then 0, so nothing non-finite
// follows.  Non-finite input sets flag[0] = 2.
__global__ __launch_bounds__(256) void k_blk2_coef(int n, cd* H, int ldh, cd* b2, int vl,
                                                   double* hfro2, int* flag, double rel,
                                                   Batch bt) {
    __shared__ double sred[4][16];
    __shared__ double sv[40];
    const int pb = bt.idx[blockIdx.x];
    H += pb * bt.small;
    b2 += pb * bt.small;
    hfro2 += 2 * pb * bt.scal;
    flag += pb * bt.flag;
    const int np2 = n + 2;
    const cd* D = b2;
    cd* M = b2 + 4 * (int64_t)vl;
    cd* a = b2 + 8 * (int64_t)vl;
    cd* Cp = b2 + 9 * (int64_t)vl;
    cd* Y = b2 + 11 * (int64_t)vl;
    cd* sc = b2 + 13 * (int64_t)vl;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double t0 = sc[0].x;
    // ---- phase 1: S^H S, S^H CV, column n-1
    double acc[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) acc[q] = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        const cd s0 = D[c], s1 = D[np2 + c], v0 = D[2 * np2 + c], v1 = D[3 * np2 + c];
        acc[0] += cabs2(s0);
        acc[1] += cabs2(s1);
        const cd s01 = cmulc(s0, s1);   // conj(s0) s1
        acc[2] += s01.x;
        acc[3] += s01.y;
        const cd p00 = cmulc(s0, v0), p01 = cmulc(s0, v1), p10 = cmulc(s1, v0),
                 p11 = cmulc(s1, v1);
        acc[4] += p00.x; acc[5] += p00.y;
        acc[6] += p01.x; acc[7] += p01.y;
        acc[8] += p10.x; acc[9] += p10.y;
        acc[10] += p11.x; acc[11] += p11.y;
        const cd h = cadd(a[c], cscale(s0, t0));
        H[c + (int64_t)(n - 1) * ldh] = h;
        acc[12] += cabs2(h);
    }
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        const double x = wave_sum(acc[q]);
        if (lane == 0) sred[wave][q] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[13];
        for (int q = 0; q < 13; ++q) tot[q] = sred[0][q] + sred[1][q] + sred[2][q] + sred[3][q];
        const double g00 = D[n].x, g11 = D[np2 + n + 1].x;
        const cd g01 = D[np2 + n];   // u_a^H u_b
        const double m00 = g00 - tot[0], m11 = g11 - tot[1];
        const cd m01 = mk(g01.x - tot[2], g01.y - tot[3]);
        const double r00 = sqrt(fmax(m00, 0.0));
        // column n-1 done: its subdiagonal is t0 r00
        const double sub = t0 * r00;
        *hfro2 += tot[12];
        int bd = (sub <= rel * sqrt(*hfro2 + sub * sub)) ? 1 : 0;
        if (!(g00 == g00) || !(g11 == g11) || !(tot[12] == tot[12]) || !(m00 == m00) ||
            fabs(g00) > 1e300)
            bd = 2;
        if (bd) {
            if (flag[0] == 0) flag[1] = n - 1;
            if (bd > flag[0]) flag[0] = bd;
        }
        H[n + (int64_t)(n - 1) * ldh] = mk(sub, 0.0);
        const double ir00 = flag[0] ? 0.0 : 1.0 / r00;
        const cd r01 = cscale(m01, ir00);
        const double r11 = sqrt(fmax(m11 - cabs2(r01), 0.0));
        sv[0] = r00; sv[1] = ir00; sv[2] = r01.x; sv[3] = r01.y; sv[4] = r11;
        // E - S^H CV (row a: u_a / u_b, column o: w1 / w2)
        const cd e00 = D[2 * np2 + n], e01 = D[3 * np2 + n], e10 = D[2 * np2 + n + 1],
                 e11 = D[3 * np2 + n + 1];
        sv[5] = e00.x - tot[4];  sv[6] = e00.y - tot[5];
        sv[7] = e01.x - tot[6];  sv[8] = e01.y - tot[7];
        sv[9] = e10.x - tot[8];  sv[10] = e10.y - tot[9];
        sv[11] = e11.x - tot[10]; sv[12] = e11.y - tot[11];
    }
    __syncthreads();
    // ---- phase 2: Y0 = H_n (Cp_a + S_a), Y1 = H_n S_b, rows 0..n
    for (int r = threadIdx.x; r <= n; r += 256) {
        cd y0 = mk(0.0, 0.0), y1 = mk(0.0, 0.0);
        for (int c = (r > 0 ? r - 1 : 0); c < n; ++c) {
            const cd h = H[r + (int64_t)c * ldh];
            cfma(y0, h, cadd(Cp[c], D[c]));
            cfma(y1, h, D[np2 + c]);
        }
        Y[r] = y0;
        Y[vl + r] = y1;
    }
    __syncthreads();
    // ---- phase 3: column n
    const double ir00 = sv[1];
    const cd r01 = mk(sv[2], sv[3]);
    const double r11 = sv[4];
    double col2 = 0.0;
    for (int r = threadIdx.x; r <= n + 1; r += 256) {
        cd base;
        if (r < n) base = csub(cadd(Cp[vl + r], D[np2 + r]), Y[r]);
        else if (r == n) base = csub(r01, Y[n]);
        else base = mk(r11, 0.0);
        const cd h = cscale(base, ir00);
        H[r + (int64_t)n * ldh] = h;
        if (r <= n) col2 += cabs2(h);
    }
    col2 = wave_sum(col2);
    if (lane == 0) sred[wave][0] = col2;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
        const double sub = r11 * ir00;
        *hfro2 += tot;
        int bd = (sub <= rel * sqrt(*hfro2 + sub * sub)) ? 1 : 0;
        if (!(tot == tot) || !(r11 == r11)) bd = 2;
        if (bd) {
            if (flag[0] == 0) flag[1] = n;
            if (bd > flag[0]) flag[0] = bd;
        }
        const double ir11 = flag[0] ? 0.0 : 1.0 / r11;
        // CQ = R^{-H} F: CQ[0][o] = F[0][o] / r00, CQ[1][o] = (F[1][o] - conj(r01) CQ[0][o]) / r11
        const cd f00 = mk(sv[5], sv[6]), f01 = mk(sv[7], sv[8]), f10 = mk(sv[9], sv[10]),
                 f11 = mk(sv[11], sv[12]);
        const cd q00 = cscale(f00, ir00), q01 = cscale(f01, ir00);
        const cd q10 = cscale(csub(f10, cmulc(r01, q00)), ir11);
        const cd q11 = cscale(csub(f11, cmulc(r01, q01)), ir11);
        // R^{-1} = [[ir00, -r01 ir00 ir11], [0, ir11]];  RiCQ = R^{-1} CQ
        const cd rinv01 = cscale(r01, -ir00 * ir11);
        const cd k00 = cadd(cscale(q00, ir00), cmul(rinv01, q10));
        const cd k01 = cadd(cscale(q01, ir00), cmul(rinv01, q11));
        const cd k10 = cscale(q10, ir11), k11 = cscale(q11, ir11);
        sv[13] = ir11;
        sv[14] = rinv01.x; sv[15] = rinv01.y;
        sv[16] = q00.x; sv[17] = q00.y; sv[18] = q01.x; sv[19] = q01.y;
        sv[20] = q10.x; sv[21] = q10.y; sv[22] = q11.x; sv[23] = q11.y;
        sv[24] = k00.x; sv[25] = k00.y; sv[26] = k01.x; sv[27] = k01.y;
        sv[28] = k10.x; sv[29] = k10.y; sv[30] = k11.x; sv[31] = k11.y;
    }
    __syncthreads();
    // ---- phase 4: update coefficients, pending column n+1, next first-pass block
    const double ir11 = sv[13];
    const cd rinv01 = mk(sv[14], sv[15]);
    const cd q00 = mk(sv[16], sv[17]), q01 = mk(sv[18], sv[19]);
    const cd q10 = mk(sv[20], sv[21]), q11 = mk(sv[22], sv[23]);
    const cd k00 = mk(sv[24], sv[25]), k01 = mk(sv[26], sv[27]);
    const cd k10 = mk(sv[28], sv[29]), k11 = mk(sv[30], sv[31]);
    const cd zero = mk(0.0, 0.0);
    for (int c = threadIdx.x; c < n + 4; c += 256) {
        cd m0, m1, m2, m3;
        if (c < n) {
            const cd s0 = D[c], s1 = D[np2 + c], v0 = D[2 * np2 + c], v1 = D[3 * np2 + c];
            const cd sr0 = cscale(s0, ir00);
            const cd sr1 = cscale(csub(s1, cmul(sr0, r01)), ir11);
            m0 = mk(-sr0.x, -sr0.y);
            m1 = mk(-sr1.x, -sr1.y);
            const cd t2 = csub(v0, cadd(cmul(sr0, q00), cmul(sr1, q10)));
            const cd t3 = csub(v1, cadd(cmul(sr0, q01), cmul(sr1, q11)));
            m2 = mk(-t2.x, -t2.y);
            m3 = mk(-t3.x, -t3.y);
        } else if (c == n) {
            m0 = mk(ir00, 0.0); m1 = rinv01; m2 = mk(-k00.x, -k00.y); m3 = mk(-k01.x, -k01.y);
        } else if (c == n + 1) {
            m0 = zero; m1 = mk(ir11, 0.0); m2 = mk(-k10.x, -k10.y); m3 = mk(-k11.x, -k11.y);
        } else if (c == n + 2) {
            m0 = zero; m1 = zero; m2 = mk(1.0, 0.0); m3 = zero;
        } else {
            m0 = zero; m1 = zero; m2 = zero; m3 = mk(1.0, 0.0);
        }
        M[c] = m0;
        M[vl + c] = m1;
        M[2 * (int64_t)vl + c] = m2;
        M[3 * (int64_t)vl + c] = m3;
    }
    for (int r = threadIdx.x; r < n + 2; r += 256) {
        cd cva, cvb;
        if (r < n) { cva = D[2 * np2 + r]; cvb = D[3 * np2 + r]; }
        else if (r == n) { cva = q00; cvb = q01; }
        else { cva = q10; cvb = q11; }
        const cd y1 = (r <= n) ? Y[vl + r] : zero;
        const cd hn = H[r + (int64_t)n * ldh];
        a[r] = cscale(csub(csub(cva, y1), cmul(hn, r01)), ir11);
        Cp[r] = cva;
        Cp[vl + r] = cvb;
    }
    if (threadIdx.x == 0) sc[0] = mk(ir11, 0.0);
}

void launch_blk2_init(cd* b2, int vl, const cd* d, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    hipLaunchKernelGGL(k_blk2_init, dim3((unsigned)bt.n), dim3(64), 0, st, b2, vl, d, bt);
    OSA_LAUNCH_CHECK();
}

void launch_blk2_coef(int n, cd* H, int ldh, cd* b2, int vl, double* hfro2, int* flag,
                      double rel, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    hipLaunchKernelGGL(k_blk2_coef, dim3((unsigned)bt.n), dim3(256), 0, st, n, H, ldh, b2, vl,
                       hfro2, flag, rel, bt);
    OSA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- norms
template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm_partial(const T* __restrict__ w, int64_t n,
                                                         double* normp, Batch bt) {
    __shared__ double sm[kWaves];
    __shared__ double so[1];
    const int pb = bt.idx[blockIdx.y];
    w += pb * bt.vec;
    normp += pb * bt.part;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double nv[1] = {(i < n) ? cabs2(tod(w[i])) : 0.0};
    block_sum<1>(nv, sm, so);
    if (threadIdx.x == 0) normp[blockIdx.x] = so[0];
}

void launch_norm_partial(const void* w, bool fp32, const TsPlan& p, double* normp,
                         hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const int rb = (int)ceil_div(p.n, kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_norm_partial<cf>), dim3(rb, bt.n), dim3(kBlock), 0, st,
                           (const cf*)w, p.n, normp, bt);
    else
        hipLaunchKernelGGL((k_norm_partial<cd>), dim3(rb, bt.n), dim3(kBlock), 0, st,
                           (const cd*)w, p.n, normp, bt);
    OSA_LAUNCH_CHECK();
}

// one block per problem: hsub = sqrt(sum normp) (+ breakdown test)
__global__ __launch_bounds__(1024) void k_norm_finish(const double* __restrict__ normp, int nb,
                                                      cd* hsub, double* hfro2, double rel,
                                                      int* flag, int step,
                                                      const cd* __restrict__ hcol, int hlen,
                                                      Batch bt) {
    __shared__ double sred[16];
    __shared__ double shcol;
    const int pb = bt.idx[blockIdx.x];
    normp += pb * bt.part;
    hsub += pb * bt.scal;
    if (hfro2) hfro2 += 2 * pb * bt.scal;
    if (flag) flag += pb * bt.flag;
    if (hcol) hcol += pb * bt.small;
    if (hcol && hfro2) {
        double a = 0;
        for (int i = threadIdx.x; i < hlen; i += blockDim.x) a += cabs2(hcol[i]);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        a = wave_sum(a);
        if (lane == 0) sred[wave] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sred[w];
            shcol = t;
        }
        __syncthreads();
    }
    double loc = 0;
    // fixed order: contiguous slices per thread, then a fixed tree
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int b0 = threadIdx.x * per;
    for (int b = b0; b < b0 + per && b < nb; ++b) loc += normp[b];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s = wave_sum(loc);
    if (lane == 0) sred[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sred[w];
        double h = sqrt(t);
        if (hcol && hfro2) *hfro2 += shcol;
        double scale = hfro2 ? sqrt(*hfro2 + t) : 0.0;
        int bd = (flag && h <= rel * scale) ? 1 : 0;
        if (!(h == h) || h > 1e300) bd = 2;   // non-finite
        if (flag && bd) {
            if (flag[0] == 0) flag[1] = step;
            if (bd > flag[0]) flag[0] = bd;
        }
        hsub->x = h;
        hsub->y = 0.0;
    }
}

// v = w / f (divide) or w * f with f = factor->x; v = 0 when flag is set.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_by(const T* __restrict__ w, T* __restrict__ v,
                                                     int64_t n, const cd* factor, const int* flag,
                                                     int divide, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    w += pb * bt.vec;
    v += pb * bt.basis;
    factor += pb * bt.scal;
    if (flag) flag += pb * bt.flag;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const bool bd = flag && *flag;
    const double f = bd ? 0.0 : (divide ? 1.0 / factor->x : factor->x);
    v[i] = fromd<T>(cscale(tod(w[i]), f));
}

void launch_normalize(const void* w, void* v, bool fp32, const TsPlan& p, const double* normp,
                      cd* hsub, double* hfro2, double rel, int* flag, int step,
                      const cd* hcol, int hlen, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const int nb = (int)ceil_div(p.n, kBlock);
    hipLaunchKernelGGL(k_norm_finish, dim3((unsigned)bt.n), dim3(256), 0, st, normp, nb, hsub,
                       hfro2, rel, flag, step, hcol, hlen, bt);
    if (!v) { OSA_LAUNCH_CHECK(); return; }
    const int rb = (int)ceil_div(p.n, kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_scale_by<cf>), dim3(rb, bt.n), dim3(kBlock), 0, st, (const cf*)w,
                           (cf*)v, p.n, (const cd*)hsub, (const int*)flag, 1, bt);
    else
        hipLaunchKernelGGL((k_scale_by<cd>), dim3(rb, bt.n), dim3(kBlock), 0, st, (const cd*)w,
                           (cd*)v, p.n, (const cd*)hsub, (const int*)flag, 1, bt);
    OSA_LAUNCH_CHECK();
}

void launch_scale_dev(const void* w, void* v, bool fp32, int64_t n, const cd* factor, bool divide,
                      hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const int rb = (int)ceil_div(n, kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_scale_by<cf>), dim3(rb, bt.n), dim3(kBlock), 0, st, (const cf*)w,
                           (cf*)v, n, factor, (const int*)nullptr, divide ? 1 : 0, bt);
    else
        hipLaunchKernelGGL((k_scale_by<cd>), dim3(rb, bt.n), dim3(kBlock), 0, st, (const cd*)w,
                           (cd*)v, n, factor, (const int*)nullptr, divide ? 1 : 0, bt);
    OSA_LAUNCH_CHECK();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale(const T* __restrict__ w, T* __restrict__ v,
                                                  int64_t n, double a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = fromd<T>(cscale(tod(w[i]), a));
}

void launch_scale(const void* w, void* v, bool fp32, int64_t n, double alpha, hipStream_t st) {
    const int rb = (int)ceil_div(n, kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_scale<cf>), dim3(rb), dim3(kBlock), 0, st, (const cf*)w, (cf*)v, n,
                           alpha);
    else
        hipLaunchKernelGGL((k_scale<cd>), dim3(rb), dim3(kBlock), 0, st, (const cd*)w, (cd*)v, n,
                           alpha);
    OSA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- rotate
// out[:, c] = sum_r B[:, r] Z[r, c]; each block: 256 rows x 8 output columns.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rotate(const T* __restrict__ B, int64_t ldb, int p,
                                                   const cd* __restrict__ Z, int ldz, int q,
                                                   T* __restrict__ out, int64_t ldo, int64_t n) {
    constexpr int C = 8;
    __shared__ cd sz[128 * C];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int c0 = blockIdx.y * C;
    const int nc = (q - c0 < C) ? q - c0 : C;
    for (int e = threadIdx.x; e < p * C; e += kBlock) {
        const int r = e / C, cc = e % C;
        sz[e] = (cc < nc) ? Z[r + (int64_t)(c0 + cc) * ldz] : mk(0.0, 0.0);
    }
    __syncthreads();
    if (i >= n) return;
    cd acc[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) acc[cc] = mk(0.0, 0.0);
    for (int r = 0; r < p; ++r) {
        const cd b = tod(B[(int64_t)r * ldb + i]);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) cfma(acc[cc], b, sz[r * C + cc]);
    }
#pragma unroll
    for (int cc = 0; cc < C; ++cc)
        if (cc < nc) out[(int64_t)(c0 + cc) * ldo + i] = fromd<T>(acc[cc]);
}

void launch_rotate(const void* B, int64_t ldb, int ncols_in, const cd* Z, int ldz, int ncols_out,
                   void* out, int64_t ldo, bool fp32, int64_t n, hipStream_t st) {
    if (ncols_in > 128) throw HipError{hipErrorInvalidValue, "launch_rotate: p > 128"};
    dim3 grid((unsigned)ceil_div(n, kBlock), (unsigned)ceil_div(ncols_out, 8)), blk(kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_rotate<cf>), grid, blk, 0, st, (const cf*)B, ldb, ncols_in, Z, ldz,
                           ncols_out, (cf*)out, ldo, n);
    else
        hipLaunchKernelGGL((k_rotate<cd>), grid, blk, 0, st, (const cd*)B, ldb, ncols_in, Z, ldz,
                           ncols_out, (cd*)out, ldo, n);
    OSA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- misc
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_convert(const TI* __restrict__ s, TO* __restrict__ d,
                                                    int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d[i] = fromd<TO>(tod(s[i]));
}

void launch_convert(const void* src, bool src_fp32, void* dst, bool dst_fp32, int64_t n,
                    hipStream_t st) {
    const int rb = (int)ceil_div(n, kBlock);
    if (src_fp32 && !dst_fp32)
        hipLaunchKernelGGL((k_convert<cf, cd>), dim3(rb), dim3(kBlock), 0, st, (const cf*)src,
                           (cd*)dst, n);
    else if (!src_fp32 && dst_fp32)
        hipLaunchKernelGGL((k_convert<cd, cf>), dim3(rb), dim3(kBlock), 0, st, (const cd*)src,
                           (cf*)dst, n);
    else if (src_fp32)
        hipLaunchKernelGGL((k_convert<cf, cf>), dim3(rb), dim3(kBlock), 0, st, (const cf*)src,
                           (cf*)dst, n);
    else
        hipLaunchKernelGGL((k_convert<cd, cd>), dim3(rb), dim3(kBlock), 0, st, (const cd*)src,
                           (cd*)dst, n);
    OSA_LAUNCH_CHECK();
}

// Zero `bytes` bytes (a multiple of 4) with a kernel: unlike hipMemsetAsync it
// records as an ordinary kernel node when a caller captures the stream.
__global__ __launch_bounds__(kBlock) void k_fill_zero(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0u;
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st,
                       (uint32_t*)p, n);
    OSA_LAUNCH_CHECK();
}

// splitmix64 finaliser as a counter-based generator
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_random(T* v, int V, int Vp, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 12LL * Vp) return;
    const int s = (int)(i % Vp);
    cd z = mk(0.0, 0.0);
    if (s < V) {
        uint64_t a = mix64(seed * 0x2545F4914F6CDD1DULL + 2 * (uint64_t)i);
        uint64_t b = mix64(seed * 0x2545F4914F6CDD1DULL + 2 * (uint64_t)i + 1);
        double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double r = sqrt(-2.0 * log(u1));
        z = mk(r * cos(6.283185307179586 * u2), r * sin(6.283185307179586 * u2));
    }
    v[i] = fromd<T>(z);
}

void launch_random_vector(void* v, bool fp32, const Geom& g, uint64_t seed, hipStream_t st) {
    const int rb = (int)ceil_div(12LL * g.Vp, kBlock);
    if (fp32)
        hipLaunchKernelGGL((k_random<cf>), dim3(rb), dim3(kBlock), 0, st, (cf*)v, g.V, g.Vp, seed);
    else
        hipLaunchKernelGGL((k_random<cd>), dim3(rb), dim3(kBlock), 0, st, (cd*)v, g.V, g.Vp, seed);
    OSA_LAUNCH_CHECK();
}

}  // namespace osa
