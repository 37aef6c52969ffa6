// Small dense kernels: the sign of the Hessenberg matrix f(H_k) e_1 (Eq. 11,
// Eq. 22) by the scaled Newton iteration, and the small Schur decomposition
// used by the eigensolver restarts.
#include <algorithm>

#include "kernels.hpp"

namespace osa {

// ====================================================================== GJ
// In-place Gauss-Jordan inversion with implicit partial row pivoting.
// Step t picks the unused row p with the largest |M[p,t]|, scales it by
// 1/M[p,t] and eliminates column t from every other row; column t then stores
// the new column of the accumulated row operations.  At the end
//   A^{-1}[t, c] = M[perm[t], pinv[c]],   pinv[perm[s]] = s.
// Each block owns a few whole columns, so reading and writing the pivot row of
// a column happen inside one block; the next pivot column is handed on from
// step to step through a double-buffered copy written by its owner.  Up to
// k = kGjPairMax one launch takes two pivots (k_gj_step2) with the arithmetic
// of two single steps; blocked (panel) schedules measured no faster here, their
// per-step critical path on one compute unit being as long as a launch.
struct GjWs {
    cd* col;        // 2 x 2 x k: two buffer sets of (column t, column t+1)
    double2* piv;   // k: (|value|, index) of the pivot chosen for step t
    int* perm;      // k
    int* pinv;      // k
    int* used;      // k: 0, or s + 1 for the pivot row of step s
};

size_t gj_ws_bytes(int k) {
    return (size_t)k * (4 * sizeof(cd) + sizeof(double2) + 3 * sizeof(int)) + 256;
}

// the workspace of problem pb of a batch (byte stride bt.ws)
__device__ __forceinline__ GjWs gj_at(GjWs w, const Batch& bt, int pb) {
    const int64_t off = pb * bt.ws;
    w.col = (cd*)((char*)w.col + off);
    w.piv = (double2*)((char*)w.piv + off);
    w.perm = (int*)((char*)w.perm + off);
    w.pinv = (int*)((char*)w.pinv + off);
    w.used = (int*)((char*)w.used + off);
    return w;
}

// Row i was the pivot of a step before step t.  Block 0 marks the pivot rows
// of a launch at its end, while other blocks of the same launch may still be
// choosing pivots: marks of step t or later must not count, or a block that
// runs after block 0 would skip the row the others chose.
__device__ __forceinline__ bool used_before(int u, int t) { return u != 0 && u <= t; }

static GjWs gj_ws(void* ws, int k) {
    char* p = (char*)ws;
    GjWs w;
    w.col = (cd*)p;            p += (size_t)4 * k * sizeof(cd);
    w.piv = (double2*)p;       p += (size_t)k * sizeof(double2);
    w.perm = (int*)p;          p += (size_t)k * sizeof(int);
    w.pinv = (int*)p;          p += (size_t)k * sizeof(int);
    w.used = (int*)p;
    return w;
}

// a * b and v - f * rp with one fixed rounding sequence (explicit fma, so that
// contraction cannot differ between call sites)
__device__ __forceinline__ cd gj_mul(cd a, cd b) {
    return mk(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ cd gj_sub(cd v, cd f, cd rp) {
    const cd q = gj_mul(f, rp);
    return mk(v.x - q.x, v.y - q.y);
}

static constexpr int kGjThreads = 256;
static constexpr int kGjCols = 4;
static constexpr int kGjPairMax = 2048;   // two pivots per launch up to this k (LDS column)

__device__ __forceinline__ void argmax_pair(double& v, int& idx, double ov, int oi) {
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
}

// block-wide argmax (ties -> smaller index), result valid in thread 0
__device__ void block_argmax(double v, int idx, double* sv, int* si, double& ov, int& oi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double v2 = __shfl_xor(v, off, 64);
        int i2 = __shfl_xor(idx, off, 64);
        argmax_pair(v, idx, v2, i2);
    }
    if (lane == 0) { sv[wave] = v; si[wave] = idx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bv = sv[0];
        int bi = si[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) argmax_pair(bv, bi, sv[w], si[w]);
        ov = bv;
        oi = bi;
    }
}

__global__ __launch_bounds__(kGjThreads) void k_gj_init(const cd* __restrict__ M, int k, GjWs w,
                                                       Batch bt) {
    __shared__ double sv[kGjThreads / 64];
    __shared__ int si[kGjThreads / 64];
    const int pb = bt.idx[blockIdx.x];
    M += pb * bt.mat;
    w = gj_at(w, bt, pb);
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < k; i += kGjThreads) {
        cd v = M[i];
        w.col[i] = v;
        if (k > 1) w.col[k + i] = M[i + (size_t)k];
        w.used[i] = 0;
        w.perm[i] = i;
        w.pinv[i] = i;
        argmax_pair(bv, bi, cabsd(v), i);
    }
    double ov;
    int oi;
    block_argmax(bv, bi, sv, si, ov, oi);
    if (threadIdx.x == 0) w.piv[0] = make_double2(ov, (double)oi);
}

__global__ __launch_bounds__(kGjThreads) void k_gj_step(cd* __restrict__ M, int k, int t, int rb,
                                                       GjWs w, double* logpiv, int* flag, Batch bt) {
    __shared__ double sv[kGjThreads / 64];
    __shared__ int si[kGjThreads / 64];
    const int pb = bt.idx[blockIdx.y];
    M += pb * bt.mat;
    w = gj_at(w, bt, pb);
    logpiv += pb * bt.small;
    flag += pb * bt.flag;
    const cd* colc = w.col + (size_t)(2 * rb) * k;   // column t, from buffer set rb
    cd* coln = w.col + (size_t)(2 * (rb ^ 1)) * k;   // column t+1, for the next launch
    // A column of NaNs selects no pivot; keep every index in range and flag it.
    const double pf = w.piv[t].y;
    const bool badp = !(pf >= 0.0 && pf < (double)k);
    const int p = badp ? t : (int)pf;
    const cd piv = colc[p];
    const bool zero = badp || (piv.x == 0.0 && piv.y == 0.0);
    const cd ipiv = zero ? mk(0.0, 0.0) : cinv(piv);
    const int j0 = blockIdx.x * kGjCols;
    for (int j = j0; j < j0 + kGjCols && j < k; ++j) {
        const cd r = (j == t) ? mk(1.0, 0.0) : M[p + (size_t)j * k];
        __syncthreads();   // everyone has read M[p,j] before row p is rewritten
        const cd rp = gj_mul(r, ipiv);
        const bool nextcol = (j == t + 1);
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int i = threadIdx.x; i < k; i += kGjThreads) {
            const cd f = colc[i];
            cd nv;
            if (j == t) {
                if (i == p) nv = ipiv;
                else { const cd q = gj_mul(f, ipiv); nv = mk(-q.x, -q.y); }
            } else {
                nv = (i == p) ? rp : gj_sub(M[i + (size_t)j * k], f, rp);
            }
            M[i + (size_t)j * k] = nv;
            if (nextcol) {
                coln[i] = nv;
                if (i != p && !used_before(w.used[i], t)) argmax_pair(bv, bi, cabsd(nv), i);
            }
        }
        if (nextcol) {
            double ov;
            int oi;
            block_argmax(bv, bi, sv, si, ov, oi);
            if (threadIdx.x == 0) w.piv[t + 1] = make_double2(ov, (double)oi);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.perm[t] = p;
        w.used[p] = t + 1;
        logpiv[t] = zero ? -1e300 : log(cabsd(piv));
        if (zero || !(piv.x == piv.x) || !(piv.y == piv.y)) *flag = 1;
    }
}

// Steps t and t+1 in one launch, with the arithmetic of two k_gj_step
// launches: every block forms column t+1 after step t (from the buffered
// columns t and t+1) and the pivot of step t+1, then applies both steps to its
// columns in one pass over them.  The owners of columns t+2 and t+3 buffer them
// for the next launch; the owner of column t+2 also picks its pivot.
__global__ __launch_bounds__(kGjThreads) void k_gj_step2(cd* __restrict__ M, int k, int t, int rb,
                                                        GjWs w, double* logpiv, int* flag,
                                                        Batch bt) {
    extern __shared__ cd c1[];   // column t+1 after step t
    __shared__ double sv[kGjThreads / 64];
    __shared__ int si[kGjThreads / 64];
    __shared__ int sp1;
    const int pb = bt.idx[blockIdx.y];
    M += pb * bt.mat;
    w = gj_at(w, bt, pb);
    logpiv += pb * bt.small;
    flag += pb * bt.flag;
    const cd* colA = w.col + (size_t)(2 * rb) * k;   // column t before step t
    const cd* colB = colA + k;                        // column t+1 before step t
    cd* outA = w.col + (size_t)(2 * (rb ^ 1)) * k;    // column t+2 after step t+1
    cd* outB = outA + k;                              // column t+3 after step t+1
    const double pf = w.piv[t].y;
    const bool badp = !(pf >= 0.0 && pf < (double)k);
    const int p = badp ? t : (int)pf;
    const cd piv = colA[p];
    const bool zero = badp || (piv.x == 0.0 && piv.y == 0.0);
    const cd ipiv = zero ? mk(0.0, 0.0) : cinv(piv);
    {
        const cd rp = gj_mul(colB[p], ipiv);
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int i = threadIdx.x; i < k; i += kGjThreads) {
            const cd nv = (i == p) ? rp : gj_sub(colB[i], colA[i], rp);
            c1[i] = nv;
            if (i != p && !used_before(w.used[i], t)) argmax_pair(bv, bi, cabsd(nv), i);
        }
        double ov = 0.0;
        int oi = 0;
        block_argmax(bv, bi, sv, si, ov, oi);
        if (threadIdx.x == 0) {
            sp1 = oi;
            if (blockIdx.x == 0) w.piv[t + 1] = make_double2(ov, (double)oi);
        }
        __syncthreads();
    }
    const int q1 = sp1;
    const bool badp1 = !(q1 >= 0 && q1 < k);
    const int p1 = badp1 ? t + 1 : q1;
    const cd piv1 = c1[p1];
    const bool zero1 = badp1 || (piv1.x == 0.0 && piv1.y == 0.0);
    const cd ipiv1 = zero1 ? mk(0.0, 0.0) : cinv(piv1);
    const int j0 = blockIdx.x * kGjCols;
    for (int j = j0; j < j0 + kGjCols && j < k; ++j) {
        // pivot-row values: step t reads row p, step t+1 row p1 after step t
        const cd r0 = (j == t) ? mk(1.0, 0.0) : M[p + (size_t)j * k];
        const cd rp0 = gj_mul(r0, ipiv);
        cd r1 = mk(1.0, 0.0);
        if (j == t) {
            if (p1 == p) r1 = ipiv;
            else { const cd q = gj_mul(colA[p1], ipiv); r1 = mk(-q.x, -q.y); }
        } else if (j != t + 1) {
            r1 = (p1 == p) ? rp0 : gj_sub(M[p1 + (size_t)j * k], colA[p1], rp0);
        }
        __syncthreads();   // everyone has read rows p and p1 of column j before it is rewritten
        const cd rp1 = gj_mul(r1, ipiv1);
        const bool nextA = (j == t + 2), nextB = (j == t + 3);
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int i = threadIdx.x; i < k; i += kGjThreads) {
            cd nv;
            if (j == t + 1) {   // the pivot column of step t+1
                if (i == p1) nv = ipiv1;
                else { const cd q = gj_mul(c1[i], ipiv1); nv = mk(-q.x, -q.y); }
            } else {
                cd v;   // column j after step t
                if (j == t) {
                    if (i == p) v = ipiv;
                    else { const cd q = gj_mul(colA[i], ipiv); v = mk(-q.x, -q.y); }
                } else {
                    v = (i == p) ? rp0 : gj_sub(M[i + (size_t)j * k], colA[i], rp0);
                }
                nv = (i == p1) ? rp1 : gj_sub(v, c1[i], rp1);
            }
            M[i + (size_t)j * k] = nv;
            if (nextA) {
                outA[i] = nv;
                if (i != p && i != p1 && !used_before(w.used[i], t)) argmax_pair(bv, bi, cabsd(nv), i);
            }
            if (nextB) outB[i] = nv;
        }
        if (nextA) {
            double ov;
            int oi;
            block_argmax(bv, bi, sv, si, ov, oi);
            if (threadIdx.x == 0) w.piv[t + 2] = make_double2(ov, (double)oi);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.perm[t] = p;
        w.used[p] = t + 1;
        logpiv[t] = zero ? -1e300 : log(cabsd(piv));
        if (zero || !(piv.x == piv.x) || !(piv.y == piv.y)) *flag = 1;
        w.perm[t + 1] = p1;
        w.used[p1] = t + 2;
        logpiv[t + 1] = zero1 ? -1e300 : log(cabsd(piv1));
        if (zero1 || !(piv1.x == piv1.x) || !(piv1.y == piv1.y)) *flag = 1;
    }
}

__global__ void k_gj_pinv(int k, GjWs w, Batch bt) {
    w = gj_at(w, bt, bt.idx[blockIdx.y]);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < k; s += gridDim.x * blockDim.x) {
        const int q = w.perm[s];
        if (q >= 0 && q < k) w.pinv[q] = s;
    }
}

__global__ __launch_bounds__(256) void k_gj_gather(const cd* __restrict__ M, cd* __restrict__ Y,
                                                  int k, GjWs w, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    M += pb * bt.mat;
    Y += pb * bt.mat;
    w = gj_at(w, bt, pb);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int t = (int)(e % k), c = (int)(e / k);
    int r = w.perm[t], q = w.pinv[c];
    r = (r >= 0 && r < k) ? r : 0;   // only reachable after a flagged breakdown
    q = (q >= 0 && q < k) ? q : 0;
    Y[e] = M[r + (size_t)q * k];
}

void gj_invert(cd* M, cd* Y, int k, double* logpiv, int* flag, void* ws, hipStream_t st,
               const Batch& bt) {
    if (bt.n <= 0) return;
    GjWs w = gj_ws(ws, k);
    const unsigned nbt = (unsigned)bt.n;
    hipLaunchKernelGGL(k_gj_init, dim3(nbt), dim3(kGjThreads), 0, st, (const cd*)M, k, w, bt);
    const int nb = (int)ceil_div(k, kGjCols);
    int t = 0, rb = 0;
    if (k <= kGjPairMax)
        for (; t + 1 < k; t += 2, rb ^= 1)
            hipLaunchKernelGGL(k_gj_step2, dim3(nb, nbt), dim3(kGjThreads), sizeof(cd) * (size_t)k,
                               st, M, k, t, rb, w, logpiv, flag, bt);
    for (; t < k; ++t, rb ^= 1)
        hipLaunchKernelGGL(k_gj_step, dim3(nb, nbt), dim3(kGjThreads), 0, st, M, k, t, rb, w,
                           logpiv, flag, bt);
    hipLaunchKernelGGL(k_gj_pinv, dim3((unsigned)ceil_div(k, 256), nbt), dim3(256), 0, st, k, w,
                       bt);
    if (Y) {
        hipLaunchKernelGGL(k_gj_gather, dim3((unsigned)ceil_div((int64_t)k * k, 256), nbt),
                           dim3(256), 0, st, (const cd*)M, Y, k, w, bt);
    }
    OSA_LAUNCH_CHECK();
}

// ================================================================ Newton
// Scaled Newton step for sign(X) (Roberts; determinantal scaling of Byers):
//   X <- (mu X + (mu X)^{-1}) / 2,  mu = |det X|^{-1/k} = exp(-sum log|piv| / k)
// Y holds X^{-1}.  Per-block partial sums of |Xnew - X|^2 and |Xnew|^2.
__global__ __launch_bounds__(256) void k_newton_combine(cd* __restrict__ X, const cd* __restrict__ Y,
                                                       int k, const double* __restrict__ logpiv,
                                                       uint64_t scale_mask, double* part,
                                                       Batch bt) {
    __shared__ double sm[8];
    __shared__ double smu;
    const int pb = bt.idx[blockIdx.y];
    X += pb * bt.mat;
    Y += pb * bt.mat;
    logpiv += pb * bt.small;
    part += pb * bt.part + 2;
    const bool scale = (scale_mask >> pb) & 1ULL;
    if (threadIdx.x == 0) {
        double mu = 1.0;
        if (scale) {
            double s = 0;
            for (int t = 0; t < k; ++t) s += logpiv[t];
            mu = exp(-s / k);
        }
        smu = mu;
    }
    __syncthreads();
    const double mu = smu, imu = 1.0 / mu;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d2 = 0, n2 = 0;
    if (e < (int64_t)k * k) {
        cd x = X[e], y = Y[e];
        cd xn = mk(0.5 * (mu * x.x + imu * y.x), 0.5 * (mu * x.y + imu * y.y));
        d2 = cabs2(csub(xn, x));
        n2 = cabs2(xn);
        X[e] = xn;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off, 64);
        n2 += __shfl_xor(n2, off, 64);
    }
    if (lane == 0) { sm[2 * wave] = d2; sm[2 * wave + 1] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int w = 0; w < 4; ++w) { a += sm[2 * w]; b += sm[2 * w + 1]; }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// red[0..1] = sums of the per-block partials: one wavefront per problem, lane q
// takes blocks q, q + 64, ... in order, then a fixed shuffle tree.
__global__ __launch_bounds__(64) void k_sum_pairs(const double* __restrict__ part, int nb,
                                                  double* red, Batch bt) {
    const int pb = bt.idx[blockIdx.x];
    red += pb * bt.part;
    part = red + 2;
    double a = 0, b = 0;
    for (int i = threadIdx.x; i < nb; i += 64) { a += part[2 * i]; b += part[2 * i + 1]; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if (threadIdx.x == 0) { red[0] = a; red[1] = b; }
}

int64_t newton_red_len(int k) { return 2 + 2 * ceil_div((int64_t)k * k, 256); }

void launch_newton_combine(cd* X, const cd* Y, int k, const double* logpiv, uint64_t scale_mask,
                           double* red, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    const int nb = (int)ceil_div((int64_t)k * k, 256);
    // per problem: red[0..1] the sums, red[2..] the per-block partials
    hipLaunchKernelGGL(k_newton_combine, dim3(nb, bt.n), dim3(256), 0, st, X, Y, k, logpiv,
                       scale_mask, red, bt);
    hipLaunchKernelGGL(k_sum_pairs, dim3(bt.n), dim3(64), 0, st, (const double*)nullptr, nb, red,
                       bt);
    OSA_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_copy_square(const cd* __restrict__ A, int lda,
                                                    cd* __restrict__ X, int k, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    A += pb * bt.basis;
    X += pb * bt.mat;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int i = (int)(e % k), j = (int)(e / k);
    X[e] = A[i + (int64_t)j * lda];
}

void launch_copy_square(const cd* A, int lda, cd* X, int k, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_copy_square, dim3((unsigned)ceil_div((int64_t)k * k, 256), bt.n),
                       dim3(256), 0, st, A, lda, X, k, bt);
    OSA_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_copy_col(const cd* __restrict__ X, int k,
                                                 cd* __restrict__ s, Batch bt) {
    const int pb = bt.idx[blockIdx.y];
    X += pb * bt.mat;
    s += pb * bt.small;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) s[i] = X[i];
}

void launch_copy_col0(const cd* X, int k, cd* s, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_copy_col, dim3((unsigned)ceil_div(k, 256), bt.n), dim3(256), 0, st, X, k,
                       s, bt);
    OSA_LAUNCH_CHECK();
}

// ================================================================= zgemm
// C = alpha op(A) op(B) + beta C, 16x16 tiles, column-major.
__global__ __launch_bounds__(256) void k_zgemm(int opA, int opB, int m, int n, int kk, cd alpha,
                                              const cd* __restrict__ A, int lda,
                                              const cd* __restrict__ B, int ldb, cd beta, cd* C,
                                              int ldc) {
    __shared__ cd sa[16][17];
    __shared__ cd sb[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.x * 16 + tx, col = blockIdx.y * 16 + ty;
    cd acc = mk(0.0, 0.0);
    for (int k0 = 0; k0 < kk; k0 += 16) {
        // op(A)[row, k0+ty]
        {
            const int r = blockIdx.x * 16 + tx, kq = k0 + ty;
            cd v = mk(0.0, 0.0);
            if (r < m && kq < kk) v = opA ? cconj(A[kq + (size_t)r * lda]) : A[r + (size_t)kq * lda];
            sa[tx][ty] = v;
        }
        // op(B)[k0+tx, col]
        {
            const int kq = k0 + tx, c = blockIdx.y * 16 + ty;
            cd v = mk(0.0, 0.0);
            if (c < n && kq < kk) v = opB ? cconj(B[c + (size_t)kq * ldb]) : B[kq + (size_t)c * ldb];
            sb[tx][ty] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) cfma(acc, sa[tx][q], sb[q][ty]);
        __syncthreads();
    }
    if (row < m && col < n) {
        cd r = cmul(alpha, acc);
        if (beta.x != 0.0 || beta.y != 0.0) r = cadd(r, cmul(beta, C[row + (size_t)col * ldc]));
        C[row + (size_t)col * ldc] = r;
    }
}

void launch_zgemm(int opA, int opB, int m, int n, int kk, cd alpha, const cd* A, int lda,
                  const cd* B, int ldb, cd beta, cd* C, int ldc, hipStream_t st) {
    if (m <= 0 || n <= 0) return;
    dim3 grid((unsigned)ceil_div(m, 16), (unsigned)ceil_div(n, 16));
    hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, st, opA, opB, m, n, kk, alpha, A, lda, B, ldb,
                       beta, C, ldc);
    OSA_LAUNCH_CHECK();
}

// ============================================================ zgemm (MFMA)
// Out = alpha A B + beta Cin + delta I for square n x n complex128 matrices
// (column-major, ld n), one problem per grid z entry, on the FP64 matrix
// cores.  The complex product is four real products per 16x16x4 step,
//   Re += Ar Br - Ai Bi,   Im += Ar Bi + Ai Br,
// each one v_mfma_f64_16x16x4 (FP64 fused multiply-add inside the unit, so
// the accumulation is FP64 throughout and its order is fixed).  A workgroup
// owns a 32 x 32 complex tile of Out; its four wavefronts own 16 x 16 quarters.
// k advances in chunks of 32 staged in LDS: A as [k][i] and B as [j][k], both
// padded by one entry so that the fragment reads of a wavefront spread over
// the banks.  Operand fragments: lane l holds A[i0 + l%16][k + l/16] and
// B[k + l/16][j0 + l%16]; result register r of lane l is
// Out[i0 + l/16 + 4r][j0 + l%16] (checked against numpy by the GEMM test).
typedef double d4v __attribute__((ext_vector_type(4)));
static constexpr int kMmT = 32;   // workgroup tile (complex rows and columns)
static constexpr int kMmK = 32;   // k chunk staged in LDS

__global__ __launch_bounds__(256) void k_zgemm_mfma(int n, cd alpha, const cd* __restrict__ A,
                                                   const cd* __restrict__ B, double beta,
                                                   const cd* Cin, double delta, cd* Out,
                                                   double* __restrict__ part, Batch bt) {
    __shared__ cd As[kMmK][kMmT + 1];
    __shared__ cd Bs[kMmT][kMmK + 1];
    __shared__ double sred[4];
    const int pb = bt.idx[blockIdx.z];
    A += pb * bt.mat;
    B += pb * bt.mat;
    Out += pb * bt.mat;
    if (Cin) Cin += pb * bt.mat;
    const int i0 = blockIdx.x * kMmT, j0 = blockIdx.y * kMmT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wi = (wave & 1) * 16, wj = (wave >> 1) * 16;
    const int fr = lane & 15, fk = lane >> 4;
    d4v cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += kMmK) {
        for (int e = t; e < kMmT * kMmK; e += 256) {
            const int r = e % kMmT, c = e / kMmT;
            const int ai = i0 + r, ak = k0 + c;   // A[ai, ak]: consecutive rows per column
            As[c][r] = (ai < n && ak < n) ? A[ai + (int64_t)ak * n] : mk(0.0, 0.0);
            const int bk = k0 + r, bj = j0 + c;   // B[bk, bj]
            Bs[c][r] = (bk < n && bj < n) ? B[bk + (int64_t)bj * n] : mk(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kMmK; kk += 4) {
            const cd a = As[kk + fk][wi + fr];
            const cd b = Bs[wj + fr][kk + fk];
            cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
        }
        __syncthreads();
    }
    double nrm = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + wi + fk + 4 * r, col = j0 + wj + fr;
        if (row < n && col < n) {
            const int64_t e = row + (int64_t)col * n;
            const cd acc = mk(cr[r], ci[r]);
            cd v = cmul(alpha, acc);
            if (beta != 0.0) {
                const cd c0 = Cin[e];
                v.x = fma(beta, c0.x, v.x);
                v.y = fma(beta, c0.y, v.y);
            }
            if (row == col) v.x += delta;
            Out[e] = v;
            nrm += cabs2(v);
        }
    }
    if (part) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if (lane == 0) sred[wave] = nrm;
        __syncthreads();
        if (t == 0)
            part[pb * bt.part + blockIdx.x + (int64_t)blockIdx.y * gridDim.x] =
                ((sred[0] + sred[1]) + sred[2]) + sred[3];
    }
}

// norm2[pb] = sum of the np partials (fixed order: lane q takes q, q + 64, ...,
// then a shuffle tree)
__global__ __launch_bounds__(64) void k_sum_partials(const double* __restrict__ part, int np,
                                                    double* __restrict__ norm2, Batch bt) {
    const int pb = bt.idx[blockIdx.x];
    part += pb * bt.part;
    double a = 0.0;
    for (int i = threadIdx.x; i < np; i += 64) a += part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (threadIdx.x == 0) norm2[pb * bt.scal] = a;
}

int64_t zgemm_part_len(int n) {
    const int64_t t = ceil_div(n, kMmT);
    return t * t;
}

void launch_zgemm_sq(int n, cd alpha, const cd* A, const cd* B, double beta, const cd* Cin,
                     double delta, cd* Out, double* part, double* norm2, hipStream_t st,
                     const Batch& bt) {
    if (bt.n <= 0 || n <= 0) return;
    if (Out == A || Out == B) throw HipError{hipErrorInvalidValue, "launch_zgemm_sq: Out aliases A or B"};
    if (beta != 0.0 && !Cin) throw HipError{hipErrorInvalidValue, "launch_zgemm_sq: beta without Cin"};
    const unsigned t = (unsigned)ceil_div(n, kMmT);
    hipLaunchKernelGGL(k_zgemm_mfma, dim3(t, t, bt.n), dim3(256), 0, st, n, alpha, A, B, beta,
                       Cin, delta, Out, part, bt);
    if (part && norm2)
        hipLaunchKernelGGL(k_sum_partials, dim3(bt.n), dim3(64), 0, st, (const double*)part,
                           (int)(t * t), norm2, bt);
    OSA_LAUNCH_CHECK();
}

// |s - [sprev; 0]|  (one block)
__global__ void k_diff_norm(const cd* __restrict__ s, int k, const cd* __restrict__ sp, int kp,
                            double* out, Batch bt) {
    __shared__ double sm[4];
    const int pb = bt.idx[blockIdx.x];
    s += pb * bt.small;
    sp += pb * bt.small;
    out += pb * bt.scal;
    double a = 0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        cd d = s[i];
        if (i < kp) d = csub(d, sp[i]);
        a += cabs2(d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) *out = sqrt(sm[0] + sm[1] + sm[2] + sm[3]);
}

void launch_diff_norm(const cd* s, int k, const cd* sprev, int kprev, double* out,
                      hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    hipLaunchKernelGGL(k_diff_norm, dim3(bt.n), dim3(256), 0, st, s, k, sprev, kprev, out, bt);
    OSA_LAUNCH_CHECK();
}

// ================================================================= Schur
// A = Z T Z^H for p <= 64: Householder reduction to Hessenberg form, complex
// single-shift QR with Wilkinson shifts (exceptional shifts every 10
// iterations without deflation), then reordering of the diagonal by adjacent
// swaps.  One wavefront; T and Z live in LDS.
// The Schur kernels below run as one 64-lane wavefront.  LDS operations of a
// wavefront execute in issue order, so lanes exchange data through LDS with a
// wavefront-scope fence and a wave barrier (ordering only for the compiler);
// a workgroup barrier would also wait for every outstanding LDS access.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static constexpr int kSchurMax = 64;

__device__ __forceinline__ double sort_key(cd v, int mode) {
    return mode == 0 ? cabsd(v) : fabs(v.x);
}

// Unitary Q with first column (a, b) = (f, g)/|(f, g)|, so Q^H [f; g] = [|(f, g)|; 0].
// The operands are first scaled by a power of two (exact) so that the sum of
// squares neither overflows nor underflows; the reciprocal square root is the
// hardware estimate refined by two Newton steps (error of a few ulp).
__device__ __forceinline__ void unit_pair(cd f, cd g, cd& a, cd& b) {
    const double m = fmax(fmax(fabs(f.x), fabs(f.y)), fmax(fabs(g.x), fabs(g.y)));
    if (m == 0.0) {
        a = mk(1.0, 0.0);
        b = mk(0.0, 0.0);
        return;
    }
    const int e = -__builtin_amdgcn_frexp_exp(m);
    f = mk(ldexp(f.x, e), ldexp(f.y, e));
    g = mk(ldexp(g.x, e), ldexp(g.y, e));
    const double s2 = cabs2(f) + cabs2(g);   // in [1/4, 4)
    double r = __builtin_amdgcn_rsq(s2);
    r = r * fma(-0.5 * s2, r * r, 1.5);
    r = r * fma(-0.5 * s2, r * r, 1.5);
    a = cscale(f, r);
    b = cscale(g, r);
}

// Value of v held by lane `src` (uniform), for every lane.
__device__ __forceinline__ double lane_value(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ cd lane_value(cd v, int src) {
    return mk(lane_value(v.x, src), lane_value(v.y, src));
}

// Similarity T <- Q^H T Q, Z <- Z Q by the 2x2 unitary Q (columns (a, b) and
// (-conj b, conj a)) on rows/columns (k, k+1), for p <= 64: lane l owns column
// l in the left update (columns >= col0) and row l in the right updates (T rows
// <= row1, all rows of Z), which share one pass over LDS.
// zero_col >= 0: the left update annihilates T[k+1, zero_col]; store an exact 0.
// Returns this lane's updated T[l, k] (meaningful for l <= row1).  WITH_Z =
// false leaves Z alone (another wavefront applies the rotation to it).
template <bool WITH_Z = true>
__device__ __forceinline__ cd rotate_pair64(cd* T, cd* Z, int p, int ld, int k, cd a, cd b,
                                            int col0, int row1, int zero_col) {
    const int l = threadIdx.x;
    if (l >= col0 && l < p) {
        const cd x = T[k + l * ld], y = T[k + 1 + l * ld];
        // Q^H [x; y] = [conj(a) x + conj(b) y ; -b x + a y]
        T[k + l * ld] = cadd(cmulc(a, x), cmulc(b, y));
        T[k + 1 + l * ld] = (l == zero_col) ? mk(0.0, 0.0) : csub(cmul(a, y), cmul(b, x));
    }
    wave_sync();
    cd tk = mk(0.0, 0.0);
    if (l < p) {
        // [x, y] Q = [a x + b y, -conj(b) x + conj(a) y]
        const cd x = T[l + k * ld], y = T[l + (k + 1) * ld];
        if (l <= row1) {
            tk = cadd(cmul(a, x), cmul(b, y));
            T[l + k * ld] = tk;
            T[l + (k + 1) * ld] = csub(cmulc(a, y), cmulc(b, x));
        }
        if (WITH_Z) {
            const cd zx = Z[l + k * ld], zy = Z[l + (k + 1) * ld];
            Z[l + k * ld] = cadd(cmul(a, zx), cmul(b, zy));
            Z[l + (k + 1) * ld] = csub(cmulc(a, zy), cmulc(b, zx));
        }
    }
    wave_sync();
    return tk;
}

static constexpr int kSchurWaves = 4;   // wavefronts of the Householder phase

__global__ __launch_bounds__(64 * kSchurWaves) void k_small_schur(const cd* __restrict__ A, int p,
                                                                 cd* Tout, cd* Zout, cd* wout,
                                                                 int mode, int* info) {
    // T and Z in LDS, column-major with the odd leading dimension ld = p + 1 so
    // that row sweeps (stride ld) and column sweeps (stride 1) are both free of
    // bank conflicts.
    extern __shared__ cd lds[];
    const int ld = p + 1;
    cd* T = lds;
    cd* Z = lds + (size_t)p * ld;
    __shared__ cd hv[kSchurMax];
    __shared__ cd pt[kSchurWaves][kSchurMax], pz[kSchurWaves][kSchurMax];
    __shared__ double sanorm[kSchurWaves];
    // rotations of one QR sweep, handed from the first wavefront (T) to the
    // second (Z), double buffered: (a, b) of rotation lo + i at 2i, 2i + 1
    __shared__ cd rlog[2][2 * kSchurMax];
    __shared__ int rsweep[2][2];   // lo, number of rotations
    __shared__ int qr_done;
    const int l = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) qr_done = 0;
#define TT(i, j) T[(i) + (j) * ld]
#define ZZ(i, j) Z[(i) + (j) * ld]
    // The QR iteration is run on B = A^H.  It tends to deflate the eigenvalues of
    // smallest modulus first, at the bottom, so B = Z_B T_B Z_B^H comes out with
    // the diagonal roughly descending.  Then A = W U W^H with W = Z_B J and
    // U = J T_B^H J (J reverses the index order): U is upper triangular and its
    // diagonal roughly ascending, which leaves the final reordering by adjacent
    // swaps (wanted values first) little to do.
    double amax = 0;
    for (int e = threadIdx.x; e < p * p; e += 64 * kSchurWaves) {
        const int i = e % p, j = e / p;
        const cd v = A[e];
        TT(j, i) = cconj(v);
        ZZ(i, j) = mk(i == j ? 1.0 : 0.0, 0.0);
        amax = fmax(amax, cabsd(v));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (l == 0) sanorm[wv] = amax;
    __syncthreads();
    const double anorm = fmax(fmax(sanorm[0], sanorm[1]), fmax(sanorm[2], sanorm[3]));
    // ---- Hessenberg reduction (Householder), four wavefronts: the reflector is
    // formed redundantly by each, the products v^H T[j+1:, c] and T[r, j+1:] v
    // are split over the wavefronts by ranges of the summation index and added
    // in wavefront order, and each wavefront updates its own range.
    for (int j = 0; j + 2 < p; ++j) {
        const int L = p - j - 1;
        double xp = 0;
        for (int i = l; i < L; i += 64) xp += cabs2(TT(j + 1 + i, j));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) xp += __shfl_xor(xp, off, 64);
        const double xn2 = xp;
        const double xn = sqrt(xn2);
        const cd x0 = TT(j + 1, j);
        const double tail = xn2 - cabs2(x0);
        if (xn == 0.0 || tail <= 1e-300) { __syncthreads(); continue; }
        const double ax0 = cabsd(x0);
        const cd ph = ax0 > 0 ? cscale(x0, 1.0 / ax0) : mk(1.0, 0.0);
        const cd alpha = cscale(ph, -xn);           // -e^{i arg x0} |x|
        // v = x - alpha e1, |v|^2 = |x|^2 - 2 Re(conj(alpha) x0) + |alpha|^2, tau = 2 / |v|^2
        if (wv == 0)
            for (int i = l; i < L; i += 64) hv[i] = (i == 0) ? csub(x0, alpha) : TT(j + 1 + i, j);
        const double vn2 = 2.0 * xn2 + 2.0 * xn * ax0;
        const double tau = 2.0 / vn2;
        // this wavefront's range of the summation index
        const int q = (L + kSchurWaves - 1) / kSchurWaves;
        const int i0 = wv * q, i1 = min(L, i0 + q);
        __syncthreads();
        // left: T[j+1:, c] -= tau v (v^H T[j+1:, c]),  c >= j   (one column per lane)
        const int c = j + l;
        if (c < p) {
            cd s0 = mk(0.0, 0.0);
#pragma unroll 4
            for (int i = i0; i < i1; ++i) cfmac(s0, hv[i], TT(j + 1 + i, c));
            pt[wv][l] = s0;
        }
        __syncthreads();
        if (c < p) {
            const cd sacc = cscale(cadd(cadd(pt[0][l], pt[1][l]), cadd(pt[2][l], pt[3][l])), tau);
#pragma unroll 4
            for (int i = i0; i < i1; ++i) TT(j + 1 + i, c) = csub(TT(j + 1 + i, c), cmul(hv[i], sacc));
        }
        __syncthreads();
        // right: T[r, j+1:] -= tau (T[r, j+1:] v) v^H, all rows; same for Z
        const int r = l;
        if (r < p) {
            cd s0 = mk(0.0, 0.0), z0 = mk(0.0, 0.0);
#pragma unroll 4
            for (int i = i0; i < i1; ++i) {
                cfma(s0, TT(r, j + 1 + i), hv[i]);
                cfma(z0, ZZ(r, j + 1 + i), hv[i]);
            }
            pt[wv][l] = s0;
            pz[wv][l] = z0;
        }
        __syncthreads();
        if (r < p) {
            const cd sacc = cscale(cadd(cadd(pt[0][l], pt[1][l]), cadd(pt[2][l], pt[3][l])), tau);
            const cd sz = cscale(cadd(cadd(pz[0][l], pz[1][l]), cadd(pz[2][l], pz[3][l])), tau);
#pragma unroll 4
            for (int i = i0; i < i1; ++i) {
                TT(r, j + 1 + i) = csub(TT(r, j + 1 + i), cmul(sacc, cconj(hv[i])));
                ZZ(r, j + 1 + i) = csub(ZZ(r, j + 1 + i), cmul(sz, cconj(hv[i])));
            }
        }
        __syncthreads();
        if (wv == 0)
            for (int i = l; i < L; i += 64) TT(j + 1 + i, j) = (i == 0) ? alpha : mk(0.0, 0.0);
        __syncthreads();
    }
    // The QR sweeps run on the first wavefront, which updates T and logs the
    // rotations of each sweep; the second applies a sweep's rotations to Z while
    // the first runs the next sweep.  One workgroup barrier per sweep hands a log
    // over (and waits for the previous one to be applied); a last one, after
    // qr_done is set, ends the second wavefront.  Everything after the QR
    // iteration runs on the first wavefront.
    if (wv >= 2) return;
    if (wv == 1) {
        for (int buf = 0;; buf ^= 1) {
            __syncthreads();
            if (qr_done) break;
            const int lo = rsweep[buf][0], n = rsweep[buf][1];
            if (l < p) {
                cd zx = ZZ(l, lo);
                for (int i = 0; i < n; ++i) {
                    const cd a = rlog[buf][2 * i], b = rlog[buf][2 * i + 1];
                    const cd zy = ZZ(l, lo + i + 1);
                    ZZ(l, lo + i) = cadd(cmul(a, zx), cmul(b, zy));
                    zx = csub(cmulc(a, zy), cmulc(b, zx));
                }
                ZZ(l, lo + n) = zx;
            }
        }
        return;
    }
    int buf = 0;
    // ---- shifted QR
    const double ulp = 2.220446049250313e-16;
    const double smlnum = 1e-300;
    int nrot = 0;
    int hi = p - 1;
    int its = 0, total = 0;
    const int maxtotal = 60 * p;
    bool fail = false;
    while (hi > 0) {
        // lo = largest l in [1, hi] with a negligible subdiagonal T[l, l-1], else 0;
        // lane l tests entry l, a ballot picks the highest one.
        bool neg = false;
        if (l >= 1 && l <= hi) {
            const double sub = cabsd(TT(l, l - 1));
            double tst = cabsd(TT(l - 1, l - 1)) + cabsd(TT(l, l));
            if (tst == 0.0) tst = anorm;
            neg = sub <= fmax(ulp * tst, smlnum);
        }
        const unsigned long long mask = __ballot(neg);
        const int lo = mask ? 63 - __clzll(mask) : 0;
        if (lo > 0) {
            wave_sync();
            if (l == 0) TT(lo, lo - 1) = mk(0.0, 0.0);
            wave_sync();
        }
        if (lo == hi) { --hi; its = 0; continue; }
        if (total++ > maxtotal) { fail = true; break; }
        ++its;
        // Wilkinson shift from the trailing 2x2 of the active block
        cd sigma;
        {
            const cd a = TT(hi - 1, hi - 1), b = TT(hi - 1, hi);
            const cd c = TT(hi, hi - 1), d = TT(hi, hi);
            if (its % 10 == 0) {
                sigma = cadd(d, mk(0.75 * cabsd(c), 0.0));   // exceptional shift
            } else {
                const cd tr2 = cscale(cadd(a, d), 0.5);
                const cd det = csub(cmul(a, d), cmul(b, c));
                const cd disc = csub(cmul(tr2, tr2), det);
                const double r = cabsd(disc);
                double sr = sqrt(0.5 * (r + disc.x));
                double si = sqrt(fmax(0.0, 0.5 * (r - disc.x)));
                if (disc.y < 0) si = -si;
                const cd sq = mk(sr, si);
                const cd e1 = cadd(tr2, sq), e2 = csub(tr2, sq);
                sigma = (cabsd(csub(e1, d)) <= cabsd(csub(e2, d))) ? e1 : e2;
            }
        }
        // bulge chase on the active block [lo, hi].  The pair (f, g) that fixes the
        // next rotation, T[k+1, k] and the bulge T[k+2, k], comes out of the right
        // update of rows k+1 and k+2 and is read from those lanes' registers.
        cd f = csub(TT(lo, lo), sigma), g = TT(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            cd a, b;
            unit_pair(f, g, a, b);
            const int col0 = (k == lo) ? lo : k - 1;
            const int row1 = (k + 2 < hi) ? k + 2 : hi;
            const cd tk =
                rotate_pair64<false>(T, Z, p, ld, k, a, b, col0, row1, (k > lo) ? k - 1 : -1);
            if (l == 0) {
                rlog[buf][2 * (k - lo)] = a;
                rlog[buf][2 * (k - lo) + 1] = b;
            }
            ++nrot;
            if (k + 1 < hi) {
                f = lane_value(tk, k + 1);
                g = lane_value(tk, k + 2);
            }
        }
        if (l == 0) {
            rsweep[buf][0] = lo;
            rsweep[buf][1] = hi - lo;
        }
        __syncthreads();   // hand the sweep to the Z wavefront
        buf ^= 1;
    }
    if (l == 0) qr_done = 1;
    __syncthreads();       // the Z wavefront has applied every sweep and leaves
    // ---- back to A: T <- J T^H J (pairs (i, j) <-> (p-1-j, p-1-i)), Z <- Z J
    if (!fail) {
        for (int e = l; e < p * p; e += 64) {
            const int i = e % p, j = e / p;
            const int i2 = p - 1 - j, j2 = p - 1 - i;
            const int e2 = i2 + j2 * p;
            if (e <= e2) {
                const cd u = TT(i, j), v = TT(i2, j2);
                TT(i, j) = cconj(v);
                TT(i2, j2) = cconj(u);
            }
        }
        for (int i = l; i < p; i += 64) {
            for (int j = 0; j < p / 2; ++j) {
                const cd u = ZZ(i, j), v = ZZ(i, p - 1 - j);
                ZZ(i, j) = v;
                ZZ(i, p - 1 - j) = u;
            }
        }
        wave_sync();
    }
    // ---- reorder the diagonal (insertion sort by adjacent swaps)
    for (int i = 1; i < p && !fail; ++i) {
        for (int j = i; j > 0; --j) {
            const cd t11 = TT(j - 1, j - 1), t22 = TT(j, j);
            if (!(sort_key(t22, mode) < sort_key(t11, mode))) break;
            const cd t12 = TT(j - 1, j);
            const cd x1 = t12, x2 = csub(t22, t11);
            if (x1.x == 0.0 && x1.y == 0.0 && x2.x == 0.0 && x2.y == 0.0) break;
            cd a, b;
            unit_pair(x1, x2, a, b);
            rotate_pair64(T, Z, p, ld, j - 1, a, b, j - 1, j, -1);
            ++nrot;
            if (l == 0) {
                TT(j, j - 1) = mk(0.0, 0.0);   // touched by both sides: set after them
                TT(j - 1, j - 1) = t22;
                TT(j, j) = t11;
            }
            wave_sync();
        }
    }
    for (int e = l; e < p * p; e += 64) {
        const int i = e % p, j = e / p;
        Tout[e] = TT(i, j);
        Zout[e] = ZZ(i, j);
    }
    for (int i = l; i < p; i += 64) wout[i] = TT(i, i);
    if (l == 0) {
        info[0] = fail ? -1 : total;
        info[1] = nrot;
    }
#undef TT
#undef ZZ
}

// ---------------------------------------------------------------------------
// Larger Schur problems (64 < p <= 96).  Only T fits in LDS, so kernel A keeps T
// there and writes every transformation applied from the right to a log: the
// Householder vectors of the Hessenberg reduction and the 2x2 unitaries of the
// QR sweeps and of the reordering.  Kernel B rebuilds Z = product of the logged
// transformations, one thread per row of Z (rows staged in LDS), applying the
// log in order.  A runs as a single wavefront (two elements per lane for
// p > 64): a two-wavefront version gave run-to-run different Schur forms for
// identical input, while this one is bitwise reproducible.
static constexpr int kSchurBig = 96;
static constexpr int kBigThreads = 64;

struct RotEntry {   // columns (k, k+1) <- [a x + b y, -conj(b) x + conj(a) y]
    cd a, b;
    int k, pad;
};

__global__ __launch_bounds__(kBigThreads) void k_schur_log(const cd* __restrict__ A, int p,
                                                           cd* Tout, cd* wout, int mode, int* info,
                                                           cd* hlog, double* tlog,
                                                           RotEntry* rlog, int rcap) {
    extern __shared__ cd lds[];
    const int ld = p + 1;
    cd* T = lds;
    __shared__ cd hv[kSchurBig];
    __shared__ double sred[kBigThreads / 64];
    __shared__ unsigned long long sball[kBigThreads / 64];
    const int l = threadIdx.x;
    const int lane = l & 63, wave = l >> 6;
#define TT(i, j) T[(i) + (j) * ld]
    double amax = 0;
    for (int e = l; e < p * p; e += kBigThreads) {
        const cd v = A[e];
        TT(e % p, e / p) = v;
        amax = fmax(amax, cabsd(v));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) sred[wave] = amax;
    wave_sync();
    const double anorm = sred[0];
    wave_sync();
    // ---- Hessenberg reduction; reflectors logged for Z
    for (int j = 0; j + 2 < p; ++j) {
        const int L = p - j - 1;
        double xp = 0;
        for (int i = l; i < L; i += kBigThreads) xp += cabs2(TT(j + 1 + i, j));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) xp += __shfl_xor(xp, off, 64);
        if (lane == 0) sred[wave] = xp;
        wave_sync();
        const double xn2 = sred[0];
        const double xn = sqrt(xn2);
        const cd x0 = TT(j + 1, j);
        const double tail = xn2 - cabs2(x0);
        wave_sync();
        if (xn == 0.0 || tail <= 1e-300) {
            if (l == 0) tlog[j] = 0.0;
            continue;
        }
        const double ax0 = cabsd(x0);
        const cd ph = ax0 > 0 ? cscale(x0, 1.0 / ax0) : mk(1.0, 0.0);
        const cd alpha = cscale(ph, -xn);
        for (int i = l; i < L; i += kBigThreads) {
            const cd v = (i == 0) ? csub(x0, alpha) : TT(j + 1 + i, j);
            hv[i] = v;
            hlog[(size_t)j * p + i] = v;
        }
        const double tau = 2.0 / (2.0 * xn2 + 2.0 * xn * ax0);
        if (l == 0) tlog[j] = tau;
        wave_sync();
        for (int c = j + l; c < p; c += kBigThreads) {
            cd sacc = mk(0.0, 0.0);
            for (int i = 0; i < L; ++i) cfmac(sacc, hv[i], TT(j + 1 + i, c));
            sacc = cscale(sacc, tau);
            for (int i = 0; i < L; ++i) TT(j + 1 + i, c) = csub(TT(j + 1 + i, c), cmul(hv[i], sacc));
        }
        wave_sync();
        for (int r = l; r < p; r += kBigThreads) {
            cd sacc = mk(0.0, 0.0);
            for (int i = 0; i < L; ++i) cfma(sacc, TT(r, j + 1 + i), hv[i]);
            sacc = cscale(sacc, tau);
            for (int i = 0; i < L; ++i) TT(r, j + 1 + i) = csub(TT(r, j + 1 + i), cmul(sacc, cconj(hv[i])));
        }
        wave_sync();
        for (int i = l; i < L; i += kBigThreads) TT(j + 1 + i, j) = (i == 0) ? alpha : mk(0.0, 0.0);
        wave_sync();
    }
    int nrot = 0;
    bool overflow = false;
    auto pair = [&](int k, cd a, cd b, int col0, int row1, int zero_col) {
        for (int c = col0 + l; c < p; c += kBigThreads) {
            const cd x = TT(k, c), y = TT(k + 1, c);
            TT(k, c) = cadd(cmulc(a, x), cmulc(b, y));
            TT(k + 1, c) = (c == zero_col) ? mk(0.0, 0.0) : csub(cmul(a, y), cmul(b, x));
        }
        wave_sync();
        for (int r = l; r <= row1 && r < p; r += kBigThreads) {
            const cd x = TT(r, k), y = TT(r, k + 1);
            TT(r, k) = cadd(cmul(a, x), cmul(b, y));
            TT(r, k + 1) = csub(cmulc(a, y), cmulc(b, x));
        }
        if (l == 0) {
            if (nrot < rcap) rlog[nrot] = RotEntry{a, b, k, 0};
        }
        if (nrot >= rcap) overflow = true;
        ++nrot;
        wave_sync();
    };
    // ---- shifted QR
    const double ulp = 2.220446049250313e-16;
    const double smlnum = 1e-300;
    int hi = p - 1;
    int its = 0, total = 0;
    const int maxtotal = 60 * p;
    bool fail = false;
    while (hi > 0) {
        auto negl = [&](int q) -> bool {
            if (q < 1 || q > hi) return false;
            const double sub = cabsd(TT(q, q - 1));
            double tst = cabsd(TT(q - 1, q - 1)) + cabsd(TT(q, q));
            if (tst == 0.0) tst = anorm;
            return sub <= fmax(ulp * tst, smlnum);
        };
        const unsigned long long m0 = __ballot(negl(l));
        const unsigned long long m1 = __ballot(negl(l + 64));
        int lo = 0;
        if (m1) lo = 64 + 63 - __clzll(m1);
        else if (m0) lo = 63 - __clzll(m0);
        wave_sync();
        if (lo > 0) {
            if (l == 0) TT(lo, lo - 1) = mk(0.0, 0.0);
            wave_sync();
        }
        if (lo == hi) { --hi; its = 0; continue; }
        if (total++ > maxtotal) { fail = true; break; }
        ++its;
        cd sigma;
        {
            const cd a = TT(hi - 1, hi - 1), b = TT(hi - 1, hi);
            const cd c = TT(hi, hi - 1), d = TT(hi, hi);
            if (its % 10 == 0) {
                sigma = cadd(d, mk(0.75 * cabsd(c), 0.0));
            } else {
                const cd tr2 = cscale(cadd(a, d), 0.5);
                const cd det = csub(cmul(a, d), cmul(b, c));
                const cd disc = csub(cmul(tr2, tr2), det);
                const double r = cabsd(disc);
                double sr = sqrt(0.5 * (r + disc.x));
                double si = sqrt(fmax(0.0, 0.5 * (r - disc.x)));
                if (disc.y < 0) si = -si;
                const cd sq = mk(sr, si);
                const cd e1 = cadd(tr2, sq), e2 = csub(tr2, sq);
                sigma = (cabsd(csub(e1, d)) <= cabsd(csub(e2, d))) ? e1 : e2;
            }
        }
        for (int k = lo; k < hi; ++k) {
            cd f, g;
            if (k == lo) { f = csub(TT(lo, lo), sigma); g = TT(lo + 1, lo); }
            else { f = TT(k, k - 1); g = TT(k + 1, k - 1); }
            const double nf = sqrt(cabs2(f) + cabs2(g));
            cd a, b;
            if (nf == 0.0) { a = mk(1.0, 0.0); b = mk(0.0, 0.0); }
            else { const double inf = 1.0 / nf; a = cscale(f, inf); b = cscale(g, inf); }
            const int col0 = (k == lo) ? lo : k - 1;
            const int row1 = (k + 2 < hi) ? k + 2 : hi;
            pair(k, a, b, col0, row1, (k > lo) ? k - 1 : -1);
        }
    }
    // ---- reorder the diagonal
    for (int i = 1; i < p && !fail; ++i) {
        for (int j = i; j > 0; --j) {
            const cd t11 = TT(j - 1, j - 1), t22 = TT(j, j);
            if (!(sort_key(t22, mode) < sort_key(t11, mode))) break;
            const cd t12 = TT(j - 1, j);
            const cd x1 = t12, x2 = csub(t22, t11);
            const double nx = sqrt(cabs2(x1) + cabs2(x2));
            if (nx == 0.0) break;
            const cd a = cscale(x1, 1.0 / nx), b = cscale(x2, 1.0 / nx);
            pair(j - 1, a, b, j - 1, j, -1);
            if (l == 0) {
                TT(j, j - 1) = mk(0.0, 0.0);
                TT(j - 1, j - 1) = t22;
                TT(j, j) = t11;
            }
            wave_sync();
        }
    }
    for (int e = l; e < p * p; e += kBigThreads) Tout[e] = TT(e % p, e / p);
    for (int i = l; i < p; i += kBigThreads) wout[i] = TT(i, i);
    if (l == 0) {
        info[0] = (fail || overflow) ? -1 : total;
        info[1] = nrot < rcap ? nrot : rcap;
    }
#undef TT
}

// Z = (I - tau_0 v_0 v_0^H)(I - tau_1 v_1 v_1^H) ... G_1 G_2 ..., row by row.
__global__ __launch_bounds__(64) void k_schur_build_z(int p, const cd* __restrict__ hlog,
                                                      const double* __restrict__ tlog,
                                                      const RotEntry* __restrict__ rlog,
                                                      const int* __restrict__ info, cd* Zout) {
    extern __shared__ cd zs[];                   // zs[c*64 + lane]: row (blockIdx*64 + lane)
    __shared__ RotEntry chunk[128];
    __shared__ cd vsh[kSchurBig];
    const int lane = threadIdx.x;
    const int r = blockIdx.x * 64 + lane;
    const bool live = r < p;
    for (int c = 0; c < p; ++c) zs[c * 64 + lane] = mk((live && c == r) ? 1.0 : 0.0, 0.0);
    for (int j = 0; j + 2 < p; ++j) {
        const double tau = tlog[j];
        if (tau == 0.0) continue;
        const int L = p - j - 1;
        wave_sync();
        for (int i = lane; i < L; i += 64) vsh[i] = hlog[(size_t)j * p + i];   // stage v_j
        wave_sync();
        cd s = mk(0.0, 0.0);
        for (int i = 0; i < L; ++i) cfma(s, zs[(j + 1 + i) * 64 + lane], vsh[i]);
        s = cscale(s, tau);
        for (int i = 0; i < L; ++i) {
            cd& z = zs[(j + 1 + i) * 64 + lane];
            z = csub(z, cmul(s, cconj(vsh[i])));
        }
    }
    const int nrot = info[1];
    for (int base = 0; base < nrot; base += 128) {
        const int cnt = (nrot - base < 128) ? nrot - base : 128;
        wave_sync();
        for (int e = lane; e < cnt; e += 64) chunk[e] = rlog[base + e];
        wave_sync();
        for (int e = 0; e < cnt; ++e) {
            const RotEntry q = chunk[e];
            cd& zx = zs[q.k * 64 + lane];
            cd& zy = zs[(q.k + 1) * 64 + lane];
            const cd x = zx, y = zy;
            zx = cadd(cmul(q.a, x), cmul(q.b, y));
            zy = csub(cmulc(q.a, y), cmulc(q.b, x));
        }
    }
    if (live)
        for (int c = 0; c < p; ++c) Zout[r + (size_t)c * p] = zs[c * 64 + lane];
}

size_t schur_ws_bytes(int p) {
    const size_t rcap = (size_t)60 * p * p + (size_t)p * p;
    return (size_t)p * p * sizeof(cd) + (size_t)p * sizeof(double) + rcap * sizeof(RotEntry) + 512;
}

static void small_schur_big(const cd* A, int p, cd* T, cd* Z, cd* w, int mode, int* info, void* ws,
                            hipStream_t st) {
    char* q = (char*)ws;
    cd* hlog = (cd*)q;               q += (size_t)p * p * sizeof(cd);
    double* tlog = (double*)q;       q += (size_t)p * sizeof(double);
    q = (char*)(((uintptr_t)q + 63) & ~(uintptr_t)63);
    RotEntry* rlog = (RotEntry*)q;
    const int rcap = 60 * p * p + p * p;
    static const bool attr = [] {
        OSA_HIP(hipFuncSetAttribute((const void*)k_schur_log,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kSchurBig * (kSchurBig + 1) * sizeof(cd))));
        OSA_HIP(hipFuncSetAttribute((const void*)k_schur_build_z,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kSchurBig * 64 * sizeof(cd))));
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(k_schur_log, dim3(1), dim3(kBigThreads), (size_t)p * (p + 1) * sizeof(cd), st,
                       A, p, T, w, mode, info, hlog, tlog, rlog, rcap);
    hipLaunchKernelGGL(k_schur_build_z, dim3((unsigned)ceil_div(p, 64)), dim3(64),
                       (size_t)p * 64 * sizeof(cd), st, p, (const cd*)hlog, (const double*)tlog,
                       (const RotEntry*)rlog, (const int*)info, Z);
    OSA_LAUNCH_CHECK();
}


void small_schur(const cd* A, int p, cd* T, cd* Z, cd* w, int mode, int* info, void* ws,
                 hipStream_t st) {
    if (p > kSchurMax) {
        if (p > kSchurBig || !ws) throw HipError{hipErrorInvalidValue, "small_schur: p out of range"};
        small_schur_big(A, p, T, Z, w, mode, info, ws, st);
        return;
    }
    if (p < 1) throw HipError{hipErrorInvalidValue, "small_schur: p out of range"};
    const size_t lds = (size_t)2 * p * (p + 1) * sizeof(cd);
    static const bool attr_set = [] {   // thread-safe one-time initialisation
        OSA_HIP(hipFuncSetAttribute((const void*)k_small_schur,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(2 * kSchurMax * (kSchurMax + 1) * sizeof(cd))));
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL(k_small_schur, dim3(1), dim3(64 * kSchurWaves), lds, st, A, p, T, Z, w, mode,
                       info);
    OSA_LAUNCH_CHECK();
}

// Eigenvectors from the Schur form: back substitution on T for each diagonal
// entry, then multiplication by Z; columns normalised to unit length.
__global__ __launch_bounds__(64) void k_small_eigvecs(const cd* __restrict__ T,
                                                     const cd* __restrict__ Z, int p, cd* Y) {
    extern __shared__ cd y[];   // p x p, column i = eigenvector of T for t_ii
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= p) return;
    // thread-private columns interleaved (stride 64) so that equal indices of
    // different threads fall in different banks
    cd* yi = y + threadIdx.x;
#define YI(r) yi[(size_t)(r) * 64]
    const cd lam = T[i + (size_t)i * p];
    double tnorm = 0;
    for (int e = 0; e < p * p; ++e) tnorm = fmax(tnorm, cabsd(T[e]));
    const double small = fmax(tnorm * 2.220446049250313e-16, 1e-300);
    for (int r = 0; r < p; ++r) YI(r) = mk(0.0, 0.0);
    YI(i) = mk(1.0, 0.0);
    for (int r = i - 1; r >= 0; --r) {
        cd s = mk(0.0, 0.0);
        for (int q = r + 1; q <= i; ++q) cfma(s, T[r + (size_t)q * p], YI(q));
        cd d = csub(T[r + (size_t)r * p], lam);
        if (cabsd(d) < small) d = mk(small, 0.0);
        YI(r) = cscale(cdiv(s, d), -1.0);
    }
    double n2 = 0;
    for (int r = 0; r < p; ++r) {
        cd s = mk(0.0, 0.0);
        for (int q = 0; q <= i; ++q) cfma(s, Z[r + (size_t)q * p], YI(q));
        Y[r + (size_t)i * p] = s;
        n2 += cabs2(s);
    }
    const double inv = 1.0 / sqrt(n2);
    for (int r = 0; r < p; ++r) Y[r + (size_t)i * p] = cscale(Y[r + (size_t)i * p], inv);
#undef YI
}

void small_eigvecs(const cd* T, const cd* Z, int p, cd* Y, hipStream_t st) {
    const size_t lds = (size_t)64 * p * sizeof(cd);
    static const bool attr_set = [] {
        OSA_HIP(hipFuncSetAttribute((const void*)k_small_eigvecs,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(64 * kSchurMax * sizeof(cd))));
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL(k_small_eigvecs, dim3((unsigned)ceil_div(p, 64)), dim3(64), lds, st, T, Z, p,
                       Y);
    OSA_LAUNCH_CHECK();
}

}  // namespace osa
