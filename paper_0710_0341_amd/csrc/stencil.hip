// Layout conversion and the Wilson-Dirac stencil at chemical potential.
//
// H_w(mu) psi = gamma_5 [ psi_n - kappa sum_nu ( e^{+mu d_{nu4}} (1+gamma_nu) U_{n,nu} psi_{n+nu}
//                                            + e^{-mu d_{nu4}} (1-gamma_nu) U^dag_{n-nu,nu} psi_{n-nu} ) ]
// (Eq. 1 and Eq. 2).  (1 +- gamma_nu) has rank two, so each hop projects the
// neighbour spinor onto a half spinor h (2 spins x 3 colours), multiplies the
// two colour vectors by the link and rebuilds the lower spin pair from h.  In
// the chiral basis (gamma_5 = diag(1,1,-1,-1)) with psi = (u0, u1, d0, d1):
//
//   nu = x : h = (u0 - s i d1, u1 - s i d0),   lower = ( s i h1,  s i h0)
//   nu = y : h = (u0 - s d1,   u1 + s d0),     lower = ( s h1,   -s h0)
//   nu = z : h = (u0 - s i d0, u1 + s i d1),   lower = ( s i h0, -s i h1)
//   nu = t : h = (u0 + s d0,   u1 + s d1),     lower = ( s h0,    s h1)
//
// with s = +1 for the forward hop (1+gamma) and s = -1 for the backward hop.
// gamma_5 then flips the sign of the lower spin pair of the result.
#include "kernels.hpp"

namespace osa {

// ------------------------------------------------------------------ layout
template <typename TI, typename TO>
__global__ void k_links_to_internal(const TI* __restrict__ in, TO* __restrict__ out, int V,
                                    int Vp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over Vp*36
    if (idx >= (int64_t)Vp * 36) return;
    int s = (int)(idx % Vp);
    int e = (int)(idx / Vp);            // e = (nu*3 + a)*3 + b
    TO val;
    if (s < V) {
        cd v = tod(in[(int64_t)s * 36 + e]);
        val = fromd<TO>(v);
    } else {
        val = fromd<TO>(mk(0.0, 0.0));
    }
    out[(int64_t)e * Vp + s] = val;
}

void launch_links_to_internal(const void* links_aos, bool in_fp32, void* links_int,
                              bool int_fp32, const Geom& g, hipStream_t st) {
    int64_t n = (int64_t)g.Vp * 36;
    dim3 grid((unsigned)ceil_div(n, 256)), blk(256);
    if (!in_fp32 && !int_fp32)
        hipLaunchKernelGGL((k_links_to_internal<cd, cd>), grid, blk, 0, st, (const cd*)links_aos,
                           (cd*)links_int, g.V, g.Vp);
    else if (in_fp32 && int_fp32)
        hipLaunchKernelGGL((k_links_to_internal<cf, cf>), grid, blk, 0, st, (const cf*)links_aos,
                           (cf*)links_int, g.V, g.Vp);
    else if (!in_fp32 && int_fp32)
        hipLaunchKernelGGL((k_links_to_internal<cd, cf>), grid, blk, 0, st, (const cd*)links_aos,
                           (cf*)links_int, g.V, g.Vp);
    else
        hipLaunchKernelGGL((k_links_to_internal<cf, cd>), grid, blk, 0, st, (const cf*)links_aos,
                           (cd*)links_int, g.V, g.Vp);
    OSA_LAUNCH_CHECK();
}

template <typename TO>
__global__ void k_vec_to_internal(const cd* __restrict__ in, TO* __restrict__ out, int V, int Vp,
                                  int nvec) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over nvec*12*Vp
    int64_t per = 12LL * Vp;
    if (idx >= per * nvec) return;
    int vec = (int)(idx / per);
    int64_t r = idx - vec * per;
    int c = (int)(r / Vp);
    int s = (int)(r - (int64_t)c * Vp);
    cd v = (s < V) ? in[(int64_t)vec * 12 * V + (int64_t)s * 12 + c] : mk(0.0, 0.0);
    out[idx] = fromd<TO>(v);
}

template <typename TI>
__global__ void k_vec_from_internal(const TI* __restrict__ in, cd* __restrict__ out, int V, int Vp,
                                    int nvec) {
    // one thread per boundary-layout entry so that the writes are coalesced
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over nvec*12*V
    int64_t per = 12LL * V;
    if (idx >= per * nvec) return;
    int vec = (int)(idx / per);
    int64_t r = idx - vec * per;
    int s = (int)(r / 12);
    int c = (int)(r - (int64_t)s * 12);
    out[idx] = tod(in[(int64_t)vec * 12 * Vp + (int64_t)c * Vp + s]);
}

void launch_vec_to_internal(const cd* aos, void* soa, bool soa_fp32, const Geom& g, int nvec,
                            hipStream_t st) {
    int64_t n = 12LL * g.Vp * nvec;
    dim3 grid((unsigned)ceil_div(n, 256)), blk(256);
    if (soa_fp32)
        hipLaunchKernelGGL(k_vec_to_internal<cf>, grid, blk, 0, st, aos, (cf*)soa, g.V, g.Vp, nvec);
    else
        hipLaunchKernelGGL(k_vec_to_internal<cd>, grid, blk, 0, st, aos, (cd*)soa, g.V, g.Vp, nvec);
    OSA_LAUNCH_CHECK();
}

void launch_vec_from_internal(const void* soa, bool soa_fp32, cd* aos, const Geom& g, int nvec,
                              hipStream_t st) {
    int64_t n = 12LL * g.V * nvec;
    dim3 grid((unsigned)ceil_div(n, 256)), blk(256);
    if (soa_fp32)
        hipLaunchKernelGGL(k_vec_from_internal<cf>, grid, blk, 0, st, (const cf*)soa, aos, g.V,
                           g.Vp, nvec);
    else
        hipLaunchKernelGGL(k_vec_from_internal<cd>, grid, blk, 0, st, (const cd*)soa, aos, g.V,
                           g.Vp, nvec);
    OSA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ stencil
// Complex arithmetic in the compute precision R (double or float).
template <typename R> struct Cx { R x, y; };
template <typename R> __device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.x, s * a.y}; }
// i * a
template <typename R> __device__ __forceinline__ Cx<R> ti(Cx<R> a) { return {-a.y, a.x}; }

template <typename R, typename T> __device__ __forceinline__ Cx<R> ld(const T* p) {
    T v = *p;
    return Cx<R>{(R)v.x, (R)v.y};
}

// w = U h  (fwd) or w = U^dag h (bwd) for a colour 3-vector; U read from SoA links.
template <typename R, bool DAG, typename LT>
__device__ __forceinline__ void su3_mul(const LT* __restrict__ U, int64_t base, int64_t Vp,
                                        const Cx<R> h[3], Cx<R> w[3]) {
    Cx<R> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ld<R>(U + base + e * Vp);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R re = 0, im = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Cx<R> m = DAG ? Cx<R>{u[b * 3 + a].x, -u[b * 3 + a].y} : u[a * 3 + b];
            re += m.x * h[b].x - m.y * h[b].y;
            im += m.x * h[b].y + m.y * h[b].x;
        }
        w[a] = Cx<R>{re, im};
    }
}

// One hop: project the neighbour spinor (NU, sign S), multiply by the link and
// accumulate coef * (reconstructed 4-spinor) into acc[12].
template <typename R, int NU, int S, typename ST, typename LT>
__device__ __forceinline__ void hop(const ST* __restrict__ in, const LT* __restrict__ U,
                                    int64_t Vp, int nb, int lsite, R coef, Cx<R> acc[12]) {
    Cx<R> u0[3], u1[3], d0[3], d1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u0[c] = ld<R>(in + (0 * 3 + c) * Vp + nb);
        u1[c] = ld<R>(in + (1 * 3 + c) * Vp + nb);
        d0[c] = ld<R>(in + (2 * 3 + c) * Vp + nb);
        d1[c] = ld<R>(in + (3 * 3 + c) * Vp + nb);
    }
    const R s = (R)S;
    Cx<R> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (NU == 0) { h0[c] = u0[c] - s * ti(d1[c]); h1[c] = u1[c] - s * ti(d0[c]); }
        if (NU == 1) { h0[c] = u0[c] - s * d1[c];     h1[c] = u1[c] + s * d0[c]; }
        if (NU == 2) { h0[c] = u0[c] - s * ti(d0[c]); h1[c] = u1[c] + s * ti(d1[c]); }
        if (NU == 3) { h0[c] = u0[c] + s * d0[c];     h1[c] = u1[c] + s * d1[c]; }
    }
    Cx<R> w0[3], w1[3];
    const int64_t base = (int64_t)(NU * 9) * Vp + lsite;
    su3_mul<R, (S < 0)>(U, base, Vp, h0, w0);
    su3_mul<R, (S < 0)>(U, base, Vp, h1, w1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Cx<R> l0, l1;
        if (NU == 0) { l0 = s * ti(w1[c]); l1 = s * ti(w0[c]); }
        if (NU == 1) { l0 = s * w1[c];     l1 = (-s) * w0[c]; }
        if (NU == 2) { l0 = s * ti(w0[c]); l1 = (-s) * ti(w1[c]); }
        if (NU == 3) { l0 = s * w0[c];     l1 = s * w1[c]; }
        acc[0 * 3 + c] = acc[0 * 3 + c] + coef * w0[c];
        acc[1 * 3 + c] = acc[1 * 3 + c] + coef * w1[c];
        acc[2 * 3 + c] = acc[2 * 3 + c] + coef * l0;
        acc[3 * 3 + c] = acc[3 * 3 + c] + coef * l1;
    }
}

struct StencilArgs {
    int lx, ly, lz, lt, V;
    int64_t Vp;
    int apt;
    double cf[4], cb[4];
    // work order (see block_work): total = site blocks x problems, per_xcd =
    // ceil(total / 8); bps > 0: site blocks per time slice (time slices in pairs)
    int total, per_xcd, bps;
};

static constexpr int kStGroup = 4;   // problems sharing one pass over a pair of slices

// Which (site block, problem) a workgroup takes.  Workgroups go to the eight
// XCDs of the chip round-robin (workgroup b to XCD b % 8), and each XCD has its
// own L2.  Giving XCD x the contiguous stretch [x per_xcd, (x+1) per_xcd) of
// the work order keeps a neighbourhood of the lattice in one L2.  The order runs
// over pairs of time slices; within a pair, over groups of up to four
// problems, and within a group over the site blocks of a slice, then the two
// slices, then the problems of the group: the time neighbour inside a pair, the
// z and y neighbours and the links (shared by a group) are all read a few
// dozen workgroups apart, so they come from that XCD's L2 rather than HBM.
// Without whole 64-site blocks per slice (bps = 0) the order is site block
// major, problem minor.  Returns false for the padding workgroups.
__device__ __forceinline__ bool block_work(const StencilArgs& a, int nprob, int& sb, int& entry) {
    const int b = (int)blockIdx.x;
    const int L = (b & 7) * a.per_xcd + (b >> 3);
    if (L >= a.total) return false;
    if (a.bps > 0) {
        // problems in groups of kStGroup: within a pair of slices, group by group
        const int per_pair = a.bps * 2 * nprob;
        const int tp = L / per_pair;
        int r = L - tp * per_pair;
        const int g0 = (r / (a.bps * 2 * kStGroup)) * kStGroup;
        const int gn = (nprob - g0 < kStGroup) ? nprob - g0 : kStGroup;
        r -= g0 * a.bps * 2;
        const int q = r / (2 * gn);
        const int r2 = r - q * 2 * gn;
        const int dt = r2 / gn;
        entry = g0 + (r2 - dt * gn);
        sb = (2 * tp + dt) * a.bps + q;
    } else {
        entry = L % nprob;
        sb = L / nprob;
    }
    return true;
}

// One block: 64 sites of one problem and two wavefronts, each with both hops of
// two directions (x and y; z and t), so the direction is uniform in a wave.  The
// two partial sums meet in LDS (24 KB per block at FP64, so six blocks fit a
// compute unit), where each wave adds the diagonal term and gamma_5 for six of
// the twelve components.  Small lattices still fill the GPU (two waves per 64
// sites), large ones keep coalesced, site-contiguous accesses.
template <typename R, typename ST, typename LT>
__global__ __launch_bounds__(128) void k_wilson_h(const ST* __restrict__ in, ST* __restrict__ out,
                                                 const LT* __restrict__ U, StencilArgs a,
                                                 Batch bt) {
    __shared__ Cx<R> part[2][12][64];
    int sb = 0, entry = 0;
    if (!block_work(a, bt.n, sb, entry)) return;   // uniform over the block
    const int pb = bt.idx[entry];
    in += pb * bt.basis;
    out += pb * bt.vec;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // 0: x, y; 1: z, t
    const int s = sb * 64 + lane;
    const int64_t Vp = a.Vp;
    Cx<R> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = Cx<R>{0, 0};
    if (s < a.V) {
        const int x = s % a.lx;
        int r = s / a.lx;
        const int y = r % a.ly;
        r /= a.ly;
        const int z = r % a.lz;
        const int t = r / a.lz;
        if (w == 0) {
            const int fx = (x + 1 == a.lx) ? s - (a.lx - 1) : s + 1;
            const int bx = (x == 0) ? s + (a.lx - 1) : s - 1;
            hop<R, 0, +1>(in, U, Vp, fx, s, (R)a.cf[0], acc);
            hop<R, 0, -1>(in, U, Vp, bx, bx, (R)a.cb[0], acc);
            const int sy = a.lx;
            const int fy = (y + 1 == a.ly) ? s - (a.ly - 1) * sy : s + sy;
            const int by = (y == 0) ? s + (a.ly - 1) * sy : s - sy;
            hop<R, 1, +1>(in, U, Vp, fy, s, (R)a.cf[1], acc);
            hop<R, 1, -1>(in, U, Vp, by, by, (R)a.cb[1], acc);
        } else {
            const int sz = a.lx * a.ly;
            const int fz = (z + 1 == a.lz) ? s - (a.lz - 1) * sz : s + sz;
            const int bz = (z == 0) ? s + (a.lz - 1) * sz : s - sz;
            hop<R, 2, +1>(in, U, Vp, fz, s, (R)a.cf[2], acc);
            hop<R, 2, -1>(in, U, Vp, bz, bz, (R)a.cb[2], acc);
            const int stt = a.lx * a.ly * a.lz;
            const int ft = (t + 1 == a.lt) ? s - (a.lt - 1) * stt : s + stt;
            const int bt_ = (t == 0) ? s + (a.lt - 1) * stt : s - stt;
            R ctf = (R)a.cf[3], ctb = (R)a.cb[3];
            if (a.apt) {
                if (t + 1 == a.lt) ctf = -ctf;
                if (t == 0) ctb = -ctb;
            }
            hop<R, 3, +1>(in, U, Vp, ft, s, ctf, acc);
            hop<R, 3, -1>(in, U, Vp, bt_, bt_, ctb, acc);
        }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) part[w][c][lane] = acc[c];
    __syncthreads();
    if (s < a.Vp) {
        // padding sites carry zeros so that whole-vector reductions stay exact
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const int c = 6 * w + i;
            ST o;
            o.x = 0;
            o.y = 0;
            if (s < a.V) {
                Cx<R> v = ld<R>(in + (int64_t)c * Vp + s) + part[0][c][lane] + part[1][c][lane];
                if (c >= 6) v = Cx<R>{-v.x, -v.y};    // gamma_5
                o.x = v.x;
                o.y = v.y;
            }
            out[(int64_t)c * Vp + s] = o;
        }
    }
}

void launch_wilson_h(const void* in, void* out, const void* U, bool links_fp32, bool spinor_fp32,
                     const Geom& g, const HopCoef& c, hipStream_t st, const Batch& bt) {
    if (bt.n <= 0) return;
    // a block covers 64 sites and writes all of them
    if (g.Vp % 64 != 0) throw HipError{hipErrorInvalidValue, "launch_wilson_h: Vp % 64 != 0"};
    StencilArgs a;
    a.lx = g.lx; a.ly = g.ly; a.lz = g.lz; a.lt = g.lt; a.V = g.V; a.Vp = g.Vp; a.apt = g.apt;
    for (int i = 0; i < 4; ++i) { a.cf[i] = c.fwd[i]; a.cb[i] = c.bwd[i]; }
    // the work covers Vp sites (padding included; Vp is a multiple of 64) for each problem
    const int64_t nsb = ceil_div(g.Vp, 64);
    const int64_t total = nsb * bt.n;
    a.total = (int)total;
    a.per_xcd = (int)ceil_div(total, 8);
    const int64_t P = (int64_t)g.lx * g.ly * g.lz;
    a.bps = (P % 64 == 0 && g.lt % 2 == 0 && (int64_t)g.V == g.Vp) ? (int)(P / 64) : 0;
    dim3 blk(128), grid((unsigned)(8 * a.per_xcd));
    if (!spinor_fp32 && !links_fp32)
        hipLaunchKernelGGL((k_wilson_h<double, cd, cd>), grid, blk, 0, st, (const cd*)in, (cd*)out,
                           (const cd*)U, a, bt);
    else if (!spinor_fp32 && links_fp32)
        hipLaunchKernelGGL((k_wilson_h<double, cd, cf>), grid, blk, 0, st, (const cd*)in, (cd*)out,
                           (const cf*)U, a, bt);
    else if (spinor_fp32 && links_fp32)
        hipLaunchKernelGGL((k_wilson_h<float, cf, cf>), grid, blk, 0, st, (const cf*)in, (cf*)out,
                           (const cf*)U, a, bt);
    else
        hipLaunchKernelGGL((k_wilson_h<float, cf, cd>), grid, blk, 0, st, (const cf*)in, (cf*)out,
                           (const cd*)U, a, bt);
    OSA_LAUNCH_CHECK();
}

void launch_wilson_h_contig(const void* in, void* out, const void* U, bool links_fp32,
                            bool spinor_fp32, const Geom& g, const HopCoef& c, int nrhs,
                            hipStream_t st) {
    const size_t es = spinor_fp32 ? sizeof(cf) : sizeof(cd);
    for (int r0 = 0; r0 < nrhs; r0 += kMaxBatch) {
        Batch bt;
        bt.n = (nrhs - r0 < kMaxBatch) ? nrhs - r0 : kMaxBatch;
        bt.basis = bt.vec = g.N();
        const size_t off = (size_t)r0 * g.N() * es;
        launch_wilson_h((const char*)in + off, (char*)out + off, U, links_fp32, spinor_fp32, g, c,
                        st, bt);
    }
}

}  // namespace osa
