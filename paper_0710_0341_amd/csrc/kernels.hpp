// Launchers of the osa HIP kernels (gfx950).  All vectors use the internal
// structure-of-arrays layout: component c = spin*3 + color of site s lives at
// v[c*Vp + s]; padding sites s in [V, Vp) hold zeros.  Links: entry (nu, a, b)
// of site s at U[((nu*3 + a)*3 + b)*Vp + s].
#pragma once

#include "common.hpp"

namespace osa {

// Hop coefficients of Eq. 2 per direction: fwd[nu] multiplies (1+gamma) U_{n,nu}
// psi_{n+nu}, bwd[nu] multiplies (1-gamma) U^dag_{n-nu,nu} psi_{n-nu}.
struct HopCoef {
    double fwd[4];
    double bwd[4];
};

// ------------------------------------------------------------- layout (S0)
void launch_links_to_internal(const void* links_aos, bool in_fp32, void* links_int,
                              bool int_fp32, const Geom& g, hipStream_t st);
void launch_vec_to_internal(const cd* aos, void* soa, bool soa_fp32, const Geom& g,
                            int nvec, hipStream_t st);
void launch_vec_from_internal(const void* soa, bool soa_fp32, cd* aos, const Geom& g,
                              int nvec, hipStream_t st);

// ------------------------------------------------------------- stencil (S1)
// out = gamma_5 D_w(mu) in, for nrhs vectors spaced by the internal length.
void launch_wilson_h(const void* in, void* out, const void* U, bool links_fp32,
                     bool spinor_fp32, const Geom& g, const HopCoef& c, int nrhs,
                     hipStream_t st);

// ------------------------------------------------- tall-skinny BLAS (S3,S4,S7)
// Workspace sizes for the two-stage reductions.
struct TsPlan {
    int64_t n;        // rows
    int rows_per_chunk;
    int nchunks;
};
TsPlan ts_plan(int64_t n);

// partial[c*nchunks + q] = sum over chunk q of conj(B[c][i]) w[i], c < ncols.
// B: ncols vectors of length n spaced by ldb; storage fp64 or fp32.
void launch_dot_partial(const void* B, int64_t ldb, int ncols, const void* w, bool fp32,
                        const TsPlan& p, cd* partial, hipStream_t st);
// out[c] = sum_q partial[c*nchunks+q] and accum[c] += out[c] (accum nullable).
// With M != nullptr (m x m, column-major) out = M * sums instead (used for
// G^{-1} L^dag w); tmp then holds ncols scratch entries.
void launch_reduce_partial(const cd* partial, int nchunks, int ncols, cd* out, cd* accum,
                           const cd* M, cd* tmp, hipStream_t st);
// w[i] = alpha*w[i] - sum_c B[c][i] coef[c]  (coef on device).  If normp != nullptr
// the kernel also writes per-chunk partial sums of |w|^2 (plan p) into normp.
void launch_update(void* w, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                   const TsPlan& p, double* normp, cd* scratch, int64_t scratch_len,
                   hipStream_t st);
// y[i] = sum_c B[c][i] coef[c] + (add ? y[i] : 0)
void launch_combine(void* y, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                    bool add, int64_t n, hipStream_t st);
// Partial sums of |w|^2 per chunk.
void launch_norm_partial(const void* w, bool fp32, const TsPlan& p, double* normp,
                         hipStream_t st);
// hsub = sqrt(sum normp); v = w / hsub unless hsub <= rel*sqrt(hfro2 + hsub^2)
// (breakdown: flag[0] = 1 and flag[1] = step of the first one, v = 0; a
// non-finite norm sets flag[0] = 2).  v == nullptr computes the norm only.
// hcol (nullable, hlen entries) is added to hfro2 first: the running squared
// Frobenius norm of the Hessenberg matrix.
void launch_normalize(const void* w, void* v, bool fp32, const TsPlan& p, const double* normp,
                      cd* hsub, double* hfro2, double rel, int* flag, int step,
                      const cd* hcol, int hlen, hipStream_t st);
// v = alpha * w (alpha on host)
void launch_scale(const void* w, void* v, bool fp32, int64_t n, double alpha, hipStream_t st);
// out[c] = sum_r B[r][i] Z[r + c*ldz], c < ncols_out, r < ncols_in  (basis rotation)
void launch_rotate(const void* B, int64_t ldb, int ncols_in, const cd* Z, int ldz,
                   int ncols_out, void* out, int64_t ldo, bool fp32, int64_t n, hipStream_t st);
// fp32 <-> fp64 vector copies
void launch_convert(const void* src, bool src_fp32, void* dst, bool dst_fp32, int64_t n,
                    hipStream_t st);
// Deterministic pseudo-random unit-variance complex vector (counter-based hash),
// zero on padding sites.
void launch_random_vector(void* v, bool fp32, const Geom& g, uint64_t seed, hipStream_t st);

// ----------------------------------------------------- small dense (S5,S6)
// Gauss-Jordan inverse of a k x k column-major complex matrix (in place in M),
// written to Y (may equal nothing else).  logpiv[t] = log|pivot_t|; flag != 0 on
// a zero pivot.  Work arrays: ws of at least gj_ws_bytes(k) bytes.
size_t gj_ws_bytes(int k);
void gj_invert(cd* M, cd* Y, int k, double* logpiv, int* flag, void* ws, hipStream_t st);
// X <- (mu X + Y / mu) / 2 with mu = exp(-sum(logpiv)/k) if scale else 1;
// red[0] += |Xnew - X|^2, red[1] += |Xnew|^2 (red zeroed by the launcher).
void launch_newton_combine(cd* X, const cd* Y, int k, const double* logpiv, bool scale,
                           double* red, hipStream_t st);
// small complex GEMM: C = alpha * op(A) op(B) + beta * C, column-major.
// opA/opB: 0 = N, 1 = conjugate transpose.
void launch_zgemm(int opA, int opB, int m, int n, int kk, cd alpha, const cd* A, int lda,
                  const cd* B, int ldb, cd beta, cd* C, int ldc, hipStream_t st);
// est = beta_ * |s - [sprev; 0]| / bnorm  written into *out (device)
void launch_diff_norm(const cd* s, int k, const cd* sprev, int kprev, double* out,
                      hipStream_t st);
// Small Schur decomposition A = Z T Z^H (p <= 96) with the diagonal of T sorted
// by |t_ii| ascending (mode 0) or |Re t_ii| ascending (mode 1).  A, T, Z:
// column-major p x p (ld = p).  w: eigenvalues (p).  info[0]: QR iterations or
// -1, info[1]: scratch (2 ints).  p > 64 needs ws of schur_ws_bytes(p) bytes.
size_t schur_ws_bytes(int p);
void small_schur(const cd* A, int p, cd* T, cd* Z, cd* w, int mode, int* info, void* ws,
                 hipStream_t st);
// Eigenvectors of A = Z T Z^H from its Schur form: Y = Z * eigvec(T), unit columns.
void small_eigvecs(const cd* T, const cd* Z, int p, cd* Y, hipStream_t st);

}  // namespace osa
