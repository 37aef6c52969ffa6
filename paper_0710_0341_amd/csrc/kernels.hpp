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

// ------------------------------------------------------------- batching
// One launch can work on several independent problems (sources) at once.
// Launch entry z works on problem idx[z]; an array argument of problem b starts
// at its base pointer plus b times the stride named below (in elements of that
// array; 0 = shared by all problems).  A default Batch is the single-problem
// case.  Each launcher states which strides it reads.
constexpr int kMaxBatch = 64;
struct Batch {
    int n = 1;
    int64_t basis = 0;   // a basis / the columns read by a dot or an update
    int64_t vec = 0;     // an N-length work vector
    int64_t small = 0;   // coefficient vectors (h columns, G^{-1} L^dag w, s)
    int64_t part = 0;    // partial-sum workspace
    int64_t scal = 0;    // per-problem scalar slots (cd)
    int64_t flag = 0;    // per-problem int flags
    int64_t mat = 0;     // small dense matrices
    int64_t ws = 0;      // small dense workspace (bytes)
    int16_t idx[kMaxBatch];
    Batch() { for (int i = 0; i < kMaxBatch; ++i) idx[i] = (int16_t)i; }
};

// ------------------------------------------------------------- layout (S0)
void launch_links_to_internal(const void* links_aos, bool in_fp32, void* links_int,
                              bool int_fp32, const Geom& g, hipStream_t st);
void launch_vec_to_internal(const cd* aos, void* soa, bool soa_fp32, const Geom& g,
                            int nvec, hipStream_t st);
void launch_vec_from_internal(const void* soa, bool soa_fp32, cd* aos, const Geom& g,
                              int nvec, hipStream_t st);

// ------------------------------------------------------------- stencil (S1)
// out = gamma_5 D_w(mu) in.  Batch strides: basis (in), vec (out).  The
// problems of a batch share the links; the launch visits each block of sites
// for all problems back to back so that the links are read from HBM once.
void launch_wilson_h(const void* in, void* out, const void* U, bool links_fp32,
                     bool spinor_fp32, const Geom& g, const HopCoef& c, hipStream_t st,
                     const Batch& bt = Batch());
// Contiguous vectors: nrhs inputs and outputs spaced by the internal length.
void launch_wilson_h_contig(const void* in, void* out, const void* U, bool links_fp32,
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
// B: ncols vectors of length n (= p.n) spaced by ldb; storage fp64 or fp32.
// The launch picks its row chunks from n and ncols (at most kMaxChunks) and
// returns their number, which the following reduction takes.
// Batch strides: basis (B), vec (w), part (partial).
constexpr int kMaxChunks = 128;
// Autotuner of the dot kernels' row chunking (process-wide, on by default):
// see blas.hip.  autotune_entries copies up to cap (n, bucket, chunk count)
// entries and returns how many there are.
void set_autotune(bool on);
bool autotune_enabled();
int autotune_entries(int64_t* n, int* bucket, int* want, int cap);
int launch_dot_partial(const void* B, int64_t ldb, int ncols, const void* w, bool fp32,
                       const TsPlan& p, cd* partial, hipStream_t st, const Batch& bt = Batch());
// out[c] = sum_q partial[c*nchunks+q] and accum[c] += out[c] (accum nullable).
// With M != nullptr (m x m, column-major) out = M * sums instead (used for
// G^{-1} L^dag w, M shared by the batch); tmp then holds ncols scratch entries.
// Batch strides: part (partial), small (out, accum, tmp).
void launch_reduce_partial(const cd* partial, int nchunks, int ncols, cd* out, cd* accum,
                           const cd* M, cd* tmp, hipStream_t st, const Batch& bt = Batch());
// w[i] = alpha*w[i] - sum_c B[c][i] coef[c]  (coef on device).  If normp != nullptr
// the kernel also writes per-256-row partial sums of |w|^2 into normp.
// scratch (scratch_len cd entries in total) is shared out among the batch.
// Batch strides: vec (w), basis (B), small (coef), part (normp).
void launch_update(void* w, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                   const TsPlan& p, double* normp, cd* scratch, int64_t scratch_len,
                   hipStream_t st, const Batch& bt = Batch());
// y[i] = sum_c B[c][i] coef[c] + (add ? y[i] : 0).  Batch strides as launch_update.
void launch_combine(void* y, const void* B, int64_t ldb, int ncols, const cd* coef, bool fp32,
                    bool add, int64_t n, hipStream_t st, const Batch& bt = Batch());
// Shared columns B (fp64) against the vectors of several problems, B read once
// per group of problems, with the per-problem arithmetic of launch_dot_partial
// (same plan, same summation order: bitwise equal results).  Returns nchunks.
// Batch strides: vec (w), part (partial).
int launch_mdot_partial(const cd* B, int64_t ldb, int ncols, const cd* w, const TsPlan& p,
                        cd* partial, hipStream_t st, const Batch& bt);
// w_v -= B coef_v for the nv vectors v of every problem b (fp64, ncols <= 64):
// vector t of problem b at w + b*bt.vec + t*off2, its coefficients at
// coef + b*bt.small + t*coff2; B read once per 24 vectors; bitwise what
// launch_update does for each vector alone whenever mupdate_matches_single(n,
// ncols).  nv is 1 or 2.
bool mupdate_matches_single(int64_t n, int ncols);
void launch_mupdate(cd* w, const cd* B, int64_t ldb, int ncols, const cd* coef, int64_t n,
                    hipStream_t st, const Batch& bt, int nv = 1, int64_t off2 = 0,
                    int64_t coff2 = 0);
// LR projection dots: partial[b*bt.part + (t*m + c)*nchunks + q] = chunk q of
// conj(L[c]) . w_(b,t) for the m <= kPdMaxM shared columns L and the nv (1 or 2)
// vectors of every problem b (vector t at w + b*bt.vec + t*off2), L and the
// vectors read once from HBM for up to 24 vectors.  The chunk plan pdot_plan
// depends on (n, m) only and every (column, vector) dot has one fixed
// summation order, so batched results are bitwise those of one vector alone.
// Returns nchunks (for launch_reduce_partial).
constexpr int kPdMaxM = 64;
TsPlan pdot_plan(int64_t n, int m);
int launch_pdot_partial(const cd* L, int64_t ldl, int m, const cd* w, int64_t off2, int nv,
                        int64_t n, cd* partial, hipStream_t st, const Batch& bt);
// w_b = a w_b + sg B coef_b for every problem b (fp64, any ncols), B read once per
// 16 problems.  Batch strides: vec (w), small (coef).
void launch_mcombine(cd* w, const cd* B, int64_t ldb, int ncols, const cd* coef, int64_t n,
                     double a, double sg, hipStream_t st, const Batch& bt);
// Delayed reorthogonalisation (step j >= 1 of the Arnoldi recurrence).
// Dots of the ncols columns of B with two vectors in one read of B:
// partial[c*nchunks + q] for w1, partial[(ncols + c)*nchunks + q] for w2.
// Batch strides: basis (B and w1, which is a column of the basis), vec (w2),
// part (partial).
int launch_dot2_partial(const void* B, int64_t ldb, int ncols, const void* w1, const void* w2,
                        bool fp32, const TsPlan& p, cd* partial, hipStream_t st,
                        const Batch& bt = Batch());
// From d = [s, u^H u, t, u^H z] (2(j+1) entries): completes column j-1 of H,
// writes the first-pass column j and sc = [1/r, c_j]; breakdown test as
// launch_normalize (flag[1] = j - 1).  hess: H is upper Hessenberg (else all
// of H[0:j+1, 0:j] enters the first-pass correction).  first_pass = false:
// d = [s, u^H u] only; column j-1 and sc[0] = 1/r are set.
// Batch strides: small (H, d), scal (sc, and hfro2 in cd slots), flag.
// Two-step block Arnoldi (see blas.hip): dots of ncols basis columns with the
// four basis columns W .. W + 3 ldw; X M into nout (2 or 4) columns from o0;
// the first-step and per-step coefficient kernels on the per-problem
// workspace b2 (slot length vl).
int launch_dot4_partial(const cd* B, int64_t ldb, int ncols, const cd* W, int64_t ldw,
                        const TsPlan& pn, cd* partial, hipStream_t st, const Batch& bt);
void launch_blk_update(cd* V, int64_t ldb, int nin, const cd* M, int ldm, int o0, int nout,
                       int64_t n, hipStream_t st, const Batch& bt);
void launch_blk2_init(cd* b2, int vl, const cd* d, hipStream_t st, const Batch& bt);
void launch_blk2_coef(int n, cd* H, int ldh, cd* b2, int vl, double* hfro2, int* flag,
                      double rel, hipStream_t st, const Batch& bt);
void launch_dcgs_coef(int j, cd* H, int ldh, const cd* d, cd* sc, double* hfro2, int* flag,
                      double rel, hipStream_t st, const Batch& bt = Batch(), bool hess = true,
                      bool first_pass = true);
// V[j] <- (V[j] - V_j s) / r and V[j+1] <- (z - V_j t - c_j V[j]) / r in one pass
// over V_j (s = coef[0:j], t = coef[j+1:2j+1], sc = [1/r, c_j]).  scratch:
// 16 n entries per problem for the column split.  Batch strides: basis (V),
// vec (z), small (coef), scal (sc).
void launch_dcgs_update(void* V, int64_t ldb, int j, const void* z, const cd* coef, const cd* sc,
                        bool fp32, int64_t n, cd* scratch, int64_t scratch_len, hipStream_t st,
                        const Batch& bt = Batch());
// Partial sums of |w|^2 per 256 rows.  Batch strides: vec (w), part (normp).
void launch_norm_partial(const void* w, bool fp32, const TsPlan& p, double* normp,
                         hipStream_t st, const Batch& bt = Batch());
// hsub = sqrt(sum normp); v = w / hsub unless hsub <= rel*sqrt(hfro2 + hsub^2)
// (breakdown: flag[0] = 1 and flag[1] = step of the first one, v = 0; a
// non-finite norm sets flag[0] = 2).  v == nullptr computes the norm only.
// hcol (nullable, hlen entries) is added to hfro2 first: the running squared
// Frobenius norm of the Hessenberg matrix.  Batch strides: part (normp),
// scal (hsub and hfro2, counted in cd slots), flag (flag), small (hcol),
// vec (w), basis (v).
void launch_normalize(const void* w, void* v, bool fp32, const TsPlan& p, const double* normp,
                      cd* hsub, double* hfro2, double rel, int* flag, int step,
                      const cd* hcol, int hlen, hipStream_t st, const Batch& bt = Batch());
// v = alpha * w (alpha on host)
void launch_scale(const void* w, void* v, bool fp32, int64_t n, double alpha, hipStream_t st);
// v = w / f (divide) or v = w * f, with the real scalar f = factor->x on the
// device.  Batch strides: vec (w), basis (v), scal (factor).
void launch_scale_dev(const void* w, void* v, bool fp32, int64_t n, const cd* factor, bool divide,
                      hipStream_t st, const Batch& bt = Batch());
// out[c] = sum_r B[r][i] Z[r + c*ldz], c < ncols_out, r < ncols_in  (basis rotation)
void launch_rotate(const void* B, int64_t ldb, int ncols_in, const cd* Z, int ldz,
                   int ncols_out, void* out, int64_t ldo, bool fp32, int64_t n, hipStream_t st);
// fp32 <-> fp64 vector copies
void launch_convert(const void* src, bool src_fp32, void* dst, bool dst_fp32, int64_t n,
                    hipStream_t st);
// Zero bytes (a multiple of 4) of device memory with a kernel.
void launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// Deterministic pseudo-random unit-variance complex vector (counter-based hash),
// zero on padding sites.
void launch_random_vector(void* v, bool fp32, const Geom& g, uint64_t seed, hipStream_t st);

// ----------------------------------------------------- small dense (S5,S6)
// Gauss-Jordan inverse of a k x k column-major complex matrix (in place in M),
// written to Y (may equal nothing else).  logpiv[t] = log|pivot_t|; flag != 0 on
// a zero pivot.  Work arrays: ws of at least gj_ws_bytes(k) bytes.
// Batch strides: mat (M, Y), small (logpiv, in doubles), flag (flag), ws (bytes).
size_t gj_ws_bytes(int k);
void gj_invert(cd* M, cd* Y, int k, double* logpiv, int* flag, void* ws, hipStream_t st,
               const Batch& bt = Batch());
// X <- (mu X + Y / mu) / 2 with mu = exp(-sum(logpiv)/k) if bit b of scale_mask
// is set for problem b, else mu = 1; red[0] = |Xnew - X|^2, red[1] = |Xnew|^2.
// red needs newton_red_len(k) doubles per problem.
// Batch strides: mat (X, Y), small (logpiv, doubles), part (red, doubles).
int64_t newton_red_len(int k);
void launch_newton_combine(cd* X, const cd* Y, int k, const double* logpiv, uint64_t scale_mask,
                           double* red, hipStream_t st, const Batch& bt = Batch());
// Copy the leading k x k block of A (leading dimension lda) to X (ld k).
// Batch strides: basis (A), mat (X).
void launch_copy_square(const cd* A, int lda, cd* X, int k, hipStream_t st,
                        const Batch& bt = Batch());
// s = first column of X (k x k).  Batch strides: mat (X), small (s).
void launch_copy_col0(const cd* X, int k, cd* s, hipStream_t st, const Batch& bt = Batch());
// small complex GEMM: C = alpha * op(A) op(B) + beta * C, column-major.
// opA/opB: 0 = N, 1 = conjugate transpose.
void launch_zgemm(int opA, int opB, int m, int n, int kk, cd alpha, const cd* A, int lda,
                  const cd* B, int ldb, cd beta, cd* C, int ldc, hipStream_t st);
// Batched square complex GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4):
//   Out = alpha A B + beta Cin + delta I   (n x n, column-major, ld n).
// Out must not alias A or B (Cin may equal Out; Cin may be null when beta = 0).
// With part != nullptr the per-workgroup partial sums of |Out|^2 go to part
// (zgemm_part_len(n) doubles per problem) and, with norm2 != nullptr, their
// fixed-order sum |Out|_F^2 to norm2.  Batch strides: mat (A, B, Cin, Out),
// part (part, doubles), scal (norm2, doubles).
int64_t zgemm_part_len(int n);
void launch_zgemm_sq(int n, cd alpha, const cd* A, const cd* B, double beta, const cd* Cin,
                     double delta, cd* Out, double* part, double* norm2, hipStream_t st,
                     const Batch& bt = Batch());
// *out = |s - [sprev; 0]|  (device).  Batch strides: small (s, sprev),
// scal (out, counted in doubles).
void launch_diff_norm(const cd* s, int k, const cd* sprev, int kprev, double* out,
                      hipStream_t st, const Batch& bt = Batch());
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
