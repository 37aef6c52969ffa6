/*
 * osa.h -- overlap sign apply: y = sign(H_w(mu)) b on AMD MI355X (gfx950).
 *
 * C ABI of the library libosa.so.  The method is the LR-deflated Arnoldi
 * approximation of Bloch, Wettig, Frommer and Lang, "An iterative method to
 * compute the overlap Dirac operator at nonzero chemical potential":
 *
 *   H_w(mu) = gamma_5 D_w(mu)                 (Eq. 1, Eq. 2)
 *   f(A) x ~ R f(Lambda) L^dag x + beta V_k f(H_k) e_1     (Eq. 22, f = sgn)
 *
 * with R, L the right/left eigenvectors of the m critical eigenvalues
 * (smallest |Re lambda|, Eq. 20), V_k, H_k the Arnoldi basis and Hessenberg
 * matrix of the deflated source (Eq. 7 applied to x_ominus, Eq. 21), and
 * f(H_k) e_1 the first column of the sign of the small Hessenberg matrix.
 *
 * CONVENTIONS (all entry points)
 *  - Pointers are DEVICE pointers unless the comment says (host).
 *  - complex = interleaved (re, im): complex128 = 2 x double, complex64 = 2 x float.
 *  - Site index  site = x + Lx*(y + Ly*(z + Lz*t)), V = Lx*Ly*Lz*Lt.
 *  - Vector index i = (site*4 + spin)*3 + color, N = 12*V complex128 entries.
 *  - Links U[((site*4 + nu)*3 + a)*3 + b] = (U_{site,nu})_{ab}; nu = 0,1,2 are
 *    x,y,z and nu = 3 is the temporal direction that carries e^{+-mu}.
 *  - Gamma matrices in the chiral basis: gamma_k = [[0,-i s_k],[i s_k,0]],
 *    gamma_4 = [[0,1],[1,0]], gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 =
 *    diag(1,1,-1,-1).  Boundary conditions are periodic, optionally
 *    antiperiodic in time.
 *  - All work is ordered on the stream given at creation (NULL = default
 *    stream).  Calls that write (host) outputs synchronise that stream first.
 *  - No exception or exit() crosses the ABI: every call returns osa_status.
 *  - Ownership: the caller owns links, sources, results and every buffer it
 *    passes; they must stay valid until the call returns.  The library copies
 *    the links at creation.  The context owns all workspace (Krylov basis,
 *    Hessenberg matrix, deflation vectors, scratch), allocated with hipMalloc
 *    at creation / deflation and freed by osa_destroy.
 */
#ifndef OSA_H
#define OSA_H

#include <stdint.h>
#include <stddef.h>

#if defined(__GNUC__)
#define OSA_API __attribute__((visibility("default")))
#else
#define OSA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OSA_OK = 0,
    OSA_NOT_CONVERGED = 1,      /* result usable: best iterate at k_max, resid_est > tol     */
    OSA_ERR_ARG = -1,           /* invalid argument; detected before any device work          */
    OSA_ERR_HIP = -2,           /* a HIP runtime call failed                                   */
    OSA_ERR_OOM = -3,           /* workspace allocation failed                                 */
    OSA_ERR_NONFINITE = -4,     /* NaN / Inf in the input or an intermediate                   */
    OSA_ERR_IMAG_AXIS = -5,     /* a deflated eigenvalue lies on the imaginary axis (sgn undefined, Eq. 5) */
    OSA_ERR_EIG_NOCONV = -6,    /* critical eigenpairs not found to the requested accuracy     */
    OSA_ERR_NEWTON_NOCONV = -7, /* the small sign iteration did not converge                  */
    OSA_ERR_STATE = -8          /* call out of order (e.g. apply before deflation when m > 0)  */
} osa_status;

typedef enum { OSA_FP64 = 0, OSA_FP32 = 1 } osa_prec;

typedef struct {
    int32_t dims[4];            /* Lx, Ly, Lz, Lt; each >= 2                                   */
    int32_t antiperiodic_t;     /* 1: factor -1 on temporal hops across the boundary          */
} osa_lattice;

/* Options; an all-zero struct selects every default. */
typedef struct {
    int32_t k_max;              /* Krylov size cap for the solve            (default 600)     */
    int32_t check_every;        /* convergence check interval (default 50); < 0: run exactly
                                   k_max steps with no check (fixed-k mode)                   */
    int32_t no_reproject;       /* 1: skip the per-step oblique re-projection (default 0)     */
    int32_t eig_ncv;            /* eigensolver block, 8..96: the Krylov-Schur active block
                                   (default nev + 16 within [64, 96], nev = wanted
                                   eigenvalues of H^2) or the filtered block (default
                                   nev + 48 within [64, 96], see eig_filter); if that run does not
                                   converge, osa_deflate runs once more with 96 and twice
                                   the restart cap                                          */
    int32_t eig_max_restarts;   /* eigensolver restart cap                 (default 2000)     */
    osa_prec eig_prec;          /* FP32: search in FP32, then refine in FP64 (default FP64)   */
    double eig_tol;             /* relative Krylov-Schur residual target   (default 1e-12)    */
    int32_t max_batch;          /* sources solved together in lockstep by osa_apply, 1..64
                                   (default 16); workspace grows with it: max_batch Krylov
                                   bases of k_max + 2 vectors of N complex128                */
    int32_t orth;               /* Arnoldi orthogonalisation of the solve (Eq. 7) and of
                                   the eigensolver's Krylov-Schur expansion:
                                   0 (default): classical Gram-Schmidt with the second pass
                                   delayed by one step: one dot pass over the basis with two
                                   vectors and one fused update pass per step (half the
                                   basis traffic); 1: classical Gram-Schmidt applied twice
                                   in the same step (four passes); 2: the solve extends
                                   the basis by two vectors (H u, H^2 u) per outer step
                                   with one dot pass and one update pass over the basis
                                   (half the basis traffic of 0), the second pass again
                                   delayed; checks at the same sizes as with 0.  Under
                                   Schur deflation the solve uses 0; the eigensolver
                                   uses 0                                                  */
    int32_t eig_filter;         /* FP64 search for the critical pairs: 0 (default)
                                   Krylov-Schur; d in 1..200: Chebyshev-filtered subspace
                                   iteration on H^2 with a degree-d filter and a block of
                                   eig_ncv vectors (default nev + 48 within [64, 96]);
                                   Krylov-Schur takes over if 80 filter iterations do not
                                   converge.  The FP32 search always uses Krylov-Schur     */
    int32_t deflation;          /* deflation scheme of the solve:
                                   0 (default): LR deflation (Eq. 20-22) with the left and
                                   right critical eigenvectors;
                                   1: Schur deflation (Eq. 13-19): right eigenvectors only
                                   (osa_deflate then skips the left ones), an orthonormal
                                   Schur basis S_m with A S_m = S_m T_m, Arnoldi vectors
                                   orthogonalised against S_m as well (plain CGS2, orth is
                                   ignored) and the coupling block Y of Eq. 17 taken from the
                                   sign of the block matrix of Eq. 15.  Data from a Schur-mode
                                   osa_deflate serves only Schur-mode solves: an LR solve or
                                   osa_apply_adjoint on it returns OSA_ERR_STATE            */
    int32_t stop_rule;          /* convergence estimate resid_est (the paper gives no stopping
                                   rule; est = beta |s_k - s_k'| / |b| is the change since the
                                   previous check k', about the error of check k'):
                                   0 (default): twice the geometric tail est rho^d /
                                   (1 - rho^d), d = k - k', with rho the per-step rate from
                                   the last two
                                   changes (the slower of the last two rates); the first
                                   estimate is the change itself;
                                   1: the change itself                                    */
    int32_t no_graphs;          /* 1: launch every Arnoldi step directly.  Default 0: the steps
                                   between two convergence checks (a segment) are recorded as a
                                   HIP graph the second time the same segment (same steps,
                                   active sources and deflation size) comes up, and replayed
                                   with one graph launch from then on (bitwise the same
                                   results); kernel timing (osa_profile_enable) and any
                                   workspace reallocation switch replay off or reset it      */
} osa_opts;

/* Per-solve diagnostics (host struct). */
typedef struct {
    double resid_est;           /* beta |s_k - s_k'| / |y|: change since the previous check   */
    double min_abs_re_lambda;   /* smallest |Re lambda| among the deflated eigenvalues         */
    double max_eig_resid;       /* max_i |H r_i - lambda_i r_i| / |r_i| (also over left vectors) */
    double t_init_ms;           /* deflation (eigensolver) time                               */
    double t_solve_ms;          /* Arnoldi + small sign + assembly time                       */
    int32_t k_used;             /* Krylov size of the returned result                        */
    int32_t n_defl;             /* number of deflated eigenpairs m                            */
    int32_t status;             /* osa_status of this source                                  */
    int32_t newton_iters;       /* iterations of the final small sign                         */
    int64_t eig_matvecs;        /* stencil applications spent in the eigensolver             */
    int32_t eig_restarts;       /* eigensolver restarts (right + left)                        */
    int32_t breakdown;          /* 1: happy Arnoldi breakdown (result exact in K_k)           */
    int32_t batch;              /* number of sources in the lockstep batch this one ran in;
                                   t_solve_ms is that batch's wall time                      */
} osa_info;

typedef struct osa_ctx osa_ctx;

/* ---------------------------------------------------------------------------
 * One-shot form: y = sign(H_w(mu)) b with n_defl deflated critical eigenpairs.
 * Operator: Eq. 2 with kappa = 1/(8 + 2 m_w), m_w in (-2, 0) (definition
 * section); method: Eq. 20-22.
 *   lat        (host) lattice extents and boundary condition
 *   links      V*4*9 complex, complex128 if link_prec == OSA_FP64 else complex64
 *              (FP32 links define the operator exactly as stored)
 *   source     N complex128;   result  N complex128 (may not alias source)
 *   tol        > 0, stop threshold on the convergence estimate
 *   n_defl     0 <= n_defl < N and n_defl <= 48 (else OSA_ERR_ARG)
 *   resid_est  (host, may be NULL) final convergence estimate
 * Returns OSA_OK, OSA_NOT_CONVERGED (result usable) or an error.
 * ------------------------------------------------------------------------- */
OSA_API osa_status overlap_sign_apply(const osa_lattice* lat, const void* links, osa_prec link_prec,
                              double mu, double m_w, const void* source, double tol,
                              int32_t n_defl, void* result, double* resid_est, void* stream);

/* ---------------------------------------------------------------------------
 * Reusable form.  The deflation data is the expensive, reusable state (the
 * initialisation phase of the Results section): create once, deflate once,
 * apply to many sources.
 * ------------------------------------------------------------------------- */

/* Create a context for H_w(mu) on the given links (copied to the device in
 * the internal layout).  opts may be NULL (defaults).  stream: hipStream_t. */
OSA_API osa_status osa_create(osa_ctx** out, const osa_lattice* lat, const void* links,
                      osa_prec link_prec, double mu, double m_w, const osa_opts* opts,
                      void* stream);

/* Compute the n_defl critical eigenpairs (Eq. 20): right eigenvectors of
 * H_w(mu) and left ones as right eigenvectors of H_w(-mu) = H_w(mu)^dag, by
 * Krylov-Schur on H^2 followed by a Rayleigh-Ritz step with H; selects the
 * n_defl eigenvalues of smallest |Re lambda| among the converged ones.
 * With opts.deflation = 1 (Schur deflation) only the right eigenvectors are
 * computed: the paper's remark that Schur deflation halves the set-up cost.
 * info (host, may be NULL) receives eigensolver statistics.
 * Errors: OSA_ERR_ARG (n_defl < 0, n_defl > 48 or n_defl >= N),
 * OSA_ERR_EIG_NOCONV, OSA_ERR_IMAG_AXIS (|Re lambda| < 1e-12 |H|). */
OSA_API osa_status osa_deflate(osa_ctx* ctx, int32_t n_defl, osa_info* info);

/* Import deflation data: R, L are m vectors each (m*N complex128, vector j at
 * offset j*N, boundary layout); lambda (host) holds m complex128 values
 * (re, im interleaved).  Only the projector R (L^dag R)^{-1} L^dag and the
 * eigenvalues matter; scale and phase of the vectors are free.  Under Schur
 * deflation (opts.deflation = 1) L may be NULL: only span(R) is used.
 * 0 <= m <= 64 and m < N, else OSA_ERR_ARG. */
OSA_API osa_status osa_set_deflation(osa_ctx* ctx, int32_t m, const void* R, const void* L,
                             const double* lambda);

/* Export the current deflation data in the same layout (buffers of m*N
 * complex128; lambda (host) 2m doubles).  m_out (host) receives m.  L must
 * be NULL when the data holds no left vectors (a Schur-mode deflation):
 * OSA_ERR_STATE otherwise. */
OSA_API osa_status osa_get_deflation(const osa_ctx* ctx, int32_t* m_out, void* R, void* L,
                             double* lambda);

/* Use only the first m deflation pairs (in |Re lambda| order); m <= current. */
OSA_API osa_status osa_set_active_deflation(osa_ctx* ctx, int32_t m);

/* Y = sign(H_w(mu)) B for nrhs sources (Eq. 22).  B, Y: nrhs*N complex128,
 * source j at offset j*N.  All sources share the operator and the deflation
 * data.  Up to opts.max_batch sources run in lockstep: each Arnoldi step
 * applies the stencil (links read once for the batch), the re-projection, the
 * Gram-Schmidt passes and the small sign to all of them with shared launches,
 * while every source keeps its own Krylov basis, convergence check and
 * stopping point (the method itself is per source, Eq. 22).  infos (host,
 * may be NULL) receives nrhs osa_info records.  Returns the first error in
 * source order, else the worst status; Y of a source with an error status is
 * left unwritten. */
OSA_API osa_status osa_apply(osa_ctx* ctx, int32_t nrhs, const void* B, void* Y, double tol,
                     osa_info* infos);

/* Y = sign(H_w(mu))^dag B for nrhs sources, with the same arguments, batching
 * and statuses as osa_apply.  Since H_w(mu)^dag = H_w(-mu) (the adjoint
 * identity behind Eq. 20), sign(H)^dag = sign(H(-mu)): the Arnoldi runs on
 * H(-mu), and the deflation data of H(mu) serves unchanged with the roles of
 * the left and right eigenvectors exchanged and lambda -> conj(lambda) (the
 * same signs of Re lambda); the remark on sign(H) and sign(H)^dag in the
 * results section.  Needs LR deflation data (left vectors): under Schur
 * deflation (opts.deflation = 1) it returns OSA_ERR_STATE. */
OSA_API osa_status osa_apply_adjoint(osa_ctx* ctx, int32_t nrhs, const void* B, void* Y,
                                     double tol, osa_info* infos);

/* Y = D_ov B = B + gamma_5 sign(H_w(mu)) B, the overlap operator of Eq. 1, for
 * nrhs sources (gamma_5 = diag(1, 1, -1, -1) in spin, chiral basis).  Same
 * arguments, batching and statuses as osa_apply; resid_est refers to the sign
 * part. */
OSA_API osa_status osa_apply_overlap(osa_ctx* ctx, int32_t nrhs, const void* B, void* Y,
                                     double tol, osa_info* infos);

/* Block Krylov variant for s sources (not the paper's method; its Eq. 11 and
 * Eq. 22 applied to a block of sources): one Krylov space is built from all s
 * sources together (block Arnoldi with classical Gram-Schmidt applied twice
 * and a Gram-Schmidt QR of every new block), and sign(H) B is approximated by
 * R sgn(Lambda) G^{-1} L^dag B + V_K sign(H_K) E_1 R_0 with the block Hessenberg
 * matrix H_K (K s x K s).  B, Y: s*N complex128 (source j at offset j*N).  Uses
 * the context's LR deflation data (OSA_ERR_STATE under Schur deflation).
 * k_blocks: block steps at most (0: ceil(4 k_max / s)); K s <= 6000.  Checks
 * every ceil(check_every / s) block steps (with check_every < 0 exactly
 * k_blocks steps); resid_est per source: the geometric-tail estimate of the
 * change of its column of sign(H_K) E_1 R_0 relative to |b|; k_used = K s.
 * Returns OSA_OK, OSA_NOT_CONVERGED (result usable) or an error. */
OSA_API osa_status osa_apply_block(osa_ctx* ctx, int32_t s, const void* B, void* Y, double tol,
                                   int32_t k_blocks, osa_info* infos);

/* Uneven batch: n independent contexts (different lattices, mu, m_w and
 * deflation data), one source each, solved concurrently: up to 8 instances at
 * a time, each on a stream of its own that waits for the work already queued
 * on the context's stream; the call returns when all are done.  Each result is
 * exactly what osa_apply gives for that context.  B[i], Y[i]: device pointers
 * to N_i complex128; infos (host, may be NULL) n records, whose t_solve_ms is
 * the instance's own wall time (the latency the instance saw once started).
 * The contexts must be distinct (OSA_ERR_ARG otherwise).  Returns the first
 * error in instance order, else the worst status. */
OSA_API osa_status osa_batch_apply(int32_t n, osa_ctx* const* ctxs, const void* const* B,
                           void* const* Y, double tol, osa_info* infos);

/* Replace the options of an existing context (NULL = defaults). */
OSA_API osa_status osa_set_opts(osa_ctx* ctx, const osa_opts* opts);

/* Y = H_w(mu) X (Eq. 1-2), nrhs vectors, boundary layout.  The stencil alone,
 * for operator checks. */
OSA_API osa_status osa_apply_hw(osa_ctx* ctx, int32_t nrhs, const void* X, void* Y);

/* Y = H_w(mu) X (Eq. 1-2) with the FP32 stencil of the FP32 eigensearch:
 * spinors and arithmetic in FP32, links as stored if FP32, else rounded once
 * to FP32.  X, Y: nrhs vectors of V*12 complex64 each (device, boundary
 * layout).  Checks the FP32 kernel instantiation against the operator. */
OSA_API osa_status osa_apply_hw32(osa_ctx* ctx, int32_t nrhs, const void* X, void* Y);

/* k Arnoldi steps (Eq. 7) on A = H(mu)^2 (adjoint = 0) or A = H(-mu)^2 =
 * (H(mu)^dag)^2 (adjoint = 1), by the expansion of the Krylov-Schur search for
 * the critical eigenpairs (Eq. 20): delayed second Gram-Schmidt pass, vectors
 * and stencil in precision prec (OSA_FP64 or OSA_FP32; FP32 links as for
 * osa_apply_hw32), reductions in FP64.  Gives A V_k = V_{k+1} S with
 * v_1 = x / |x|, orthonormal V and upper Hessenberg S (real positive
 * subdiagonal).  x: V*12 complex128 (device, boundary layout, not zero).
 * V: k+1 such vectors (device, output; FP32 values promoted exactly).
 * S: (k+1) x k complex128, column-major (device, output).  1 <= k <= 64 and
 * k + 1 <= 12 V, else OSA_ERR_ARG.  A check entry of the eigensearch's
 * kernels. */
OSA_API osa_status osa_krylov_h2(osa_ctx* ctx, int32_t prec, int32_t adjoint, int32_t k,
                                 const void* x, void* V, void* S);

/* s = sign(A) e_1 for a k x k complex128 matrix A stored column-major (device,
 * leading dimension k), by the scaled Newton iteration used for f(H_k) e_1.
 * s: k complex128 (device).  iters (host, may be NULL).  Standalone entry of
 * the small-sign kernel for checks; stream-ordered on `stream`. */
OSA_API osa_status osa_small_sign(int32_t k, const void* A, void* s, int32_t* iters, void* stream);

/* Allocation-free form of osa_small_sign, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same result, bit for bit, with every work array
 * in one file-scope device array of the library instead of hipMalloc'd
 * buffers.  Each GPU holds its own copy of that array (about 3.2 MB) until the
 * process ends; its device address is looked up once per device, on the first
 * call with that device current.  The caller passes A and s as for
 * osa_small_sign.  Limit: 1 <= k <= OSA_NOALLOC_MAX_K (256), else OSA_ERR_ARG
 * before any device work.  No hipMalloc, hipFree or hipMemset is issued (the
 * flags are cleared by a kernel); the host staging of the read-backs is a
 * per-thread static buffer.  All calls on one GPU share the array and it keeps
 * the last call's contents: calls that overlap in time on one GPU (several
 * streams or host threads) race and must be serialised by the caller. */
#define OSA_NOALLOC_MAX_K 256
OSA_API osa_status osa_small_sign_noalloc(int32_t k, const void* A, void* s, int32_t* iters,
                                          void* stream);

/* C_b = A_b B_b for nb pairs of n x n complex128 matrices (column-major, ld n,
 * problem b at offset b*n*n in each of A, B, C; device), on the FP64 matrix
 * cores: the product kernel of the Newton-Schulz steps X <- (3X - X^3)/2 that
 * finish the small sign f(H_k) e_1 (Eq. 11, Eq. 22).  C must not overlap A or
 * B.  1 <= n <= 4000, 1 <= nb <= 64.  Standalone entry of the kernel for
 * checks; stream-ordered on `stream`. */
OSA_API osa_status osa_small_gemm(int32_t n, int32_t nb, const void* A, const void* B, void* C,
                                  void* stream);

/* Schur decomposition A = Z T Z^H of a p x p complex128 matrix (column-major,
 * device, 1 <= p <= 96), with the diagonal of T ordered by |t_ii| ascending
 * (mode 0) or |Re t_ii| ascending (mode 1): the small dense step of the
 * eigensolver restarts.  T, Z: p x p column-major (device); w: p eigenvalues.
 * Standalone entry of the kernel for checks; stream-ordered on `stream`. */
OSA_API osa_status osa_small_schur(int32_t p, const void* A, void* T, void* Z, void* w,
                                   int32_t mode, void* stream);

/* Replace the gauge links of an existing context (same lattice, same link
 * precision, device pointer in the boundary layout).  Reuses all workspace;
 * the deflation data is dropped (m becomes 0) because it belongs to the old
 * operator. */
OSA_API osa_status osa_set_links(osa_ctx* ctx, const void* links);

/* Kernel timing with HIP events on the context's stream, for measurement.
 * Classes: 0 Gram-Schmidt / projection dot products (V^H w), 1 Gram-Schmidt
 * updates (w - V h), 2 stencil H_w(mu), 3 one small-matrix inversion of the
 * Newton iteration, 4 small Schur decomposition of an eigensolver restart,
 * 5 whole eigensolver restart (host wall clock, including synchronisation),
 * 6 complex GEMM of a Newton-Schulz step on the FP64 matrix cores.
 * every <= 0 disables timing; every = n >= 1 brackets one launch in n of each
 * class with events (the first, then every n-th), which keeps the overhead of
 * the events (a few microseconds per bracketed launch) small.  ms[], bytes[]
 * and launches[] cover the bracketed launches only, calls[] counts all of
 * them, so ms/launches is the average duration and ms/launches*calls the
 * estimated class total.  bytes[] counts the algorithmic HBM bytes of each
 * launch (vectors read and written once); flops[] the algorithmic flops of
 * each launch (class 6: 8 n^3 per complex n x n product).  counters[]: 0 QR sweeps and 1 plane
 * rotations (sweeps plus reordering) of the small Schur decompositions,
 * 2 Newton iterations of the small sign, 3 eigensolver Arnoldi steps.
 * Enabling resets everything. */
#define OSA_PROFILE_CLASSES 7
typedef struct {
    double ms[OSA_PROFILE_CLASSES];
    double bytes[OSA_PROFILE_CLASSES];
    int64_t launches[OSA_PROFILE_CLASSES];
    int64_t counters[4];
    int64_t calls[OSA_PROFILE_CLASSES];
    double flops[OSA_PROFILE_CLASSES];
} osa_profile;
OSA_API osa_status osa_profile_enable(osa_ctx* ctx, int32_t every);
OSA_API osa_status osa_profile_read(osa_ctx* ctx, osa_profile* out);

/* Autotuner of the dot kernels' row chunking (process-wide, on by default).
 * The first launch for a vector length n and column bucket ceil(ncols / 32)
 * times the candidate chunk counts (8 ... 64) on that launch's own operands and
 * keeps the fastest for every later launch with the same (n, bucket), so the
 * summation order of a problem depends on (n, ncols) alone within a process
 * (batched and single-source results stay bitwise equal); across processes the
 * chosen chunking, and with it the last bits of results, may differ.
 * osa_set_autotune(0) uses the built-in choice for keys not yet tuned.
 * osa_autotune_table copies up to cap entries (host arrays, may be NULL) and
 * returns the number of tuned keys. */
OSA_API osa_status osa_set_autotune(int32_t on);
OSA_API int32_t osa_autotune_table(int64_t* n, int32_t* bucket, int32_t* chunks, int32_t cap);

/* Graph replay counters of a context (host outputs, may be NULL): segments
 * recorded as HIP graphs, and graph launches that replaced direct launches. */
OSA_API osa_status osa_graph_stats(const osa_ctx* ctx, int64_t* captures, int64_t* launches);

/* Human-readable detail of the last error on this context ("" if none);
 * valid until the next call on the context. */
OSA_API const char* osa_last_message(const osa_ctx* ctx);

/* Device workspace allocator (process-wide).  With alloc and dealloc set, every
 * workspace buffer created afterwards comes from alloc(bytes, stream, user)
 * and returns through dealloc(ptr, stream, user) (stream is always NULL: the
 * workspace lives as long as its context, outside stream order).  The library
 * synchronises the device after each alloc and before each dealloc, so the
 * allocator may hand out blocks last used on any stream (a caching allocator
 * such as PyTorch's).  A buffer is returned through the hook that allocated
 * it, so the hook's functions must stay callable until every context created
 * under it is destroyed.  alloc returning NULL makes the calling entry point
 * fail with OSA_ERR_OOM.  Both NULL restores hipMalloc/hipFree; exactly one NULL
 * is OSA_ERR_ARG.  Pinned host staging buffers always use hipHostMalloc.
 * Not safe to call while another thread is inside the library. */
OSA_API osa_status osa_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* user),
                                     void (*dealloc)(void* ptr, void* stream, void* user),
                                     void* user);

OSA_API void osa_destroy(osa_ctx* ctx);
OSA_API const char* osa_status_string(osa_status s);
OSA_API const char* osa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OSA_H */
