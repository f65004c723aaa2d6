/*
 * gep_ci.h -- C ABI of the MI355X (gfx950) contour-integral eigensolver.
 *
 * Computes every eigenpair (lambda, x) of a sparse real symmetric pencil
 * A x = lambda B x, B symmetric positive definite (paper Sec. 3.1, Eq. GEP),
 * whose eigenvalue lies in the keep window of one of the given circular
 * contours.  The method is the moment-based CI pipeline of the paper's
 * Appendix "Numerical Implementation of CI Methods" (quadrature equation,
 * Alg. "Standard CI pipeline with contour partitioning and
 * orthogonalization", moment matrices S_m):
 *
 *   V (n x L, real Gaussian) -> for each circle and each trapezoid node z_j
 *   in the upper half plane: solve (z_j B - A) Y_j = B V (Jacobi-
 *   preconditioned COCG, all nodes x right-hand sides batched) ->
 *   S_m = sum_j 2 Re(w_j zeta_j^m Y_j) -> B-orthonormal basis Q (SVQB then a
 *   Cholesky pass) -> Rayleigh-Ritz on Q^T A Q, Q^T B Q -> Ritz vectors,
 *   residuals, keep-window selection, merge across contours.
 *
 * Conventions shared by all entry points:
 *  - Return value: 0 on success, a negative GEP_E* code on error (nothing
 *    is returned in *out), or a positive GEP_W* warning code (the result is
 *    valid but flagged).  gep_strerror() names a code; gep_last_error()
 *    gives the calling thread's last detailed message.
 *  - Inputs are borrowed: read during the call only, never retained or
 *    written.  Results are library-owned until the matching *_free call.
 *  - Pointers marked "host or device" follow gep_opts.inputs_on_device.
 *  - The library allocates its own device memory (hipMalloc) and runs all
 *    GPU work on gep_opts.stream; the call returns after that work is done.
 *  - One GPU (the current HIP device).  Calls on different streams may run
 *    concurrently; calls are not re-entrant on the same stream.
 */
#ifndef GEP_CI_H
#define GEP_CI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GEP_OK 0
#define GEP_EINVAL (-1)     /* bad argument: NULL pointer, n <= 0, odd or < 2 nodes,
                               moments/block < 1, tol <= 0, radius <= 0, keep window
                               outside the circle's real diameter, NaN/Inf values,
                               unsorted or out-of-range column indices, nnz >= 2^31 */
#define GEP_ENOTSYM (-2)    /* A or B not symmetric (|a_ij - a_ji| > 1e-12 max|a|) */
#define GEP_ENOTSPD (-3)    /* B has a non-positive diagonal entry, or a reduced
                               B-Gram matrix lost positive definiteness */
#define GEP_ENOMEM (-4)     /* not even one contour fits in device memory */
#define GEP_EDEVICE (-5)    /* a HIP runtime call failed (see gep_last_error) */
#define GEP_WNOCONV 1       /* some kept pairs have residual > tol after refinement;
                               they are returned with converged = 0 */
#define GEP_WSATURATED 2    /* some contour's subspace is saturated (its weakest
                               moment direction keeps weight > 1e-3 of the
                               strongest): eigenvalues may be missed; split the
                               contour or raise block*moments */

/* ---- method ------------------------------------------------------------ */
#define GEP_CIRR 0          /* moment-based CI (the block V, M moments, one pass, then
                               FEAST-type refinement passes if a kept pair misses tol) */
#define GEP_FEAST 1         /* FEAST subspace iteration (paper appendix, "Algorithm
                               Families"): one moment, and up to max_refine further
                               passes with V <- the contour's Ritz vectors until every
                               kept pair meets tol; block >= the contour's count */

/* ---- precision of the shifted solves --------------------------------- */
#define GEP_FP64 0          /* FP64 complex COCG throughout */
#define GEP_MIXED 1         /* shifted solves in FP32 complex (COCG with FP64
                               residual replacement, or FP32 banded factors with
                               FP64 residual refinement); orthonormalisation,
                               Rayleigh-Ritz and residuals FP64 */

/* Sparse matrix in CSR form, both triangles stored, column indices sorted
 * ascending within each row, 0-based.  rowptr has n+1 entries. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t* rowptr;   /* host or device */
    const int32_t* colind;   /* host or device */
    const double* val;       /* host or device */
} gep_csr;

/* Circle |z - center| = radius; eigenvalues in [keep_lo, keep_hi) are kept
 * from this contour.  Requires center - radius <= keep_lo < keep_hi <=
 * center + radius (paper Sec. 4.2: circle from an interval with inflation). */
typedef struct {
    double center;
    double radius;
    double keep_lo;
    double keep_hi;
} gep_contour;

typedef struct {
    uint64_t seed;          /* seed of the counter-based Gaussian block V
                               (SplitMix64 + Box-Muller, column-major counters) */
    int precision;          /* GEP_FP64 (default) or GEP_MIXED */
    int max_refine;         /* FEAST-type refinement passes when a kept pair
                               misses tol (default 1) */
    double solve_tol;       /* per-column COCG stop ||r||/||b|| (default 1e-9) */
    int max_iter;           /* COCG iteration cap (default 100000) */
    int check_every;        /* iterations between convergence read-backs (default 16) */
    void* stream;           /* hipStream_t, NULL = default stream */
    int inputs_on_device;   /* 1: gep_csr arrays and rhs are device pointers */
    const double* rhs;      /* optional V, n x block, column-major, host or device;
                               NULL = draw V from seed */
    double mem_limit_bytes; /* device-memory budget for one wave of contours;
                               0 = 85% of free memory */
    int timing;             /* 1: time every kernel class with HIP events */
    int rows_per_block;     /* rows per work-group of the streaming COCG kernels,
                               rounded up to a whole number of row groups
                               (0 = automatic: 16 with 4-row groups, 8 without) */
    int verbose;            /* > 0: progress line on stderr every `verbose` COCG iterations */
    int use_graph;          /* 1 (default): replay each chunk of check_every COCG
                               iterations from a captured HIP graph; 2: also the
                               banded factorisation's launches, captured once per
                               pencil and layout (not with timing) */
    const int* blocks;      /* optional per-contour block sizes (host, each
                               1..block): contour k uses the first blocks[k]
                               columns of V.  One entry per contour; for the
                               batched entry points the problems' entries one
                               after another (sum of n_contours entries).  NULL:
                               every contour uses `block`.  Ignored by
                               gep_ci_solve_smallest. */
    int row_group;          /* rows whose neighbour gathers the COCG kernels share:
                               4 (groups of 4 consecutive rows of one pencil, union
                               of their columns), 1 (plain CSR), 0 (default:
                               4 when that saves at least 20% of the gathers).
                               Results do not depend on it. */
    int solver;             /* shifted solves (z_j B - A) Y = B V: 2 = banded
                               L D L^T of every system (complex symmetric, no
                               pivoting, FP64 residual check and iterative
                               refinement with the factors: up to 3 sweeps
                               with FP64 factors, 12 with FP32 ones; pencils
                               of half bandwidth <= 4096), 1 = batched
                               Jacobi COCG, 0 (default) = banded when every
                               pencil's half bandwidth is <= 4096, else COCG.
                               With precision GEP_MIXED the banded factors
                               are FP32 (the residuals and the solution FP64).
                               3 = multi-shift COCG: for a single pencil (not
                               a batch) whose B is beta I (no off-diagonal
                               entries, constant diagonal, beta != 0; else
                               GEP_EINVAL), each contour's nodes share one
                               Krylov space per right-hand side, iterated on
                               the node nearest the real axis; no
                               preconditioner; FP64 regardless of precision.
                               A column stops when its residual estimate
                               ||r|| / |pi| is <= solve_tol ||B v||. */
    int band_kernels;       /* banded factorisation kernels: 0 (default) =
                               register-panel kernels with lookahead for FP64
                               factors of half bandwidth <= 480 (a panel row
                               per thread of one work-group), wide-band
                               kernels otherwise; 1 = the one-work-group
                               kernels for FP64 factors up to half bandwidth
                               1024 (panels beyond 480 kept in global
                               memory); 2 = wide-band kernels always.  Results
                               agree to rounding. */
    int method;             /* GEP_CIRR (default) or GEP_FEAST */
    int band_group;         /* wide-band kernels: factor at most this many shifted
                               systems at once (0, the default: as many as the
                               device memory holds); each group is factored,
                               solved and refined before the next */
} gep_opts;

typedef struct gep_result gep_result;

/* Fill *opts with the defaults listed above. */
void gep_opts_default(gep_opts* opts);

/* Solve one pencil over n_contours circles (Alg. "Standard CI pipeline").
 * n_nodes: trapezoid nodes per circle N (even, >= 2); only the N/2 nodes in
 * the upper half plane are solved (conjugate symmetry of a real pencil).
 * moments: M >= 1.  block: L >= 1 right-hand sides.  tol: residual
 * threshold ||Ax - lambda Bx||_2 / (||A||_inf ||x||_2) for acceptance.
 * On success *out holds the merged, ascending eigenpairs. */
int gep_ci_solve(const gep_csr* A, const gep_csr* B, const gep_contour* contours,
                 int n_contours, int n_nodes, int moments, int block, double tol,
                 const gep_opts* opts, gep_result** out);

/* Batched solve of n_problems independent pencils (A[p], B[p]) with their
 * own circles contours[p][0..n_contours[p]) and common n_nodes, moments,
 * block and tol.  The shifted systems of every contour of every pencil are
 * iterated together (one set of kernel launches per COCG iteration); pencils
 * of different sizes share the launches through per-tile row ranges.
 * Problem p draws V from seed opts->seed + p (opts->rhs must be NULL).
 * out[p] receives problem p's result (free each with gep_result_free).
 * Returns the worst status over the problems (errors: no result is kept). */
int gep_ci_solve_batch(int n_problems, const gep_csr* A, const gep_csr* B,
                       const gep_contour* const* contours, const int* n_contours, int n_nodes,
                       int moments, int block, double tol, const gep_opts* opts,
                       gep_result** out);

/* Number m of returned eigenpairs and the problem size n. */
int gep_result_count(const gep_result* res, int64_t* m, int64_t* n);

/* Copy results to caller-owned HOST buffers (any may be NULL):
 * evals[m] ascending; evecs n x m column-major, B-normalised, largest-|.|
 * entry positive; resid[m]; contour_id[m]; converged[m] (1 if resid <= tol).
 * The eigenvectors stay in device memory owned by the result until
 * gep_result_free; evecs is filled by a synchronous device-to-host copy
 * (GEP_EDEVICE if it fails). */
int gep_result_copy(const gep_result* res, double* evals, double* evecs, double* resid,
                    int32_t* contour_id, uint8_t* converged);

/* Copy the eigenvectors (n x m column-major, as gep_result_copy) into a
 * caller-owned DEVICE buffer of n * m doubles on the same GPU, for callers
 * that use them there: a device-to-device copy enqueued on `stream` (NULL =
 * the default stream); the call returns without waiting for it, and
 * gep_result_free waits for it before releasing the result's copy.  A result
 * with m = 0 copies nothing.  GEP_EDEVICE if the copy cannot be enqueued. */
int gep_result_copy_evecs_device(const gep_result* res, double* evecs_dev, void* stream);

/* Boundary-proximity check (the paper's robustness safeguards, appendix on
 * mild distribution shifts): filter[m] receives, for each returned pair, the
 * value at its eigenvalue of the rational filter that the N-node trapezoid rule
 * of its contour applies, Re sum_j w_j / (z_j - lambda): 1 at the centre, 1/2
 * on the circle.  Pairs below 0.9 lie in the filter's transition band (the
 * statistics count them as near_boundary_pairs); a caller may enlarge or split
 * such contours.  filter is a caller-owned HOST buffer of m doubles. */
int gep_result_filter(const gep_result* res, double* filter);

/* JSON statistics (iterations, passes, ranks, per-phase times, bytes) into
 * json[cap]; *needed receives the full length including the terminator. */
int gep_result_stats(const gep_result* res, char* json, size_t cap, size_t* needed);

void gep_result_free(gep_result* res);

const char* gep_strerror(int status);
const char* gep_last_error(void);

/* ---- component entry points (kernel-level checks and measurement) -----
 * These expose single steps of the hot path on caller-owned DEVICE buffers.
 * Work is enqueued on `stream` (NULL = default stream) and the stream is
 * synchronised before the call returns.  Errors as above. */

typedef struct gep_pencil gep_pencil;

/* Validate and pack A, B into the device format (union pattern, interleaved
 * (a_ij, b_ij) values, diagonals, ||A||_inf).  Inputs host or device per
 * inputs_on_device. */
int gep_pencil_create(const gep_csr* A, const gep_csr* B, int inputs_on_device, void* stream,
                      gep_pencil** out);
void gep_pencil_free(gep_pencil* p);
/* n, nnz of the packed union pattern, and ||A||_inf. */
int gep_pencil_info(const gep_pencil* p, int64_t* n, int64_t* nnz, double* a_inf);

/* gep_ci_solve on an already packed pencil (same arguments and results);
 * opts->inputs_on_device then only concerns opts->rhs. */
int gep_ci_solve_pencil(gep_pencil* p, const gep_contour* contours, int n_contours, int n_nodes,
                        int moments, int block, double tol, const gep_opts* opts,
                        gep_result** out);

/* Batch form of gep_pencil_create: n_problems independent pencils packed
 * once, device-resident, into one block-diagonal pencil (problem p owns the
 * rows after those of problems 0..p-1).  Inputs host or device per
 * inputs_on_device; errors name the failing problem. */
int gep_pencil_create_batch(int n_problems, const gep_csr* A, const gep_csr* B, int inputs_on_device,
                            void* stream, gep_pencil** out);
/* Number of problems packed in a pencil (1 for gep_pencil_create). */
int gep_pencil_problems(const gep_pencil* p, int* n_problems);

/* gep_ci_solve_batch on a pencil from gep_pencil_create_batch: contours[p],
 * n_contours[p] for each of its problems, results in out[p] (same
 * conventions); the pencil keeps its device workspace between calls.  A
 * pencil of several problems must be solved with this entry point. */
int gep_ci_solve_pencil_batch(gep_pencil* p, const gep_contour* const* contours, const int* n_contours,
                              int n_nodes, int moments, int block, double tol, const gep_opts* opts,
                              gep_result** out);

/* The m smallest eigenpairs with eigenvalue >= lower (the paper's target of
 * the M smallest eigenvalues, Sec. 5 "Experiment Settings"), on a pencil of
 * one problem.  The upper end of the window is not known.  The first window
 * is [lower, lower + (m / n)^2 (lmax - lower)), lmax from a power iteration
 * on diag(B)^-1 A (the count grows no faster than (lambda / lmax)^(1/2) n
 * on 1D-3D grids, so it holds at most about m); while fewer than m pairs are
 * found the covered range is extended by the density found so far, in
 * uniform circles of about per_contour expected eigenvalues (radius 1.1 x
 * half the circle's interval).  A circle whose subspace is saturated or that
 * leaves a kept pair above tol is solved again as three circles (at most
 * four times).  Each round is solved as gep_ci_solve_pencil does.  *out
 * holds the m smallest pairs found (fewer, with GEP_WNOCONV, if the rounds
 * ran out); contour ids count the circles of all rounds; the statistics
 * list each round's.  With equal eigenvalues at the cut, which of their
 * vectors is returned is open. */
int gep_ci_solve_smallest(gep_pencil* p, int64_t m, double lower, int per_contour, int n_nodes,
                          int moments, int block, double tol, const gep_opts* opts, gep_result** out);

/* Shifted complex SpMM, Y[:, c] = z_c B X[:, c] - A X[:, c] (quadrature
 * equation's operator), FP64 complex, on the tiled layout: column c of an
 * n x W multivector lives at element ((c / 64) * n + i) * 64 + c % 64,
 * each element an interleaved (re, im) double pair; W a multiple of 64.
 * shifts: W interleaved complex doubles.  pq (optional, W complex doubles):
 * receives sum_i X[i,c] Y[i,c] (bilinear, no conjugation). */
int gep_spmm_shifted(const gep_pencil* p, const double* shifts, const double* X, double* Y,
                     int64_t W, double* pq, void* stream);

/* The direction step that opens every iteration of the batched COCG solve
 * of the shifted systems (quadrature equation's operator K_c = z_c B - A,
 * Jacobi-preconditioned residual U): Pn[:, c] = U[:, c] + beta_c P[:, c] and
 * pq[c] = sum_i Pn[i, c] (K_c Pn)[i, c] (bilinear, no conjugation); K_c Pn
 * itself is not stored.  Same tiled FP64 complex layout as
 * gep_spmm_shifted; shifts, beta and pq: W interleaved complex doubles;
 * all pointers device.  row_group 4 walks groups of 4 rows sharing their
 * neighbour gathers (the pencil's 4-row form), 1 plain CSR rows: the
 * results agree to rounding.  GEP_EINVAL for other values. */
int gep_cocg_direction(const gep_pencil* p, const double* shifts, const double* beta,
                       const double* U, const double* P, double* Pn, int64_t W, double* pq,
                       int row_group, void* stream);

/* FP32 complex variant of gep_spmm_shifted (shifts stay FP64 complex). */
int gep_spmm_shifted_f32(const gep_pencil* p, const double* shifts, const float* X, float* Y,
                         int64_t W, void* stream);

/* Real multivector products on row-major n x k blocks (leading dim ld >= k):
 * YA = A X and/or YB = B X (either output may be NULL). */
int gep_spmm_real(const gep_pencil* p, const double* X, int64_t k, int64_t ld, double* YA,
                  double* YB, void* stream);

/* G = X^T Y for row-major X (n x k1, ld1) and Y (n x k2, ld2), G row-major
 * k1 x k2, FP64 MFMA with split-K over n.  Deterministic. */
int gep_gram(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n, int64_t k1,
             int64_t k2, double* G, void* stream);

/* gep_gram without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as gep_gram; the split-K
 * partial tiles go to a static device array of the library, 8 Mi doubles
 * (64 MiB) per GPU, held until the process ends.  GEP_EINVAL, with a message,
 * when the partials of (n, k1, k2) need more than that (gep_gram plans
 * splits * k1 * k2 doubles, about 4 Mi for k1, k2 <= 1024 and at most
 * k1 * k2 beyond).  All calls on one GPU share the array: calls that overlap
 * on one GPU (other streams or threads) race and must be serialised by the
 * caller.  The stream is synchronised before the call returns. */
int gep_gram_noalloc(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n,
                     int64_t k1, int64_t k2, double* G, void* stream);

/* C = X T for row-major X (n x k, ldx), T (k x m, row-major, ldt), C (n x m, ldc);
 * FP64 MFMA. */
int gep_gemm_tall(const double* X, int64_t ldx, const double* T, int64_t ldt, int64_t n, int64_t k,
                  int64_t m, double* C, int64_t ldc, void* stream);

/* Symmetric eigen-decomposition of `batch` k x k row-major matrices, k <= 1024
 * (two-sided block Jacobi: 32-index blocks paired round robin, each 64 x 64
 * subproblem diagonalised in LDS, the rotations applied to the block rows and
 * columns as small products): eigenvalues ascending into w[batch*k],
 * orthonormal eigenvectors as columns of V[batch*k*k] (row-major).  A is
 * overwritten; a device work area is allocated per call; the stream is
 * synchronised once per sweep.  GEP_EINVAL for bad sizes. */
int gep_sym_eig(double* A, double* w, double* V, int64_t k, int batch, void* stream);

/* Counter-based Gaussian block (the V of the solve): row-major n x L with
 * V[i*L + l] = entry at counter l*n + i of the SplitMix64 + Box-Muller
 * stream of `seed`. */
int gep_gaussian_block(uint64_t seed, int64_t n, int64_t L, double* V, void* stream);

/* ---- learned contours (spectral prior + KDE) ----------------------------
 * KDE contour construction (paper Sec. 4.2, interval sparsity function and
 * Alg. "Adaptive Contour Construction via KDE"): recursively split the
 * initial interval at the minimiser of G_k(t) = sum_j exp(-w (t - lam_j)^2 /
 * (e - s)^2) over midpoints between consecutive predicted eigenvalues until
 * every interval holds <= nmax of them, merge intervals holding < nmin with
 * the smaller neighbour (splitting again above nmax), and map [s, e) to the
 * circle centre (s+e)/2, radius (1+alpha)(e-s)/2.  The initial interval is
 * [window_lo, window_hi] when both are finite, else [min - eps, max + eps],
 * eps = beta (max - min).  lam_hat: host array of m predictions.  *count
 * receives the number of contours; out (host, cap entries) may be NULL to
 * query it.  Host computation; no GPU work. */
int gep_kde_contours(const double* lam_hat, int64_t m, int nmin, int nmax, double w, double alpha,
                     double beta, double window_lo, double window_hi, gep_contour* out, int cap,
                     int* count);

/* Input of the spectral-density network (paper Sec. 4.1: the predictor
 * reads the discretised coefficient field): block averages of a row-major
 * FP32 field g[nz][ny][nx] (DEVICE) onto a side^3 grid (side^2 when nz == 1)
 * written to out (DEVICE, cells ordered [z][y][x]).  Cell c along an axis of
 * n entries averages the entries a with floor(a side / n) == c.  Requires
 * side <= each dimension (> 1).  The stream is synchronised. */
int gep_field_downsample(const float* g, int nz, int ny, int nx, int side, float* out, void* stream);

/* Spectral-density network: 3-layer MLP din -> dhidden -> dhidden -> dout,
 * GELU, BF16 matrix-core GEMMs with FP32 accumulation, FP32 master weights
 * and Adam state (paper Sec. 4.1: the learned spectral predictor, trained
 * with a mean squared error).  Device pointers; rows of X are samples
 * (row-major B x din, FP32); max_batch bounds B.  Weights: Glorot-uniform
 * from SplitMix64(seed). */
typedef struct gep_density gep_density;
int gep_density_create(int din, int dhidden, int dout, int max_batch, uint64_t seed,
                       gep_density** out);
void gep_density_free(gep_density* net);
/* Y (device, B x dout FP32) = net(X). */
int gep_density_forward(gep_density* net, const float* X, int B, float* Y, void* stream);
/* Forward, loss = mean((Y - T)^2) over B x dout (T device FP32), and the
 * gradients of all parameters (kept in the net).  *loss (host) if non-NULL. */
int gep_density_grads(gep_density* net, const float* X, const float* T, int B, double* loss,
                      void* stream);
/* One Adam step (Kingma and Ba) with the stored gradients. */
int gep_density_adam(gep_density* net, float lr, float beta1, float beta2, float eps, void* stream);
/* Copy parameter tensor `which` (0: W1 din x dh, 1: b1, 2: W2, 3: b2, 4: W3 dh x dout,
 * 5: b3; row-major) or its gradient (grad = 1) to (set = 0) or from (set = 1)
 * a HOST buffer. */
int gep_density_param(gep_density* net, int which, int grad, float* host, int set);
/* C = op(A) op(B) on BF16 matrix cores, FP32 accumulation (the network's
 * GEMM): A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] as raw BF16
 * bit patterns, C row-major M x N FP32 with ldc.  Device pointers. */
int gep_gemm_bf16(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                  int64_t sbn, float* C, int64_t ldc, int M, int N, int K, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GEP_CI_H */
