// Internal declarations shared by the host orchestrator and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace gep {

// One wavefront covers 64 columns of a multivector tile.
constexpr int kTile = 64;
// Work-group size of the streaming kernels: 4 wavefronts (one row group per
// wave in the COCG kernels; 8-wave work-groups measured slower).
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kTile;

void set_error(const std::string& msg);

// Device-resident packed pencil: union CSR pattern with interleaved (a, b).
struct DevPencil {
    int64_t n = 0, nnz = 0;
    int32_t* rowptr = nullptr;  // n + 1
    int32_t* colind = nullptr;  // nnz
    double2* ab = nullptr;      // nnz (a_ij, b_ij)
    float2* ab32 = nullptr;     // nnz FP32 copy (mixed precision)
    double* dA = nullptr;       // diag(A)
    double* dB = nullptr;       // diag(B)
    double a_inf = 0.0;         // max absolute row sum of A
    int max_row_nnz = 0;
    // Row-group form used by the COCG kernels (cocg.hip, group_walk): groups of
    // `grp` consecutive rows of one pencil of a batch, the sorted union of
    // their columns and an grp-wide coefficient block per union column.
    // grp == 1 aliases the CSR arrays.
    // The packed pencil holds the 4-row form; `grp`, gptr, gcol, gab and
    // gab32 are the view a solve uses (set per solve; grp == 1 is the CSR).
    int grp = 1;
    int32_t* gptr = nullptr;    // groups + 1
    int32_t* gcol = nullptr;    // union columns
    double2* gab = nullptr;     // union columns * grp (a, b); zero where a row has no entry
    float2* gab32 = nullptr;    // FP32 copy
    int32_t* g4ptr = nullptr;
    int32_t* g4col = nullptr;
    double2* g4ab = nullptr;
    float2* g4ab32 = nullptr;
    int64_t g4nnz = 0;          // union columns of the 4-row form
    int auto_grp = 1;           // 4 when the 4-row form saves at least 20% of the gathers
    // real lower bands (a_ij, b_ij) of the problems whose half bandwidth is at
    // most kBandMaxBw (band.hip); offsets and widths are kept on the host
    double2* band = nullptr;
};

// XCD-aware remap of a flat work-group id: the hardware deals work-groups
// round-robin over the 8 XCDs; this gives each XCD a contiguous range of
// logical ids so neighbouring rows of one column tile share an L2.
__device__ inline int xcd_logical(int b, int grid) {
    const int per = grid >> 3;   // grid is always padded to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

inline int pad8(int g) { return (g + 7) & ~7; }

// ---- launchers (all enqueue on `s`, return hipError_t) -------------------
// complex FP64 shifted SpMM over active tiles (tiled layout), optional
// bilinear dot partials [tile][nrb][64].
hipError_t launch_spmm_c64(const DevPencil& P, const double2* shifts, const double2* X,
                           double2* Y, const int32_t* tiles, const int32_t* n_active,
                           int n_active_host, int nrb, double2* partial, hipStream_t s);
hipError_t launch_spmm_c32(const DevPencil& P, const double2* shifts, const float2* X, float2* Y,
                           const int32_t* tiles, const int32_t* n_active, int n_active_host,
                           int nrb, double2* partial, hipStream_t s);
// rows [row0, row0 + nloc) of the (concatenated) pencil; nloc < 0 means all n.
hipError_t launch_spmm_real(const DevPencil& P, const double* X, int64_t k, int64_t ld,
                            double* YA, double* YB, hipStream_t s, int64_t row0 = 0,
                            int64_t nloc = -1);

// Geometry of the tiles of a multivector that may span several pencils of a
// batch: tile t holds rows [row0[t], row0[t] + n[t]) of the concatenated
// pencil, element (i, lane) at base[t] + i * 64 + lane.
struct TileGeom {
    const int64_t* base = nullptr;
    const int32_t* n = nullptr;
    const int32_t* row0 = nullptr;
    const int32_t* g0 = nullptr;   // row-group index of the tile's row 0
};

// COCG state (cocg.hip).  FP64 path: x, u, p, pn.  Mixed path: x (FP64
// solution), x32, u32, p32, pn32 (FP32 recurrence).
struct CocgState {
    int64_t n = 0;
    int ntiles = 0;              // W / 64
    double2* x = nullptr;        // tiled n x W
    double2* u = nullptr;        // preconditioned residual D^-1 r
    double2* p = nullptr;        // search direction (read)
    double2* pn = nullptr;       // search direction (written)
    float2* x32 = nullptr;
    float2* u32 = nullptr;
    float2* p32 = nullptr;
    float2* pn32 = nullptr;
    double2* shifts = nullptr;   // [W]
    int64_t* bsrc = nullptr;     // [W] offset in B V of column c's right-hand side at its
                                 // pencil's row 0 (rows stride ldbv); -1: none
    double2* rho = nullptr;      // [W]
    double2* alpha = nullptr;    // [W]
    double2* beta = nullptr;     // [W]
    double* bb = nullptr;        // [W] ||b||^2
    double* rr = nullptr;        // [W] ||r||^2
    double* rmax = nullptr;      // [W] mixed: max recursive ||r||^2 since the last replacement
    int32_t* flag = nullptr;     // [W] mixed: replace this column's residual at the next check
    double* rbest = nullptr;     // [W] mixed: smallest true ||r||^2 seen at a replacement
    int32_t* stall = nullptr;    // [W] mixed: replacements since rbest last fell 4x
    int32_t* stalled = nullptr;  // [W] mixed: FP32 recurrence gave up; finish in FP64
    int32_t* active = nullptr;   // [W]
    int32_t* iters = nullptr;    // [W]
    int32_t* tile_active = nullptr;  // [ntiles] active columns per tile
    int32_t* tiles = nullptr;        // [ntiles] compacted active list
    int32_t* counts = nullptr;       // [2]: active tiles, active columns
    double2* part_c = nullptr;       // [ntiles][nrb][64]
    double* part_r = nullptr;        // [ntiles][nrb][64]
    int nrb = 0;
    int rpb = 0;                     // rows per work-group
    int G = 0;                       // first-level groups of the partial sums (0: none)
    double2* part2_c = nullptr;      // [ntiles][G][64]
    double* part2_r = nullptr;
    TileGeom geom;
};

hipError_t cocg_init(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv, int nrb,
                     hipStream_t s);
hipError_t cocg_spmm_dir(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                         hipStream_t s);
hipError_t cocg_update(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                       hipStream_t s);
hipError_t cocg_reduce_alpha(CocgState& S, int n_active_host, int nrb, hipStream_t s);
hipError_t cocg_reduce_beta(CocgState& S, int n_active_host, int nrb, double tol2, int max_iter,
                            int hold, hipStream_t s);
hipError_t cocg_compact(CocgState& S, hipStream_t s);
hipError_t cocg32_init(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv, int nrb,
                       hipStream_t s);
hipError_t cocg32_spmm_dir(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                           hipStream_t s);
hipError_t cocg32_update(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                         hipStream_t s);
// FP64 completion of the columns the FP32 recurrence gave up on: r = b - K x
// in FP64, u = D^-1 r, p = 0, beta = 0; those columns become the active set
// of an FP64 COCG run that continues from x.  u, p and pn must be zero.
hipError_t cocg64_restart(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv,
                          int nrb, double tol2, hipStream_t s);
hipError_t cocg32_fold(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                       hipStream_t s);
hipError_t cocg32_replace(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv,
                          int n_active_host, int nrb, double tol2, hipStream_t s);

// moments: S_k[i][m*L + l] = sum_j Re(coef[k][j][m] * x[coff[k] + j*L + l][i]) for
// i < cn[k]; S_k starts at S + soff[k]; nmax = max cn.
hipError_t launch_moments(const double2* X, const TileGeom& g, int64_t nmax, int K, int NH, int L,
                          int M, const int64_t* coff, const int32_t* cn, const int64_t* soff,
                          const double2* coef, double* S, hipStream_t s);

// ---- banded direct solves (band.hip) ----------------------------------
// One shifted system z B - A of one pencil of the batch, stored as a
// column-major lower band: entry (i, j), 0 <= i - j <= bw, at
// off + j * (bw + 1) + (i - j).
struct BandSys {
    int64_t off = 0;    // element offset of the system's band in the factor array
    int64_t aoff = 0;   // element offset of its pencil's real (a, b) band (-1: none kept)
    int32_t n = 0, bw = 0;
    double2 z{0.0, 0.0};
    int32_t row0 = 0;   // first row of its pencil in the concatenated CSR
    int32_t pad = 0;
};
// Up to 16 consecutive columns of one band system inside one tile of a
// multivector (the unit of the wide-band solves).
struct WbChunk {
    int32_t sys = 0, tile = 0, lane0 = 0, cnt = 0;
};

// Panel width of the banded factorisation (every step re-reads and re-writes
// the trailing bw x bw window, so wider panels cut that traffic) and the LDS
// budget of the generic solves.
constexpr int kPanel = 32;
// Widest half bandwidth for which a pencil's band is kept (the automatic
// solver choice takes the band path up to kBandAutoBw).
constexpr int64_t kBandMaxBw = 4096;
constexpr int64_t kBandAutoBw = 1024;
// Iterative-refinement sweeps after a banded solve at most.
constexpr int kBandRefineMax = 3;
// ... and with FP32 factors (each sweep gains about cond(K) * 6e-8).
constexpr int kBandRefineMax32 = 12;
constexpr size_t kBandLds = 64 * 1024;

hipError_t band_form(const BandSys* sys, int nsys, const double2* AB, double2* F, hipStream_t s);
// One panel step: factor panel [k0, k0 + kPanel) (flag: zero or non-finite
// pivot per system), then update the trailing window.
// e0, e1 (optional, timing events): attached to the kernel's dispatch
// (start and end of its execution).
hipError_t band_panel(const BandSys* sys, int nsys, int bwmax, double2* F, int k0, int32_t* flag,
                      hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// part 0: the whole trailing window; 1: only the next panel's columns
// [k0 + kPanel, k0 + 2 kPanel), with the contributions of panel k0 and of
// panel k0 - kPanel; 2: the window from k0 + 3 kPanel on (panel k0 only).
hipError_t band_update(const BandSys* sys, int nsys, int bwmax, double2* F, int k0, int part,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Columns per work-group of the solves for a half bandwidth bw.
int band_chunk_columns(int bw);
// In place: X <- K^-1 X for every column (colsys: system of each tiled column,
// -1 = none).  chunk = 8 or 16 when every aligned chunk of that many columns
// belongs to one system (register-window sweeps), else 0.
hipError_t band_solve(const BandSys* sys, const int32_t* colsys, const double2* F,
                      const TileGeom& g, int ntiles, int bwmax, double2* X, hipStream_t s,
                      int chunk);
// Multi-shift COCG (multishift.hip).  Seed vectors: nseed_tiles tiles of
// 64 columns over n rows.  Seed residual update with the partials of r^T r
// and ||r||^2 per seed tile, row block (nrb blocks) and column; the shifted
// columns' solution and search-vector update (coef[3 c + 0..2] = alpha_c,
// beta_c, 1 / pi_c; col_l[c] = seed column, -1 for padding); the seed search
// vector p_s = r + beta p_s.
hipError_t ms_seed_update(int n, int nseed_tiles, int nrb, const double2* alpha, const double2* q, double2* r,
                          double2* part_rho, double* part_nrm, hipStream_t s);
hipError_t ms_shift_update(const TileGeom& g, int ntiles, int64_t nmax, int n_seed, const int32_t* col_l,
                           const int32_t* active, const double2* coef, const double2* r, double2* X, double2* P,
                           hipStream_t s);
hipError_t ms_seed_p(int n, int nseed_tiles, const double2* beta, const double2* r, double2* ps, hipStream_t s);
hipError_t band_rhs(const TileGeom& g, const int64_t* bsrc, const double* BV, int64_t ldbv,
                    int ntiles, double2* X, hipStream_t s);
// R = b - K X, rel[col] = ||R|| / ||b||; part holds ntiles * nrb_cap * 64 entries.
hipError_t band_residual(const DevPencil& P, const TileGeom& g, const double2* shifts,
                         const int64_t* bsrc, const double* BV, int64_t ldbv, const double2* X,
                         double2* R, int ntiles, int64_t nmax, double2* part, int nrb_cap,
                         double* rel, hipStream_t s);
hipError_t band_axpy(const TileGeom& g, const double2* R, int ntiles, double2* X, hipStream_t s);

// ---- wide-band and FP32 factors (band_wide.hip) ---------------------------
// Half bandwidth from which the wide-band kernels factor a system (below it
// the register-panel kernels of band.hip, FP64 only, are used).
constexpr int64_t kBandWideBw = 1024;
// F (factor array of `fp32 ? float2 : double2`) = z B - A from the CSR rows;
// F must be zero beforehand.
hipError_t wb_form(const DevPencil& P, const BandSys* sys, int nsys, void* F, bool fp32, hipStream_t s);
// One step of two panels: [k0, k0 + 2 kPanel) and the trailing window.
hipError_t wb_step(const BandSys* sys, int nsys, int bwmax, void* F, bool fp32, int k0, int nmax,
                   int32_t* flag, hipStream_t s);
// In place X <- K^-1 X on the chunks' columns (X of the factor's type);
// nmax: the largest system size; Dfar: wb_scratch_bytes(nchunks) of scratch.
hipError_t wb_solve(const BandSys* sys, const WbChunk* chunks, int nchunks, const void* F, bool fp32,
                    const TileGeom& g, void* X, int nmax, void* Dfar, hipStream_t s);
size_t wb_scratch_bytes(int nchunks);
// D (FP32) = S (FP64) on the chunks' columns.
hipError_t wb_narrow(const BandSys* sys, const WbChunk* chunks, int nchunks, const TileGeom& g,
                     const double2* S, float2* D, hipStream_t s);
// X += D (set: X = D) on the chunks' columns; D FP32 or FP64.
hipError_t wb_accumulate(const BandSys* sys, const WbChunk* chunks, int nchunks, const TileGeom& g,
                         const void* D, bool fp32, double2* X, int set, hipStream_t s);

// RNG
hipError_t launch_gaussian(uint64_t seed, int64_t n, int64_t L, double* V, hipStream_t s);

// dense (gemm.hip / dense.hip)
hipError_t launch_gram(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n,
                       int64_t k1, int64_t k2, double* G, double* work, size_t work_elems,
                       hipStream_t s);
size_t gram_work_elems(int64_t n, int64_t k1, int64_t k2);
// Allocation-free Gram: device address of the library's static partial-tile
// array on the current device, and its size in doubles.
hipError_t gram_scratch(double** ptr);
size_t gram_scratch_elems();
hipError_t launch_gemm_tall(const double* X, int64_t ldx, const double* T, int64_t ldt, int64_t n,
                            int64_t k, int64_t m, double* C, int64_t ldc, hipStream_t s);
// Batched symmetric eigensolver; matrix b is ks[b] x ks[b] (row-major, leading
// dimension ks[b]) at offset b * kmax^2; ks == NULL means all kmax.
// work holds sym_eig_work_elems(kmax, batch) doubles.  Synchronises the
// stream once per Jacobi sweep (convergence test on the host).
hipError_t launch_sym_eig(double* A, double* w, double* V, int64_t kmax, int batch,
                          const int32_t* ks, double* work, hipStream_t s);
size_t sym_eig_work_elems(int64_t kmax, int batch);
// Cholesky of SPD matrices (same batching); writes L^-T (upper) into LinvT;
// status[b] = 0 ok, j+1 if pivot j failed.
hipError_t launch_chol_inv(const double* G, double* LinvT, int64_t kmax, int batch,
                           const int32_t* ks, double* work, int32_t* status, hipStream_t s);
// C = op(A) op(B) for k x k row-major small matrices (ta/tb transpose flags).
hipError_t launch_small_gemm(const double* A, int ta, const double* B, int tb, double* C,
                             int64_t m, int64_t n, int64_t kk, int64_t lda, int64_t ldb,
                             int64_t ldc, hipStream_t s);
hipError_t launch_symmetrise(double* A, int64_t k, hipStream_t s);
// SVQB scaling: T[i][j] = U[i][k-r+j] / sqrt(w[k-r+j]), i < k, j < r
hipError_t launch_svqb_scale(const double* U, const double* w, int64_t k, int64_t r, double* T,
                             hipStream_t s);
// residual norms for row-major n x k blocks: num[j] = ||AX_j - th_j BX_j||, den[j] = ||X_j||
hipError_t launch_resid_norms(const double* AX, const double* BX, const double* X,
                              const double* theta, int64_t n, int64_t k, double* num, double* den,
                              double* work, hipStream_t s);
// gather selected columns of row-major X (n x k) into column-major out (n x m),
// sign-normalised (largest-|.| entry positive, lowest index on ties); work
// holds gather_cols_work(n, m) doubles
size_t gather_cols_work(int64_t n, int m);
hipError_t launch_gather_cols(const double* X, int64_t n, int64_t k, const int32_t* sel, int m,
                              double* out, double* work, hipStream_t s);

}  // namespace gep
