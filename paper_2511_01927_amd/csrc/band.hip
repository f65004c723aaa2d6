// Banded direct solves of the shifted systems (z B - A) Y = B V of the
// quadrature equation (paper Appendix, "Numerical Quadrature": the N_q
// shifted solves are the dominant cost and independent).  The paper leaves
// the linear solver open; for pencils whose (union) pattern lies within a
// band of half width bw -- 2D grids in natural order have bw ~ sqrt(n) --
// every shifted system is factored as K = L D L^T (complex symmetric, L unit
// lower, D diagonal, no pivoting) and solved for all right-hand sides.
//
// Storage: column-major lower band.  Entry (i, j), 0 <= i - j <= bw, of one
// system lives at off + j * (bw + 1) + (i - j); entries past row n are zero.
// After the factorisation the same slots hold d_j (i = j) and l_ij (i > j).
//
// Factorisation, right-looking by panels of kPanel columns, one step per
// panel (all systems of a batch advance together):
//   k_band_panel_rows  one work-group per system, one thread per panel row
//                  (kPanel + bw <= 512): unblocked L D L^T of the panel's
//                  kPanel columns with each row's entries in registers
//                  (k_band_panel: wider bands, when asked for, the panel
//                  in global memory);
//   k_band_strip   the next panel's columns take the contributions of this
//                  panel and the one before (critical path of the step);
//   k_band_update  the rest of the trailing window, from the panel after
//                  next on: C -= W diag(d) W^T, lower triangle, 64 x 64
//                  tiles staged through LDS, products on the FP64 matrix
//                  cores; it runs on a second stream beside the next two
//                  panel steps (lookahead).
// Solves, in place on the tiled multivector (element (i, c) at
// (tile * n + i) * 64 + lane), a work-group per (tile, chunk of columns):
//   k_band_fwd_pipe / k_band_bwd_pipe  32-row blocks: a triangular
//                    solve of the block's rows (readlane broadcasts) and
//                    the block's coupling to the next (previous) bw rows as
//                    v_mfma_f64_16x16x4 products, in two wave roles so that
//                    the products of one block overlap the solve of the
//                    next, pending rows in an LDS ring; used for 16-column
//                    chunks and bw <= 384;
//   k_band_sweep     row-by-row sweeps with the window in registers (one
//                    half wavefront per column), for 8-column chunks or
//                    wider bands;
//   k_band_forward / k_band_backward  the same with an LDS window, for the
//                    remaining cases.
// Unpivoted elimination is safe here in practice (growth ~1 measured on the
// shifted Q1 systems); every solve is followed by an FP64 residual check and
// iterative refinement with the same factors, and a zero or non-finite pivot
// is flagged per system.
#include <hip/hip_ext.h>

#include "internal.h"

namespace gep {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a -= b * c
__device__ inline void cfms(double2& a, double2 b, double2 c) {
    a.x = fma(-b.x, c.x, fma(b.y, c.y, a.x));
    a.y = fma(-b.x, c.y, fma(-b.y, c.x, a.y));
}

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// Value of v in lane l (wave-uniform l) of the wavefront, through SGPRs.
__device__ inline double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double2 readlane2(double2 v, int l) { return make_double2(readlane_d(v.x, l), readlane_d(v.y, l)); }

constexpr int band_threads_per_column(int cw) { return 256 / cw > 64 ? 64 : 256 / cw; }

}  // namespace

// F = z B - A on the band of each system.  Work-group row blockIdx.y takes
// systems y, y + gridDim.y, ...; consecutive systems of a pass share their
// pencil, so each (a, b) pair is read once for all of them when they do
// (aoff equal), and F is written with non-temporal stores (the factorisation
// reaches most of it long after).
__global__ __launch_bounds__(256) void k_band_form(const BandSys* __restrict__ sys, int nsys,
                                                   const double2* __restrict__ AB,
                                                   double2* __restrict__ F) {
    for (int y = blockIdx.y; y < nsys;) {
        const BandSys S = sys[y];
        const int64_t total = (int64_t)S.n * (S.bw + 1);
        // the run of systems after y (stride gridDim.y) on the same pencil band
        int yend = y + gridDim.y;
        while (yend < nsys && sys[yend].aoff == S.aoff && sys[yend].n == S.n && sys[yend].bw == S.bw)
            yend += gridDim.y;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
             e += (int64_t)gridDim.x * blockDim.x) {
            const double2 v = AB[S.aoff + e];
            for (int q = y; q < yend; q += gridDim.y) {
                const BandSys Q = sys[q];
                __builtin_nontemporal_store(Q.z.x * v.y - v.x, &F[Q.off + e].x);
                __builtin_nontemporal_store(Q.z.y * v.y, &F[Q.off + e].y);
            }
        }
        y = yend;
    }
}

// Unblocked L D L^T of panel columns [k0, k0 + kPanel) of every system.
__global__ __launch_bounds__(256) void k_band_panel(const BandSys* __restrict__ sys,
                                                    double2* F, int k0,
                                                    int32_t* __restrict__ flag) {
    const BandSys S = sys[blockIdx.x];
    if (k0 >= S.n) return;
    const int ld = S.bw + 1;
    const int ncols = min(kPanel, S.n - k0);
    // P and col address the same band (different columns are read and written)
    double2* P = F + S.off + (int64_t)k0 * ld;
    for (int jj = 0; jj < ncols; ++jj) {
        double2* col = P + (int64_t)jj * ld;
        const int j = k0 + jj;
        const int emax = min(S.bw, S.n - 1 - j);   // rows j+1 .. j+emax
        const double2 d = col[0];
        const double m2 = d.x * d.x + d.y * d.y;
        if (!(m2 > 0.0) || !isfinite(m2)) {
            if (threadIdx.x == 0) flag[blockIdx.x] = 1;
        }
        const double2 inv = make_double2(d.x / m2, -d.y / m2);
        for (int e = 1 + (int)threadIdx.x; e <= emax; e += blockDim.x) col[e] = cmul(col[e], inv);
        __syncthreads();
        // columns j + t (t = 1 .. ncols-1-jj) of the panel: rows j+t+e2 <= j+emax
        const int left = min(ncols - 1 - jj, emax);
        const int work = left * ld;
        for (int w = threadIdx.x; w < work; w += blockDim.x) {
            const int t = 1 + w / ld;
            const int e2 = w - (t - 1) * ld;
            if (e2 > emax - t) continue;
            const double2 f = cmul(d, col[t]);
            cfms(P[(int64_t)(jj + t) * ld + e2], col[t + e2], f);
        }
        __syncthreads();
    }
}

// Panel factorisation with one thread per row: thread t holds row k0 + t of
// the panel (its kPanel entries, column c at slot c - k0) in registers; the
// panel's rows are k0 .. k0 + ncols - 1 + bw, so NT >= kPanel + bw.  For
// column j the rows k0 .. k0 + ncols - 1 publish a_kj (the diagonal one also
// 1 / d_j) in LDS; every row i in (j, j + bw] then forms l_ij = a_ij / d_j
// and a_ik -= l_ij a_kj for the later panel columns k, column j + 1 first so
// that column can be published before the others are updated.  Slots above
// the diagonal or past the last column may collect garbage: they are never
// published, used or stored.  One barrier per column (double-buffered LDS).
template <int NT>
__global__ __launch_bounds__(NT) void k_band_panel_rows(const BandSys* __restrict__ sys, double2* F,
                                                        int k0, int32_t* __restrict__ flag) {
    __shared__ double2 cb[2][kPanel + 1];
    const BandSys S = sys[blockIdx.x];
    if (k0 >= S.n) return;
    const int ld = S.bw + 1;
    const int ncols = min(kPanel, S.n - k0);
    const int t = threadIdx.x;
    const int i = k0 + t;
    const bool row_ok = t < ncols + S.bw && i < S.n;
    double2* Fs = F + S.off;
    double2 a[kPanel];
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const bool ok = row_ok && k < ncols && t >= k && t - k <= S.bw;
        a[k] = ok ? Fs[(int64_t)(k0 + k) * ld + (t - k)] : make_double2(0.0, 0.0);
    }
    // rows k0 .. k0 + ncols - 1 publish column jj (slot jj) and the pivot
    // row its inverse
    auto publish = [&](double2* c, int jj, double2 v) {
        if (t >= jj && t < ncols) c[t] = v;
        if (t == jj) {
            const double m2 = v.x * v.x + v.y * v.y;
            if (!(m2 > 0.0) || !isfinite(m2)) flag[blockIdx.x] = 1;
            c[kPanel] = make_double2(v.x / m2, -v.y / m2);
        }
    };
    publish(cb[0], 0, a[0]);
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kPanel; ++jj) {
        if (jj < ncols) {   // uniform
            const double2* c = cb[jj & 1];
            const int jn = jj + 1 < kPanel ? jj + 1 : jj;
            const bool upd = row_ok && t > jj && t - jj <= S.bw;
            double2 l = make_double2(0.0, 0.0);
            if (upd) {
                l = cmul(a[jj], c[kPanel]);
                a[jj] = l;
                if (jj + 1 < kPanel) cfms(a[jn], l, c[jn]);
            }
            // column jj + 1 is final now: publish it (its pivot's division
            // overlaps the rest of this column's updates)
            if (jj + 1 < ncols) publish(cb[(jj + 1) & 1], jj + 1, a[jn]);
            if (upd) {
#pragma unroll
                for (int kb = jj + 2; kb < kPanel; kb += 8) {
                    double2 cc[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (kb + q < kPanel) cc[q] = c[kb + q];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (kb + q < kPanel) cfms(a[kb + q], l, cc[q]);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const bool ok = row_ok && k < ncols && t >= k && t - k <= S.bw;
        if (ok) Fs[(int64_t)(k0 + k) * ld + (t - k)] = a[k];
    }
}

// Trailing update after panel [k0, k0 + kPanel) on the window
// [k0 + kPanel, wend), wend = min(n, k0 + kPanel + bw), lower triangle,
// restricted to columns [c0, c1) (rows [c0, wend)): C -= W_i diag(d) W_j^T
// over the lower-triangular set of 64 x 64 tiles (bi >= bj) from (c0, c0),
// ntile tiles per system.  FP64 matrix cores: wave w owns the tile's 16-column
// block w and all four 16-row blocks; per 4-deep K step one A operand
// (l_jk d_k, from registers) serves four complex products (four
// v_mfma_f64_16x16x4 each), formed transposed so that the read-modify-write
// of C is coalesced.  Operand layouts (lane l): A(i, k) at i = l % 16,
// k = l / 16; B(k, j) at k = l / 16, j = l % 16; result register v is
// D(l / 16 + 4 v, l % 16).  Only the row operand W_i (shared by the four
// waves) is staged in LDS; each wave reads its own column operand straight
// into registers, so that four work-groups fit a CU and the launch one round
// of the chip.  Work-group order as in k_band_strip: the
// tiles of system s run on XCD s mod 8 and share its L2.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_band_update(const BandSys* __restrict__ sys, int nsys, int ntile, double2* F, int k0, int c0, int c1) {
    __shared__ double2 Wi[64][kPanel + 1];
    __shared__ double2 dsh[kPanel];
    const int g = blockIdx.x, r = g >> 3;
    const int si = (g & 7) + 8 * (r / ntile), x = r % ntile;
    if (si >= nsys) return;   // uniform over the work-group
    const BandSys S = sys[si];
    const int wend = min(S.n, k0 + kPanel + S.bw);
    const int cend = min(c1, wend);
    if (c0 >= cend) return;
    int bi = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= x) ++bi;
    while (bi * (bi + 1) / 2 > x) --bi;
    const int bj = x - bi * (bi + 1) / 2;
    const int i0 = c0 + 64 * bi, j0 = c0 + 64 * bj;
    if (i0 >= wend || j0 >= cend) return;
    const int ld = S.bw + 1;
    double2* Fs = F + S.off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < kPanel) dsh[threadIdx.x] = k0 + threadIdx.x < S.n ? Fs[(int64_t)(k0 + threadIdx.x) * ld] : make_double2(0.0, 0.0);
    for (int idx = threadIdx.x; idx < 64 * kPanel; idx += blockDim.x) {
        const int rr = idx & 63, kk = idx >> 6;   // lanes run down a band column
        const int k = k0 + kk, i = i0 + rr;
        Wi[rr][kk] = i < wend && i - k <= S.bw ? Fs[(int64_t)k * ld + (i - k)] : make_double2(0.0, 0.0);
    }
    // A(j, k) = l_jk for this wave's 16 columns j; every row here lies below
    // the panel (j >= c0 > k), so only the band limits the entries read
    const int jr = j0 + 16 * wave + (lane & 15);
    double2 wj[kPanel / 4];
#pragma unroll
    for (int q = 0; q < kPanel / 4; ++q) {
        const int k = k0 + 4 * q + (lane >> 4);
        wj[q] = jr < cend && jr - k <= S.bw ? Fs[(int64_t)k * ld + (jr - k)] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    mfma_f64x4 pre[4], pim[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        pre[rb] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
        pim[rb] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < kPanel / 4; ++q) {
        const int kk = 4 * q + (lane >> 4);
        const double2 a = cmul(wj[q], dsh[kk]);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const double2 b = Wi[rb * 16 + (lane & 15)][kk];
            // P^T += W_j W_i^T (complex): re = a.x b.x - a.y b.y, im = a.x b.y + a.y b.x
            pre[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, pre[rb], 0, 0, 0);
            pre[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, pre[rb], 0, 0, 0);
            pim[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, pim[rb], 0, 0, 0);
            pim[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, pim[rb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + 16 * wave + (lane >> 4) + 4 * v;
            const int i = i0 + rb * 16 + (lane & 15);
            if (j >= cend || i >= wend || i < j) continue;
            double2& c = Fs[(int64_t)j * ld + (i - j)];
            c.x -= pre[rb][v];
            c.y -= pim[rb][v];
        }
}

// Strip update of the next panel's columns [w0, w0 + kPanel), w0 = k0 +
// kPanel, with the contributions of panel k0 and (npan = 2) of the panel
// before it: C[i, j] -= sum_k l_ik d_k l_jk for rows [w0, wend) in 32-row
// tiles.  Short and on the critical path of the factorisation, so every
// load is issued at once and the work fits one round of the chip: wave w
// takes the 16 x 16 output sub-tile (w & 1, w >> 1) of its tile over both
// panels (K = 64), reads its operands straight from the band into
// registers, and forms D(j, i) = sum_k (l_jk d_k) l_ik
// on v_mfma_f64_16x16x4 (a complex product is four real ones), so that each
// lane's outputs run down a column and the update of C is coalesced.
// Work-group order: work-group g runs on XCD g mod 8, and the tiles of
// system s take the work-groups of XCD s mod 8, so the tiles of a system
// share the L2 that holds its panel rows l_jk (read by every tile).
// (Three waves per SIMD: 640 work-groups of the 300-wide band fit at once.)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_band_strip(const BandSys* __restrict__ sys, int nsys, int ntile, double2* F, int k0, int npan) {
    __shared__ double2 dsh[2][kPanel];
    const int g = blockIdx.x, r = g >> 3;
    const int si = (g & 7) + 8 * (r / ntile), tile = r % ntile;
    if (si >= nsys) return;   // uniform over the work-group
    const BandSys S = sys[si];
    const int w0 = k0 + kPanel;
    const int wend = min(S.n, k0 + kPanel + S.bw);
    const int cend = min(w0 + kPanel, wend);
    const int i0 = w0 + 32 * tile;
    if (w0 >= cend || i0 >= wend) return;   // uniform over the work-group
    const int ld = S.bw + 1;
    double2* Fs = F + S.off;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int rw = wave & 1, cw = wave >> 1;
    if (t < 2 * kPanel) {
        const int q = t / kPanel, k = k0 - kPanel * q + t % kPanel;
        dsh[q][t % kPanel] = (q < npan && k >= 0 && k < S.n) ? Fs[(int64_t)k * ld] : make_double2(0.0, 0.0);
    }
    // A(j, k) = l_jk (column j of C, lane row j), B(k, i) = l_ik; every row
    // here lies below the panels (j, i >= w0 > k), so only the band limits
    // the entries read.
    const int jr = w0 + 16 * cw + (lane & 15);
    const int ir = i0 + 16 * rw + (lane & 15);
    double2 la[2][kPanel / 4], lb[2][kPanel / 4];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
        const int kp = k0 - kPanel * pp;
        const bool act = pp < npan && kp >= 0;   // uniform
#pragma unroll
        for (int q = 0; q < kPanel / 4; ++q) {
            const int k = kp + 4 * q + (lane >> 4);
            la[pp][q] = act && jr < cend && jr - k <= S.bw ? Fs[(int64_t)k * ld + (jr - k)] : make_double2(0.0, 0.0);
            lb[pp][q] = act && ir < wend && ir - k <= S.bw ? Fs[(int64_t)k * ld + (ir - k)] : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    mfma_f64x4 cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
        if (pp < npan) {   // uniform
#pragma unroll
            for (int q = 0; q < kPanel / 4; ++q) {
                const double2 a = cmul(la[pp][q], dsh[pp][4 * q + (lane >> 4)]);
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, lb[pp][q].x, cre, 0, 0, 0);
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, lb[pp][q].y, cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, lb[pp][q].y, cim, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, lb[pp][q].x, cim, 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = w0 + 16 * cw + (lane >> 4) + 4 * v;
        if (j >= cend || ir >= wend || ir < j) continue;
        double2& c = Fs[(int64_t)j * ld + (ir - j)];
        c.x -= cre[v];
        c.y -= cim[v];
    }
}

// X (tiled, in place) = b: column c of a tile takes B V column bsrc[c] over
// its pencil's rows; padding columns get zero.
__global__ __launch_bounds__(256) void k_band_rhs(TileGeom geom, const int64_t* __restrict__ bsrc,
                                                  const double* __restrict__ BV, int64_t ldbv,
                                                  int ntiles, double2* __restrict__ X) {
    const int tile = blockIdx.y;
    const int n = geom.n[tile];
    const int64_t base = geom.base[tile];
    const int lane = threadIdx.x & 63;
    const int64_t bs = bsrc[tile * kTile + lane];
    for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += gridDim.x * 4) {
        const double b = bs >= 0 ? BV[bs + (int64_t)i * ldbv] : 0.0;
        X[base + (int64_t)i * kTile + lane] = make_double2(b, 0.0);
    }
}

// L y = b, then z = y / d, in place on columns [c0, c0 + CW) of a tile.
// colsys[tile * 64 + lane] is the column's system (-1: padding column).
template <int CW>
__global__ __launch_bounds__(256) void k_band_forward(const BandSys* __restrict__ sys,
                                                      const int32_t* __restrict__ colsys,
                                                      const double2* __restrict__ F, TileGeom geom,
                                                      double2* __restrict__ X) {
    extern __shared__ double2 win[];   // [(bw + 1)][CW]
    const int tile = blockIdx.y;
    const int c0 = blockIdx.x * CW;
    const int n = geom.n[tile];
    const int64_t base = geom.base[tile];
    // every column of a chunk belongs to one pencil (same n, bw); the first
    // real column gives bw
    int bw = -1;
    for (int c = 0; c < CW; ++c) {
        const int s = colsys[tile * kTile + c0 + c];
        if (s >= 0) {
            bw = sys[s].bw;
            break;
        }
    }
    if (bw < 0) return;
    const int ld = bw + 1;
    // per-thread column for the load/store phase
    const int myc = threadIdx.x % CW;
    const int mys = colsys[tile * kTile + c0 + myc];
    for (int r = threadIdx.x / CW; r < ld; r += blockDim.x / CW)
        win[r * CW + myc] = r < n ? X[base + (int64_t)r * kTile + c0 + myc] : make_double2(0.0, 0.0);
    __syncthreads();
    const int upd = bw * CW;
    for (int i = 0; i < n; ++i) {
        const int slot = i % ld;
        // pending value of row i is final: y_i
        if (threadIdx.x < CW && mys >= 0) {
            const double2 y = win[slot * CW + myc];
            const double2 d = F[sys[mys].off + (int64_t)i * ld];
            const double m2 = d.x * d.x + d.y * d.y;
            X[base + (int64_t)i * kTile + c0 + myc] =
                make_double2((y.x * d.x + y.y * d.y) / m2, (y.y * d.x - y.x * d.y) / m2);
        }
        const int dmax = min(bw, n - 1 - i);
        // rows i+1 .. i+dmax -= l_{i+d, i} y_i ; column index slowest so that
        // consecutive threads read consecutive entries of column i of L
        for (int w = threadIdx.x; w < upd; w += blockDim.x) {
            const int c = w / bw;
            const int dd = 1 + (w - c * bw);
            if (dd > dmax) continue;
            const int s = colsys[tile * kTile + c0 + c];
            if (s < 0) continue;
            const double2 y = win[slot * CW + c];
            const double2 l = F[sys[s].off + (int64_t)i * ld + dd];
            cfms(win[((i + dd) % ld) * CW + c], l, y);
        }
        __syncthreads();
        // the slot of row i now takes row i + bw + 1 (untouched so far)
        if (threadIdx.x < CW) {
            const int r = i + ld;
            win[slot * CW + myc] = r < n ? X[base + (int64_t)r * kTile + c0 + myc] : make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
}

// L^T x = z in place (x_i = z_i - sum_d l_{i+d, i} x_{i+d}), rows from the
// bottom up; the solved rows i+1 .. i+bw sit in the LDS window.
template <int CW>
__global__ __launch_bounds__(256) void k_band_backward(const BandSys* __restrict__ sys,
                                                       const int32_t* __restrict__ colsys,
                                                       const double2* __restrict__ F, TileGeom geom,
                                                       double2* __restrict__ X) {
    extern __shared__ double2 win[];   // [(bw + 1)][CW]
    constexpr int TP = band_threads_per_column(CW);   // threads per column, <= one wavefront
    const int tile = blockIdx.y;
    const int c0 = blockIdx.x * CW;
    const int n = geom.n[tile];
    const int64_t base = geom.base[tile];
    int bw = -1;
    for (int c = 0; c < CW; ++c) {
        const int s = colsys[tile * kTile + c0 + c];
        if (s >= 0) {
            bw = sys[s].bw;
            break;
        }
    }
    if (bw < 0) return;
    const int ld = bw + 1;
    const int c = threadIdx.x / TP;     // this thread's column
    const int q = threadIdx.x - c * TP; // its share of the dot product
    const int s = colsys[tile * kTile + c0 + c];
    const int64_t fo = s >= 0 ? sys[s].off : 0;
    for (int i = n - 1; i >= 0; --i) {
        const int dmax = min(bw, n - 1 - i);
        double2 acc = make_double2(0.0, 0.0);
        if (s >= 0) {
            for (int dd = 1 + q; dd <= dmax; dd += TP) {
                const double2 l = F[fo + (int64_t)i * ld + dd];
                const double2 xv = win[((i + dd) % ld) * CW + c];
                acc.x = fma(l.x, xv.x, fma(-l.y, xv.y, acc.x));
                acc.y = fma(l.x, xv.y, fma(l.y, xv.x, acc.y));
            }
        }
        // sum the TP partial dot products of the column (TP divides 64)
#pragma unroll
        for (int o = TP / 2; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o, TP);
            acc.y += __shfl_xor(acc.y, o, TP);
        }
        if (q == 0 && s >= 0) {
            const int64_t o = base + (int64_t)i * kTile + c0 + c;
            const double2 z = X[o];
            const double2 xv = make_double2(z.x - acc.x, z.y - acc.y);
            X[o] = xv;
            win[(i % ld) * CW + c] = xv;
        }
        __syncthreads();
    }
}

// r = b - K x per column (FP64, CSR of the concatenated pencil), stored in
// R; partials of ||r||^2 (x) and ||b||^2 (y) per row block.
template <bool WRITE_R>
__global__ __launch_bounds__(256) void k_band_residual(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const double2* __restrict__ ab, TileGeom geom, const double2* __restrict__ shifts,
    const int64_t* __restrict__ bsrc, const double* __restrict__ BV, int64_t ldbv,
    const double2* __restrict__ X, double2* __restrict__ R, int ntiles, int nrb, int rpb,
    double2* __restrict__ part) {
    __shared__ double2 red[4][kTile];
    // consecutive row blocks of a tile on one XCD, so that the rows a block
    // gathers from its neighbours (a grid row away in a 2D pencil) mostly
    // come from that XCD's L2
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int tile = lb / nrb;
    const int rb = lb - tile * nrb;
    if (tile >= ntiles) return;   // uniform over the work-group
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = geom.n[tile];
    const int row0 = geom.row0[tile];
    const int64_t base = geom.base[tile];
    const int64_t goff = base - (int64_t)row0 * kTile;
    const int col = tile * kTile + lane;
    const double2 z = shifts[col];
    const int64_t bs = bsrc[col];
    const int r0 = min(nt, rb * rpb), r1 = min(nt, r0 + rpb);
    double rr = 0.0, bb = 0.0;
    for (int i = r0 + wave; i < r1; i += 4) {
        const int g = row0 + i;
        double ar = 0, ai = 0, br = 0, bi = 0;
        const int ke = rowptr[g + 1];
        int k = rowptr[g];
        // four gathers in flight; the products are summed in entry order
        for (; k + 4 <= ke; k += 4) {
            double2 v[4], xj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = ab[k + u];
                xj[u] = X[goff + (int64_t)colind[k + u] * kTile + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ar = fma(v[u].x, xj[u].x, ar);
                ai = fma(v[u].x, xj[u].y, ai);
                br = fma(v[u].y, xj[u].x, br);
                bi = fma(v[u].y, xj[u].y, bi);
            }
        }
        for (; k < ke; ++k) {
            const double2 v = ab[k];
            const double2 xj = X[goff + (int64_t)colind[k] * kTile + lane];
            ar = fma(v.x, xj.x, ar);
            ai = fma(v.x, xj.y, ai);
            br = fma(v.y, xj.x, br);
            bi = fma(v.y, xj.y, bi);
        }
        const double b = bs >= 0 ? BV[bs + (int64_t)i * ldbv] : 0.0;
        const double rx = b - (z.x * br - z.y * bi - ar);
        const double ry = -(z.x * bi + z.y * br - ai);
        if (WRITE_R) R[base + (int64_t)i * kTile + lane] = make_double2(rx, ry);
        rr += rx * rx + ry * ry;
        bb += b * b;
    }
    red[wave][lane] = make_double2(rr, bb);
    __syncthreads();
    if (wave == 0) {
        double2 a = red[0][lane];
        for (int w = 1; w < 4; ++w) {
            a.x += red[w][lane].x;
            a.y += red[w][lane].y;
        }
        part[((int64_t)tile * nrb + rb) * kTile + lane] = a;
    }
}

// rel[col] = ||r|| / ||b|| from the row-block partials (fixed order).
__global__ __launch_bounds__(256) void k_band_relres(int nrb, const double2* __restrict__ part,
                                                     double* __restrict__ rel) {
    // wave w sums row blocks w, w + 4, ... and the four sums are added in
    // wave order: a fixed order for every launch
    __shared__ double2 red[4][kTile];
    const int tile = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double rr = 0.0, bb = 0.0;
    for (int rb = wave; rb < nrb; rb += 4) {
        const double2 p = part[((int64_t)tile * nrb + rb) * kTile + lane];
        rr += p.x;
        bb += p.y;
    }
    red[wave][lane] = make_double2(rr, bb);
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < 4; ++w) {
            rr += red[w][lane].x;
            bb += red[w][lane].y;
        }
        rel[tile * kTile + lane] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    }
}

// X += R over the rows of every tile.
__global__ __launch_bounds__(256) void k_band_axpy(TileGeom geom, const double2* __restrict__ R,
                                                   double2* __restrict__ X) {
    const int tile = blockIdx.y;
    const int n = geom.n[tile];
    const int64_t base = geom.base[tile];
    const int lane = threadIdx.x & 63;
    for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += gridDim.x * 4) {
        const int64_t o = base + (int64_t)i * kTile + lane;
        const double2 r = R[o];
        double2 x = X[o];
        x.x += r.x;
        x.y += r.y;
        X[o] = x;
    }
}


// ---- register-window sweeps ---------------------------------------------
// Each CPL columns of a chunk of CPW columns (one system) are owned by a half
// wavefront (CPL = 2 halves the LDS reads of the staged L per column).  Lane l keeps K registers: register k holds row p + l + 32 k,
// where p advances (forward) or retreats (backward) by 32 every 32 rows and
// the registers rotate by one; K * 32 >= bw + 32 covers rows i .. i + bw.
// The L columns of R consecutive rows are staged in LDS (double buffered,
// the next block loaded into registers while the current one is used) as
// 32 K entries: entry 0 and the entries past bw are zero, so every register
// reads entry max(row - i, 0) with no other test (only register 0 can point
// below the row, the others read at constant offsets); the diagonal is
// staged apart (as 1 / d_i for the forward sweep).  One work-group barrier
// per R rows, none per row.
//   forward: the lane holding row i broadcasts y_i = pending + b_i by a
//     shuffle, writes y_i / d_i, and every register subtracts l_{row,i} y_i;
//   backward: every register adds l_{row,i} x_row, the half wave reduces
//     the sum, and the lane holding row i keeps x_i = z_i - sum.
constexpr int kStageLds = 131072;   // bytes of LDS for the staged blocks (one work-group per CU)

// Bytes of LDS for the two staged blocks of a T-thread work-group: the next
// block is prefetched through registers, 8 entries per thread.
constexpr int sweep_stage_bytes(int T) { return T * 2 * 8 * 16 < kStageLds ? T * 2 * 8 * 16 : kStageLds; }

template <int K, int CPW, int CPL, bool FWD>
__global__ __launch_bounds__(CPW * 32 / CPL) void k_band_sweep(const BandSys* __restrict__ sys,
                                                               const int32_t* __restrict__ colsys,
                                                               const double2* __restrict__ F,
                                                               TileGeom geom, double2* __restrict__ X,
                                                               int R, int xcd_map) {
    constexpr int T = CPW * 32 / CPL;
    constexpr int W = 32 * K;   // staged entries per row
    constexpr int CPT = kTile / CPW;   // chunks per tile
    extern __shared__ double2 sh[];
    // Work-groups are dealt to the 8 XCDs round robin by id; with xcd_map the
    // CPT chunks of a tile (one system, the same L) get ids of one residue
    // mod 8, so they share an XCD's L2 while they stream the same factor.
    int tile, chunk;
    if (xcd_map) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        tile = (slot / CPT) * 8 + xcd;
        chunk = slot % CPT;
    } else {
        tile = blockIdx.x / CPT;
        chunk = blockIdx.x % CPT;
    }
    const int c0 = chunk * CPW;
    const int s0 = colsys[tile * kTile + c0];
    if (s0 < 0) return;   // padding chunk (chunks never straddle systems)
    const BandSys S = sys[s0];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const int64_t base = geom.base[tile];
    const int lane = threadIdx.x & 31;
    const int c = (threadIdx.x >> 5) * CPL;   // this half wave's first column (CPL columns)
    const bool upper = (threadIdx.x & 32) != 0;   // upper half of the wavefront
    const int RW = R * W, RC = R * CPW;
    const int stage = RW + R + RC;     // entries per staged block
    double2* Ls = sh;                  // [2][R][W]
    double2* Ds = sh + 2 * RW;         // [2][R]
    double2* bs = Ds + 2 * R;          // [2][R][CPW]
    const double2* Fs = F + S.off;
    const int nblk = (n + R - 1) / R;
    constexpr int PF = (sweep_stage_bytes(T) / (2 * (int)sizeof(double2)) + T - 1) / T;
    double2 pf[PF];
    auto issue = [&](int blk) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = threadIdx.x + q * T;
            double2 v = make_double2(0.0, 0.0);
            if (idx < RW) {
                const int r = idx / W, d = idx - r * W;
                const int i = blk * R + r;
                if (i < n && d >= 1 && d <= bw) v = Fs[(int64_t)i * ld + d];
            } else if (idx < RW + R) {
                const int i = blk * R + (idx - RW);
                if (i < n) {
                    v = Fs[(int64_t)i * ld];
                    if (FWD) {   // the forward sweep divides by d_i: stage 1 / d_i
                        const double m2 = v.x * v.x + v.y * v.y;
                        v = make_double2(v.x / m2, -v.y / m2);
                    }
                }
            } else if (idx < stage) {
                const int r = (idx - RW - R) / CPW, cc = (idx - RW - R) - r * CPW;
                const int i = blk * R + r;
                if (i < n) v = X[base + (int64_t)i * kTile + c0 + cc];
            }
            pf[q] = v;
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = threadIdx.x + q * T;
            if (idx < RW)
                Ls[buf * RW + idx] = pf[q];
            else if (idx < RW + R)
                Ds[buf * R + idx - RW] = pf[q];
            else if (idx < stage)
                bs[buf * RC + idx - RW - R] = pf[q];
        }
    };
    double2 win[CPL][K];
#pragma unroll
    for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int k = 0; k < K; ++k) win[q][k] = make_double2(0.0, 0.0);
    int p = FWD ? 0 : ((n - 1) / 32) * 32;
    issue(FWD ? 0 : nblk - 1);
    commit(0);
    __syncthreads();
    for (int t = 0; t < nblk; ++t) {
        const int blk = FWD ? t : nblk - 1 - t;
        const int buf = t & 1;
        if (t + 1 < nblk) issue(FWD ? blk + 1 : blk - 1);
        for (int rr = 0; rr < R; ++rr) {
            const int r = FWD ? rr : R - 1 - rr;
            const int i = blk * R + r;
            if (i >= n) continue;
            const double2* Lr = Ls + buf * RW + r * W;
            if (FWD) {
                if (i - p == 32) {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
#pragma unroll
                        for (int k = 0; k + 1 < K; ++k) win[q][k] = win[q][k + 1];
                        win[q][K - 1] = make_double2(0.0, 0.0);
                    }
                    p += 32;
                }
                const int ol = i - p;
                const int b0 = p - i + lane;
                double2 lv[K];
#pragma unroll
                for (int k = 0; k < K; ++k) lv[k] = k == 0 ? Lr[max(b0, 0)] : Lr[b0 + 32 * k];
                double2 y[CPL];
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    // row i's pending value sits in register 0 of lane ol of each
                    // half wave; ol is uniform, so read it with readlane (no LDS)
                    const double2 b = bs[buf * RC + r * CPW + c + q];
                    const double2 va = readlane2(win[q][0], ol), vb = readlane2(win[q][0], ol + 32);
                    y[q].x = (upper ? vb.x : va.x) + b.x;
                    y[q].y = (upper ? vb.y : va.y) + b.y;
                }
                if (lane == ol) {
                    const double2 dinv = Ds[buf * R + r];
#pragma unroll
                    for (int q = 0; q < CPL; ++q) X[base + (int64_t)i * kTile + c0 + c + q] = cmul(y[q], dinv);
                }
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int q = 0; q < CPL; ++q) cfms(win[q][k], lv[k], y[q]);
                if (lane == ol)
#pragma unroll
                    for (int q = 0; q < CPL; ++q) win[q][0] = make_double2(0.0, 0.0);
            } else {
                if (i < p) {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
#pragma unroll
                        for (int k = K - 1; k > 0; --k) win[q][k] = win[q][k - 1];
                        win[q][0] = make_double2(0.0, 0.0);
                    }
                    p -= 32;
                }
                const int b0 = p - i + lane;
                double2 lv[K];
#pragma unroll
                for (int k = 0; k < K; ++k) lv[k] = k == 0 ? Lr[max(b0, 0)] : Lr[b0 + 32 * k];
                double2 part[CPL];
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    part[q] = make_double2(0.0, 0.0);
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        part[q].x = fma(lv[k].x, win[q][k].x, fma(-lv[k].y, win[q][k].y, part[q].x));
                        part[q].y = fma(lv[k].x, win[q][k].y, fma(lv[k].y, win[q][k].x, part[q].y));
                    }
                }
#pragma unroll
                for (int o = 16; o > 0; o >>= 1)
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        part[q].x += __shfl_xor(part[q].x, o, 32);
                        part[q].y += __shfl_xor(part[q].y, o, 32);
                    }
                if (lane == i - p) {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        const double2 z = bs[buf * RC + r * CPW + c + q];
                        const double2 xv = make_double2(z.x - part[q].x, z.y - part[q].y);
                        X[base + (int64_t)i * kTile + c0 + c + q] = xv;
                        win[q][0] = xv;
                    }
                }
            }
        }
        if (t + 1 < nblk) commit(buf ^ 1);
        __syncthreads();
    }
}

// ---- blocked forward sweep (FP64 matrix cores) --------------------------
// L y = b, z = D^-1 y for the 16 columns of a chunk (one system), 32 rows
// per block: the block's rows are solved against the 32 x 32 diagonal block
// of L (one half wavefront per two columns, lane = row, the solved value of
// row i broadcast by readlane), then the next bw rows take the block's
// contribution, W[r, :] -= L[r, block] Y[block, :], as complex products on
// v_mfma_f64_16x16x4 tiles (16 rows x 16 columns, 4 block rows per step; a
// complex product is four real ones).  The pending rows live in an LDS ring
// of WS >= bw + 32 rows (row r at slot r mod WS); rows enter the ring from X
// when they first come into reach of a block.  MFMA operand layouts (lane l):
// A(i, k) at i = l % 16, k = l / 16; B(k, j) at k = l / 16, j = l % 16;
// result register v of lane l is D(l / 16 + 4 v, l % 16).
constexpr int kBlkRows = 32;
constexpr int kBlkFwdThreads = 512;   // 4 product waves + 4 solve waves
constexpr int kBlkBwdThreads = 512;   // 4 product waves + 4 solve waves
constexpr int kBlkMaxBw = 384;

// Ring slot of row J0 + d (jb = J0 mod WS, 0 <= d < 2 WS): no division.
__device__ inline int ring_slot(int jb, int d, int WS) {
    int s = jb + d;
    s -= s >= WS ? WS : 0;
    s -= s >= WS ? WS : 0;
    return s;
}

__host__ __device__ constexpr int blk_ring_rows(int bw) { return kBlkRows * ((bw + kBlkRows + kBlkRows - 1) / kBlkRows); }

// The forward sweep's waves work in two roles, so that the matrix-core
// products of block j overlap the triangular solve of block j + 1 instead of
// following it.
// Waves 0-3 (product waves) apply block j to the rows below it, 16-row tiles
// dealt round robin; their first tiles (0-3) cover block j + 1's rows and
// finish before the mid-block barrier.  Waves 4-7 (solve waves) then solve
// block j + 1 (one half wave per two columns) while the product waves finish
// block j's other tiles, and they keep the diagonal blocks of L, 1 / d and
// the rows entering the ring.  Two barriers per block; Y alternates between
// two LDS buffers (block j's is read by the product waves at the start of
// their iteration, block j + 1's written after the mid-block barrier).
template <int NT>
__global__ __launch_bounds__(NT) void k_band_fwd_pipe(const BandSys* __restrict__ sys,
                                                      const int32_t* __restrict__ colsys,
                                                      const double2* __restrict__ F, TileGeom geom,
                                                      double2* __restrict__ X, int xcd_map) {
    constexpr int CPW = 16, CPT = kTile / CPW;
    constexpr int NP = NT / 128;                 // product waves (and solve waves)
    constexpr int NS = NT / 2;                   // solve threads
    constexpr int CPH = CPW * 32 / NS;           // columns per solve half wave
    __shared__ double2 Ld[kBlkRows][kBlkRows + 1];   // L[J0 + r][J0 + c], r > c
    __shared__ double2 Dinv[kBlkRows];
    __shared__ double2 Yb[2][kBlkRows][CPW + 1];
    extern __shared__ double2 ring[];                 // [WS][CPW]
    int tile, chunk;
    if (xcd_map) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        tile = (slot / CPT) * 8 + xcd;
        chunk = slot % CPT;
    } else {
        tile = blockIdx.x / CPT;
        chunk = blockIdx.x % CPT;
    }
    const int c0 = chunk * CPW;
    const int s0 = colsys[tile * kTile + c0];
    if (s0 < 0) return;
    const BandSys S = sys[s0];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const int WS = blk_ring_rows(bw);
    const int64_t base = geom.base[tile];
    const double2* Fs = F + S.off;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const bool prod = wave < NP;                 // uniform over the wave
    const int ts = t - NS;                       // solve thread index (solve waves)
    const int hl = ts & 31, hw = ts >> 5;        // solve half-wave lane (block row) and index
    const bool upper = (ts & 32) != 0;
    for (int e = t; e < (kBlkRows + bw) * CPW; e += NT) {
        const int r = e / CPW, c = e - r * CPW;
        ring[ring_slot(0, r, WS) * CPW + c] = r < n ? X[base + (int64_t)r * kTile + c0 + c] : make_double2(0.0, 0.0);
    }
    const int nblk = (n + kBlkRows - 1) / kBlkRows;
    constexpr int kLdPer = kBlkRows * kBlkRows / NS;
    constexpr int kNewPer = kBlkRows * CPW / NS;
    auto load_ld = [&](int J0, double2 (&pl)[kLdPer], double2& pd) {
#pragma unroll
        for (int m = 0; m < kLdPer; ++m) {
            const int e = ts + NS * m, r = e / kBlkRows, c = e % kBlkRows;
            pl[m] = (r > c && r - c <= bw && J0 + r < n) ? Fs[(int64_t)(J0 + c) * ld + (r - c)]
                                                         : make_double2(0.0, 0.0);
        }
        pd = (ts < kBlkRows && J0 + ts < n) ? Fs[(int64_t)(J0 + ts) * ld] : make_double2(1.0, 0.0);
    };
    auto store_ld = [&](const double2 (&pl)[kLdPer], double2 pd) {
#pragma unroll
        for (int m = 0; m < kLdPer; ++m) {
            const int e = ts + NS * m;
            Ld[e / kBlkRows][e % kBlkRows] = pl[m];
        }
        if (ts < kBlkRows) {
            const double m2 = pd.x * pd.x + pd.y * pd.y;
            Dinv[ts] = make_double2(pd.x / m2, -pd.y / m2);
        }
    };
    // block J0's rows from the ring: y = L_JJ^-1 w, Yb[buf] = y, X = D^-1 y
    auto solve_block = [&](int J0, int buf) {
        const int slot = ring_slot(J0 % WS, hl, WS) * CPW + CPH * hw;
        double2 v[CPH];
#pragma unroll
        for (int q = 0; q < CPH; ++q) v[q] = ring[slot + q];
#pragma unroll
        for (int i = 0; i < kBlkRows; ++i) {
            const double2 l = Ld[hl][i];   // zero unless hl > i
#pragma unroll
            for (int q = 0; q < CPH; ++q) {
                const double2 a = readlane2(v[q], i), b = readlane2(v[q], i + 32);
                cfms(v[q], l, upper ? b : a);
            }
        }
#pragma unroll
        for (int q = 0; q < CPH; ++q) Yb[buf][hl][CPH * hw + q] = v[q];
        if (J0 + hl < n) {
            const double2 di = Dinv[hl];
            double2* xo = X + base + (int64_t)(J0 + hl) * kTile + c0 + CPH * hw;
#pragma unroll
            for (int q = 0; q < CPH; ++q) xo[q] = cmul(v[q], di);
        }
    };
    auto load_a = [&](int J0, int r0, int wend, double2 (&av)[8]) {
        const int ra = r0 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = J0 + 4 * q + (lane >> 4);
            av[q] = (ra < wend && ra - k <= bw) ? Fs[(int64_t)k * ld + (ra - k)] : make_double2(0.0, 0.0);
        }
    };
    double2 pl[kLdPer], pd;
    double2 av[8];
    // rows [J0 + 32 + bw, J0 + 64 + bw) of X, which block J0 brings into
    // reach, read a block ahead so that their loads overlap the solve
    double2 nx[kNewPer];
    auto load_new = [&](int J0) {
#pragma unroll
        for (int m = 0; m < kNewPer; ++m) {
            const int e = ts + NS * m;
            const int r = J0 + kBlkRows + bw + e / CPW, c = e % CPW;
            nx[m] = r < n ? X[base + (int64_t)r * kTile + c0 + c] : make_double2(0.0, 0.0);
        }
    };
    if (!prod) load_new(0);
    if (!prod) load_ld(0, pl, pd);
    __syncthreads();   // ring filled
    if (!prod) store_ld(pl, pd);
    __syncthreads();
    if (!prod) {
        solve_block(0, 0);
        if (nblk > 1) load_ld(kBlkRows, pl, pd);
    } else if (wave < (min(n, kBlkRows + bw) - kBlkRows + 15) / 16) {
        load_a(0, kBlkRows + 16 * wave, min(n, kBlkRows + bw), av);
    }
    __syncthreads();   // Y of block 0 ready
    for (int j = 0; j < nblk; ++j) {
        const int J0 = j * kBlkRows;
        const int jb = J0 % WS;
        const int wend = min(n, J0 + kBlkRows + bw);
        const int ntl = (wend - (J0 + kBlkRows) + 15) / 16;
        // one 16-row tile of block j's product (tile tl, operands in av; the
        // next tile of this wave, tl + NP, loaded meanwhile), Y from LDS per
        // K step
        auto do_tile = [&](int tl) {
            const int r0 = J0 + kBlkRows + 16 * tl;
            double2 an[8];
            if (tl + NP < ntl) load_a(J0, r0 + 16 * NP, wend, an);
            mfma_f64x4 cre, cim;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + (lane >> 4) + 4 * v;
                const double2 w = r < wend ? ring[ring_slot(jb, r - J0, WS) * CPW + (lane & 15)] : make_double2(0.0, 0.0);
                cre[v] = w.x;
                cim[v] = w.y;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double2 y = Yb[j & 1][4 * q + (lane >> 4)][lane & 15];
                // C -= L Y: re -= L_re y_re - L_im y_im, im -= L_re y_im + L_im y_re
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].x, -y.x, cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].x, -y.y, cim, 0, 0, 0);
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].y, y.y, cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].y, -y.x, cim, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + (lane >> 4) + 4 * v;
                if (r < wend) ring[ring_slot(jb, r - J0, WS) * CPW + (lane & 15)] = make_double2(cre[v], cim[v]);
            }
            if (tl + NP < ntl) {
#pragma unroll
                for (int q = 0; q < 8; ++q) av[q] = an[q];
            }
        };
        if (prod) {
            if (wave < ntl) do_tile(wave);   // tiles 0 .. NP-1: block j + 1's rows among them
        } else {
            if (j + 1 < nblk) store_ld(pl, pd);   // L_JJ and 1 / d of block j + 1
            // rows [J0 + 32 + bw, J0 + 64 + bw) come into reach of block j + 1
            // (for narrow bands some are block j + 1's own rows, which its
            // solve below reads): their ring slots held rows of block j,
            // solved in the previous iteration, and no tile of block j
            // reaches them
#pragma unroll
            for (int m = 0; m < kNewPer; ++m) {
                const int e = ts + NS * m;
                const int r = J0 + kBlkRows + bw + e / CPW, c = e % CPW;
                ring[ring_slot(jb, r - J0, WS) * CPW + c] = nx[m];
            }
        }
        __syncthreads();   // rows of block j + 1 final; its L_JJ in LDS
        if (prod) {
            for (int tl = wave + NP; tl < ntl; tl += NP) do_tile(tl);
            if (j + 1 < nblk) {   // first tile of block j + 1 for this wave
                const int J1 = J0 + kBlkRows, wend1 = min(n, J1 + kBlkRows + bw);
                if (wave < (wend1 - (J1 + kBlkRows) + 15) / 16) load_a(J1, J1 + kBlkRows + 16 * wave, wend1, av);
            }
        } else {
            if (j + 1 < nblk) {
                solve_block(J0 + kBlkRows, (j + 1) & 1);
                if (j + 2 < nblk) load_ld(J0 + 2 * kBlkRows, pl, pd);
                load_new(J0 + kBlkRows);
            }
        }
        __syncthreads();
    }
}

// ---- backward sweep in two wave roles ----------------------------------------
// L^T x = z (z = D^-1 y from the forward sweep, in X), 32-row blocks from the
// bottom, right-looking: once block j's x is known, the rows above it within
// the band take z_i -= sum_{r in block j} L[r, i] x_r (a 16-row tile per
// matrix-core product, K = 32 over the block, operands L[r, i] read down
// column i of the band and x from LDS).  Waves 0-3 (product waves) apply
// block j to those rows in 16-row tiles dealt round robin, nearest first, so
// that their first tiles (0-3) cover block j - 1's rows before the mid-block
// barrier.  Waves 4-7 (solve waves) meanwhile insert the rows entering reach
// and keep block j - 1's diagonal block of L; after the barrier they solve
// block j - 1 from its last row up (half wave per two columns, readlane
// broadcast) while the product waves finish block j's other tiles.  Pending
// rows live in an LDS ring (row r in slot r mod WS, WS >= bw + 32); x of the
// last solved block alternates between two LDS buffers.
template <int NT>
__global__ __launch_bounds__(NT) void k_band_bwd_pipe(const BandSys* __restrict__ sys,
                                                      const int32_t* __restrict__ colsys,
                                                      const double2* __restrict__ F, TileGeom geom,
                                                      double2* __restrict__ X, int xcd_map) {
    constexpr int CPW = 16, CPT = kTile / CPW;
    constexpr int NS = 256;                      // solve threads (four waves)
    constexpr int NP = (NT - NS) / 64;           // product waves
    static_assert(NP >= 2 && NP * 64 + NS == NT, "two or more product waves, then four solve waves");
    constexpr int CPH = CPW * 32 / NS;           // columns per solve half wave
    __shared__ double2 Ld[kBlkRows][kBlkRows + 1];   // L[J0 + r][J0 + c], r > c
    __shared__ double2 Yb[2][kBlkRows][CPW + 1];      // x of the last solved block
    extern __shared__ double2 ring[];                 // [WS][CPW]
    int tile, chunk;
    if (xcd_map) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        tile = (slot / CPT) * 8 + xcd;
        chunk = slot % CPT;
    } else {
        tile = blockIdx.x / CPT;
        chunk = blockIdx.x % CPT;
    }
    const int c0 = chunk * CPW;
    const int s0 = colsys[tile * kTile + c0];
    if (s0 < 0) return;
    const BandSys S = sys[s0];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const int WS = blk_ring_rows(bw);
    const int64_t base = geom.base[tile];
    const double2* Fs = F + S.off;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const bool prod = wave < NP;                 // uniform over the wave
    const int ts = t - 64 * NP;                  // solve thread index (solve waves)
    const int hl = ts & 31, hw = ts >> 5;        // solve half-wave lane (block row) and index
    const bool upper = (ts & 32) != 0;
    const int nblk = (n + kBlkRows - 1) / kBlkRows;
    const int Jl = (nblk - 1) * kBlkRows;
    // the bottom block and the rows above it within reach; rows past n are zero
    for (int e = t; e < (kBlkRows + bw) * CPW; e += NT) {
        const int r = Jl - bw + e / CPW, c = e % CPW;
        if (r >= 0) ring[(r % WS) * CPW + c] = r < n ? X[base + (int64_t)r * kTile + c0 + c] : make_double2(0.0, 0.0);
    }
    constexpr int kLdPer = kBlkRows * kBlkRows / NS;
    constexpr int kNewPer = kBlkRows * CPW / NS;
    auto load_ld = [&](int J0, double2 (&pl)[kLdPer]) {
#pragma unroll
        for (int m = 0; m < kLdPer; ++m) {
            const int e = ts + NS * m, r = e / kBlkRows, c = e % kBlkRows;
            pl[m] = (r > c && r - c <= bw && J0 + r < n) ? Fs[(int64_t)(J0 + c) * ld + (r - c)]
                                                         : make_double2(0.0, 0.0);
        }
    };
    auto store_ld = [&](const double2 (&pl)[kLdPer]) {
#pragma unroll
        for (int m = 0; m < kLdPer; ++m) {
            const int e = ts + NS * m;
            Ld[e / kBlkRows][e % kBlkRows] = pl[m];
        }
    };
    // block J0's rows from the ring, solved from the last row up: x to X and Yb[buf]
    auto solve_block = [&](int J0, int buf) {
        const int slot = ((J0 + hl) % WS) * CPW + CPH * hw;
        double2 v[CPH];
#pragma unroll
        for (int q = 0; q < CPH; ++q) v[q] = ring[slot + q];
#pragma unroll
        for (int i = kBlkRows - 1; i >= 0; --i) {
            const double2 l = Ld[i][hl];   // L[J0 + i][J0 + hl], zero unless i > hl
#pragma unroll
            for (int q = 0; q < CPH; ++q) {
                const double2 a = readlane2(v[q], i), b = readlane2(v[q], i + 32);
                cfms(v[q], l, upper ? b : a);
            }
        }
#pragma unroll
        for (int q = 0; q < CPH; ++q) Yb[buf][hl][CPH * hw + q] = J0 + hl < n ? v[q] : make_double2(0.0, 0.0);
        if (J0 + hl < n) {
            double2* xo = X + base + (int64_t)(J0 + hl) * kTile + c0 + CPH * hw;
#pragma unroll
            for (int q = 0; q < CPH; ++q) xo[q] = v[q];
        }
    };
    // A operands of tile rows [I0, I0 + 16) for block J0: A(i, k) = L[J0 + k][I0 + i]
    auto load_a = [&](int J0, int I0, int lo, double2 (&av)[8]) {
        const int ia = I0 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = J0 + 4 * q + (lane >> 4);
            av[q] = (ia >= lo && r < n && r - ia <= bw) ? Fs[(int64_t)ia * ld + (r - ia)] : make_double2(0.0, 0.0);
        }
    };
    double2 pl[kLdPer];
    double2 av[8];
    // rows [J0 - 32 - bw, J0 - bw) of X, which block J0 brings into reach
    // (those at or above row 0), read a block ahead so that their loads
    // overlap the solve
    double2 nx[kNewPer];
    auto load_new = [&](int J0) {
#pragma unroll
        for (int m = 0; m < kNewPer; ++m) {
            const int e = ts + NS * m;
            const int r = J0 - kBlkRows - bw + e / CPW, c = e % CPW;
            nx[m] = r >= 0 ? X[base + (int64_t)r * kTile + c0 + c] : make_double2(0.0, 0.0);
        }
    };
    if (!prod && nblk > 1) load_new(Jl);
    if (!prod) load_ld(Jl, pl);
    __syncthreads();   // ring filled
    if (!prod) store_ld(pl);
    __syncthreads();
    if (!prod) {
        solve_block(Jl, (nblk - 1) & 1);
        if (nblk > 1) load_ld(Jl - kBlkRows, pl);
    } else if (wave < (min(bw, Jl) + 15) / 16) {
        load_a(Jl, Jl - 16 * (wave + 1), max(0, Jl - bw), av);
    }
    __syncthreads();   // x of the bottom block ready
    for (int j = nblk - 1; j > 0; --j) {
        const int J0 = j * kBlkRows;
        const int lo = max(0, J0 - bw);
        const int ntl = (J0 - lo + 15) / 16;
        // one 16-row tile of block j's product (tile tl: rows [J0 - 16 (tl + 1), J0 - 16 tl),
        // operands in av; the next tile of this wave, tl + NP, loaded meanwhile)
        auto do_tile = [&](int tl) {
            const int I0 = J0 - 16 * (tl + 1);
            double2 an[8];
            if (tl + NP < ntl) load_a(J0, I0 - 16 * NP, lo, an);
            mfma_f64x4 cre, cim;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = I0 + (lane >> 4) + 4 * v;
                const double2 w = r >= lo ? ring[(r % WS) * CPW + (lane & 15)] : make_double2(0.0, 0.0);
                cre[v] = w.x;
                cim[v] = w.y;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double2 y = Yb[j & 1][4 * q + (lane >> 4)][lane & 15];
                // C -= A x: re -= A_re x_re - A_im x_im, im -= A_re x_im + A_im x_re
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].x, -y.x, cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].x, -y.y, cim, 0, 0, 0);
                cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].y, y.y, cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q].y, -y.x, cim, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = I0 + (lane >> 4) + 4 * v;
                if (r >= lo) ring[(r % WS) * CPW + (lane & 15)] = make_double2(cre[v], cim[v]);
            }
            if (tl + NP < ntl) {
#pragma unroll
                for (int q = 0; q < 8; ++q) av[q] = an[q];
            }
        };
        if (prod) {
            if (wave < ntl) do_tile(wave);   // tiles 0 .. NP-1: block j - 1's rows among them
        } else {
            store_ld(pl);   // L_JJ of block j - 1
            // rows [J0 - 32 - bw, J0 - bw) come into reach of block j - 1 (for
            // narrow bands some are block j - 1's own rows, which its solve
            // below reads); their slots held rows of block j or below, whose
            // solves are done, and no tile of block j reaches them
#pragma unroll
            for (int m = 0; m < kNewPer; ++m) {
                const int e = ts + NS * m;
                const int r = J0 - kBlkRows - bw + e / CPW, c = e % CPW;
                if (r >= 0) ring[(r % WS) * CPW + c] = nx[m];
            }
        }
        __syncthreads();   // rows of block j - 1 final; its L_JJ in LDS
        if (prod) {
            for (int tl = wave + NP; tl < ntl; tl += NP) do_tile(tl);
            if (j > 1) {   // first tile of block j - 1 for this wave
                const int J1 = J0 - kBlkRows, lo1 = max(0, J1 - bw);
                if (wave < (J1 - lo1 + 15) / 16) load_a(J1, J1 - 16 * (wave + 1), lo1, av);
            }
        } else {
            solve_block(J0 - kBlkRows, (j - 1) & 1);
            if (j > 1) {
                load_ld(J0 - 2 * kBlkRows, pl);
                load_new(J0 - kBlkRows);
            }
        }
        __syncthreads();
    }
}

template <int K, int CPW, int CPL>
static hipError_t sweep_reg(const BandSys* sys, const int32_t* colsys, const double2* F,
                            const TileGeom& g, int ntiles, double2* X, hipStream_t s, int bwmax) {
    constexpr int W = 32 * K;
    constexpr int T = CPW * 32 / CPL;
    // R staged rows: 2 buffers of R * (W + 1 + CPW) entries within the stage bytes
    const int R = std::max(1, std::min(16, sweep_stage_bytes(T) / (2 * (W + 1 + CPW) * (int)sizeof(double2))));
    const size_t lds = (size_t)2 * R * (W + 1 + CPW) * sizeof(double2);
    const int xcd_map = ntiles % 8 == 0;
    const dim3 grid((kTile / CPW) * ntiles);
    // dynamic LDS above 64 KiB (gfx950 has 160 KiB per work-group)
    hipError_t e = hipFuncSetAttribute((const void*)k_band_sweep<K, CPW, CPL, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_band_sweep<K, CPW, CPL, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (CPW == 16 && bwmax <= kBlkMaxBw) {   // blocked forward sweep on the matrix cores
        const size_t ring = (size_t)blk_ring_rows(bwmax) * 16 * sizeof(double2);
        e = hipFuncSetAttribute((const void*)k_band_fwd_pipe<kBlkFwdThreads>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)ring);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_band_fwd_pipe<kBlkFwdThreads>), grid, dim3(kBlkFwdThreads), ring, s, sys, colsys, F,
                           g, X, xcd_map);
    } else {
        hipLaunchKernelGGL((k_band_sweep<K, CPW, CPL, true>), grid, dim3(T), lds, s, sys, colsys, F, g, X, R,
                           xcd_map);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (CPW == 16 && bwmax <= kBlkMaxBw) {
        const size_t ring = (size_t)blk_ring_rows(bwmax) * 16 * sizeof(double2);
        e = hipFuncSetAttribute((const void*)k_band_bwd_pipe<kBlkBwdThreads>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)ring);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_band_bwd_pipe<kBlkBwdThreads>), grid, dim3(kBlkBwdThreads), ring, s, sys, colsys, F,
                           g, X, xcd_map);
    } else {
        hipLaunchKernelGGL((k_band_sweep<K, CPW, CPL, false>), grid, dim3(T), lds, s, sys, colsys, F, g, X, R,
                           xcd_map);
    }
    return hipGetLastError();
}

template <int CPW>
static hipError_t sweep_reg_k(const BandSys* sys, const int32_t* colsys, const double2* F,
                              const TileGeom& g, int ntiles, int bw, double2* X, hipStream_t s) {
    const int need = (bw + 32 + 31) / 32;   // K * 32 >= bw + 32
    // one column per lane (two per lane, CPL = 2, halves the LDS reads but
    // also the waves per CU, and measured slower)
    if (need <= 2) return sweep_reg<2, CPW, 1>(sys, colsys, F, g, ntiles, X, s, bw);
    if (need <= 4) return sweep_reg<4, CPW, 1>(sys, colsys, F, g, ntiles, X, s, bw);
    if (need <= 8) return sweep_reg<8, CPW, 1>(sys, colsys, F, g, ntiles, X, s, bw);
    if (need <= 11) return sweep_reg<11, CPW, 1>(sys, colsys, F, g, ntiles, X, s, bw);
    return sweep_reg<17, CPW, 1>(sys, colsys, F, g, ntiles, X, s, bw);
}

// ---- launchers ---------------------------------------------------------

hipError_t band_form(const BandSys* sys, int nsys, const double2* AB, double2* F, hipStream_t s) {
    // 1024 work-groups: 128 along each band x 8 system lanes
    const int ys = std::min(nsys, 8);
    hipLaunchKernelGGL(k_band_form, dim3(1024 / ys, ys), dim3(256), 0, s, sys, nsys, AB, F);
    return hipGetLastError();
}

// Launch with the optional events e0 (start) and e1 (end) attached to the
// dispatch (hipExtLaunchKernel); without events the plain launch, whose host
// cost is lower.
template <typename... KArgs, typename... Args>
static hipError_t launch_ev(void (*kernel)(KArgs...), dim3 g, dim3 b, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1, Args... args) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, g, b, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, g, b, 0, s, args...);
    return hipGetLastError();
}

hipError_t band_panel(const BandSys* sys, int nsys, int bwmax, double2* F, int k0, int32_t* flag,
                      hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    // one thread per panel row while kPanel + bw rows fit 512 threads
    const int rows = kPanel + bwmax;
    if (rows <= 64) {
        return launch_ev(k_band_panel_rows<64>, dim3(nsys), dim3(64), s, e0, e1, sys, F, k0, flag);
    } else if (rows <= 128) {
        return launch_ev(k_band_panel_rows<128>, dim3(nsys), dim3(128), s, e0, e1, sys, F, k0, flag);
    } else if (rows <= 256) {
        return launch_ev(k_band_panel_rows<256>, dim3(nsys), dim3(256), s, e0, e1, sys, F, k0, flag);
    } else if (rows <= 384) {
        return launch_ev(k_band_panel_rows<384>, dim3(nsys), dim3(384), s, e0, e1, sys, F, k0, flag);
    } else if (rows <= 512) {
        return launch_ev(k_band_panel_rows<512>, dim3(nsys), dim3(512), s, e0, e1, sys, F, k0, flag);
    }
    // wider bands (only with band_kernels = 1; by default the wide-band
    // kernels take them): the panel stays in global memory
    return launch_ev(k_band_panel, dim3(nsys), dim3(256), s, e0, e1, sys, F, k0, flag);
}

hipError_t band_update(const BandSys* sys, int nsys, int bwmax, double2* F, int k0, int part,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int w0 = k0 + kPanel;
    if (part == 1) {
        const int T = (bwmax + 31) / 32;
        if (T == 0) {   // diagonal systems: nothing couples the panels
            if (e0) {
                hipError_t e = hipEventRecord(e0, s);
                if (e != hipSuccess) return e;
            }
            return e1 ? hipEventRecord(e1, s) : hipSuccess;
        }
        // XCD-grouped order: 8 work-group slots per group of 8 systems and tile
        const int groups = (nsys + 7) / 8;
        return launch_ev(k_band_strip, dim3(8 * groups * T), dim3(256), s, e0, e1, sys, nsys, T, F, k0,
                         k0 >= kPanel ? 2 : 1);
    }
    const int c0 = part == 2 ? w0 + 2 * kPanel : w0, c1 = w0 + bwmax;
    const int T = (w0 + bwmax - c0 + 63) / 64;
    const int tiles = T * (T + 1) / 2;
    if (tiles <= 0 || c0 >= c1) {   // nothing to update (narrow band): the events still bracket a point
        if (e0) {
            hipError_t e = hipEventRecord(e0, s);
            if (e != hipSuccess) return e;
        }
        return e1 ? hipEventRecord(e1, s) : hipSuccess;
    }
    // XCD-grouped order: 8 work-group slots per group of 8 systems and tile
    const int groups = (nsys + 7) / 8;
    return launch_ev(k_band_update, dim3(8 * groups * tiles), dim3(256), s, e0, e1, sys, nsys, tiles, F, k0, c0, c1);
}

int band_chunk_columns(int bw) {
    const size_t ld = (size_t)bw + 1;
    int cw = 16;
    while (cw > 1 && ld * cw * sizeof(double2) > kBandLds) cw >>= 1;
    return cw;
}

template <int CW>
static hipError_t solve_cw(const BandSys* sys, const int32_t* colsys, const double2* F,
                           const TileGeom& g, int ntiles, int bw, double2* X, hipStream_t s) {
    const size_t lds = (size_t)(bw + 1) * CW * sizeof(double2);
    hipLaunchKernelGGL((k_band_forward<CW>), dim3(kTile / CW, ntiles), dim3(256), lds, s, sys,
                       colsys, F, g, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_band_backward<CW>), dim3(kTile / CW, ntiles),
                       dim3(CW * band_threads_per_column(CW)), lds, s, sys, colsys, F, g, X);
    return hipGetLastError();
}

hipError_t band_solve(const BandSys* sys, const int32_t* colsys, const double2* F,
                      const TileGeom& g, int ntiles, int bwmax, double2* X, hipStream_t s,
                      int chunk) {
    // register-window sweeps when every chunk of `chunk` columns is one
    // system and the window fits 16 slots per lane
    if ((chunk == 16 || chunk == 8) && bwmax + 32 <= 32 * 17) {
        if (chunk == 16) return sweep_reg_k<16>(sys, colsys, F, g, ntiles, bwmax, X, s);
        return sweep_reg_k<8>(sys, colsys, F, g, ntiles, bwmax, X, s);
    }
    switch (band_chunk_columns(bwmax)) {
        case 16: return solve_cw<16>(sys, colsys, F, g, ntiles, bwmax, X, s);
        case 8: return solve_cw<8>(sys, colsys, F, g, ntiles, bwmax, X, s);
        case 4: return solve_cw<4>(sys, colsys, F, g, ntiles, bwmax, X, s);
        case 2: return solve_cw<2>(sys, colsys, F, g, ntiles, bwmax, X, s);
        default: return solve_cw<1>(sys, colsys, F, g, ntiles, bwmax, X, s);
    }
}

hipError_t band_rhs(const TileGeom& g, const int64_t* bsrc, const double* BV, int64_t ldbv,
                    int ntiles, double2* X, hipStream_t s) {
    hipLaunchKernelGGL(k_band_rhs, dim3(256, ntiles), dim3(256), 0, s, g, bsrc, BV, ldbv, ntiles, X);
    return hipGetLastError();
}

hipError_t band_residual(const DevPencil& P, const TileGeom& g, const double2* shifts,
                         const int64_t* bsrc, const double* BV, int64_t ldbv, const double2* X,
                         double2* R, int ntiles, int64_t nmax, double2* part, int nrb_cap,
                         double* rel, hipStream_t s) {
    const int rpb = (int)std::max<int64_t>(16, (nmax + nrb_cap - 1) / nrb_cap);
    const int nrb = (int)((nmax + rpb - 1) / rpb);
    if (R)
        hipLaunchKernelGGL(k_band_residual<true>, dim3(pad8(ntiles * nrb)), dim3(256), 0, s, P.rowptr, P.colind,
                           P.ab, g, shifts, bsrc, BV, ldbv, X, R, ntiles, nrb, rpb, part);
    else
        hipLaunchKernelGGL(k_band_residual<false>, dim3(pad8(ntiles * nrb)), dim3(256), 0, s, P.rowptr, P.colind,
                           P.ab, g, shifts, bsrc, BV, ldbv, X, R, ntiles, nrb, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_relres, dim3(ntiles), dim3(256), 0, s, nrb, part, rel);
    return hipGetLastError();
}

hipError_t band_axpy(const TileGeom& g, const double2* R, int ntiles, double2* X, hipStream_t s) {
    hipLaunchKernelGGL(k_band_axpy, dim3(256, ntiles), dim3(256), 0, s, g, R, X);
    return hipGetLastError();
}

}  // namespace gep
