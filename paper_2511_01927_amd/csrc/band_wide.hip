// Banded L D L^T of the shifted systems for wide bands and for FP32 factors
// (the quadrature equation's N_q shifted solves; paper Appendix, "Numerical
// Quadrature").  3D grids in natural order have half bandwidth n^(2/3)
// (4096 on 64^3), where one step of the factorisation is a large,
// parallel trailing update instead of a latency-bound chain of short
// kernels, and where Jacobi-preconditioned COCG does not converge on the
// interior shifted systems.  Every kernel here is templated on the complex
// type of the factor: double2 (FP64) or float2 (FP32 factor, FP64 residual
// refinement by the caller: the mixed-precision path).
//
// Storage is the band layout of band.hip (column-major lower band, entry
// (i, j), 0 <= i - j <= bw, at off + j (bw + 1) + (i - j)), in the factor's
// own precision.
//
// Factorisation, right-looking by panels of kPanel columns:
//   k_wb_scatter  F = z B - A from the pencil's CSR rows (the band is
//                 zeroed first; the pencil's own band is never stored);
//   k_wb_panel    one work-group per (system, chunk of 224 panel rows): the
//                 32 pivot rows are factored redundantly in every chunk (one
//                 thread per row, the row's panel entries in registers) and
//                 each chunk applies the column eliminations to its rows;
//   k_wb_update   the trailing window C -= W diag(d) W^T, lower triangle,
//                 64 x 64 tiles on the matrix cores (v_mfma_f64_16x16x4 or
//                 v_mfma_f32_16x16x4); panels go in pairs: the second
//                 panel's columns take the first's contribution (a strip),
//                 and the window beyond them takes both panels' in one
//                 read-modify-write.
// Solves on the tiled multivector by chunks of at most 16 columns of one
// system: 32-row blocks grouped in big blocks of 256 rows; each block's
// coupling to the rows solved before it (forward: the bw rows above;
// backward: the bw rows below) is a matrix-core product whose K dimension
// runs over those rows in 64-row tiles staged through LDS; the part that
// reaches past the current big block is formed for its eight blocks in
// parallel (k_wb_far), the rest and the blocks' triangles in order
// (k_wb_near).  The forward sweep leaves y = L^-1 b; the backward sweep
// divides by d on the fly.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gep {

namespace {

template <typename C>
struct Real;
template <>
struct Real<double2> {
    using T = double;
};
template <>
struct Real<float2> {
    using T = float;
};

__device__ inline double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

template <typename C>
__device__ inline C mkc(typename Real<C>::T x, typename Real<C>::T y) {
    C c;
    c.x = x;
    c.y = y;
    return c;
}
template <typename C>
__device__ inline C czero() {
    return mkc<C>(0, 0);
}
template <typename C>
__device__ inline C cmulT(C a, C b) {
    return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a -= b * c
template <typename C>
__device__ inline void cfmsT(C& a, C b, C c) {
    a.x = fmaT(-b.x, c.x, fmaT(b.y, c.y, a.x));
    a.y = fmaT(-b.x, c.y, fmaT(-b.y, c.x, a.y));
}

typedef double wb_f64x4 __attribute__((ext_vector_type(4)));
typedef float wb_f32x4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core product per wavefront: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; result register v of lane l holds D[row(l, v)][l % 16].
template <typename C>
struct Mma;
template <>
struct Mma<double2> {
    using V = wb_f64x4;
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mma<float2> {
    using V = wb_f32x4;
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// acc_re += a b (real part), acc_im += a b (imaginary part) for complex operands
template <typename C>
__device__ inline void cmma(C a, C b, typename Mma<C>::V& re, typename Mma<C>::V& im) {
    re = Mma<C>::mma(a.x, b.x, re);
    re = Mma<C>::mma(-a.y, b.y, re);
    im = Mma<C>::mma(a.x, b.y, im);
    im = Mma<C>::mma(a.y, b.x, im);
}

constexpr int kWbRows = 256 - kPanel;   // non-pivot panel rows per work-group

}  // namespace

// ---- forming F = z B - A ---------------------------------------------------
// blockIdx.y: system; rows of the system in a grid-stride loop over blockIdx.x.
template <typename C>
__global__ __launch_bounds__(256) void k_wb_scatter(const BandSys* __restrict__ sys,
                                                    const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colind,
                                                    const double2* __restrict__ ab, C* __restrict__ F) {
    using R = typename Real<C>::T;
    const BandSys S = sys[blockIdx.y];
    const int ld = S.bw + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += gridDim.x * blockDim.x) {
        const int g = S.row0 + i;
        for (int e = rowptr[g]; e < rowptr[g + 1]; ++e) {
            const int j = colind[e] - S.row0;
            if (j > i || i - j > S.bw) continue;
            const double2 v = ab[e];   // (a_ij, b_ij)
            F[S.off + (int64_t)j * ld + (i - j)] = mkc<C>((R)(S.z.x * v.y - v.x), (R)(S.z.y * v.y));
        }
    }
}

// ---- panel -------------------------------------------------------------------
// Panel [k0, k0 + kPanel) of every system (blockIdx.y), rows split in chunks
// of kWbRows (blockIdx.x).  Thread t < kPanel holds pivot row k0 + t, thread
// t >= kPanel row k0 + kPanel + blockIdx.x * kWbRows + (t - kPanel), each
// with its panel entries (column k at slot k) in registers.  Column jj: the
// pivot rows publish a_kj and 1 / d_j in LDS; every row i with i - j in
// (0, bw] forms l_ij = a_ij / d_j and a_ik -= l_ij a_kj for the later panel
// columns k (column jj + 1 first, so that it can be published before the
// rest of the update).  Every chunk factors the pivot rows itself (the same
// arithmetic in every chunk); chunk 0 stores them and flags a zero or
// non-finite pivot.
template <typename C>
__global__ __launch_bounds__(256) void k_wb_panel(const BandSys* __restrict__ sys, C* F, int k0,
                                                  int32_t* __restrict__ flag) {
    using R = typename Real<C>::T;
    __shared__ C cb[2][kPanel + 1];
    const BandSys S = sys[blockIdx.y];
    if (k0 >= S.n) return;
    const int ld = S.bw + 1;
    const int ncols = min(kPanel, S.n - k0);
    const int t = threadIdx.x;
    const bool pivot = t < kPanel;
    const int rel = pivot ? t : kPanel + (int)blockIdx.x * kWbRows + (t - kPanel);
    if (blockIdx.x > 0 && (int)blockIdx.x * kWbRows >= S.bw) return;   // chunk past this band (uniform)
    const int i = k0 + rel;
    const bool row_ok = (pivot ? rel < ncols : rel < ncols + S.bw) && i < S.n;
    C* Fs = F + S.off;
    C a[kPanel];
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const bool ok = row_ok && k < ncols && rel >= k && rel - k <= S.bw;
        a[k] = ok ? Fs[(int64_t)(k0 + k) * ld + (rel - k)] : czero<C>();
    }
    auto publish = [&](C* c, int jj, C v) {
        if (pivot && t >= jj && t < ncols) c[t] = v;
        if (t == jj) {
            const R m2 = v.x * v.x + v.y * v.y;
            if (blockIdx.x == 0 && (!(m2 > (R)0) || !isfinite(m2))) flag[blockIdx.y] = 1;
            c[kPanel] = mkc<C>(v.x / m2, -v.y / m2);
        }
    };
    publish(cb[0], 0, a[0]);
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kPanel; ++jj) {
        if (jj < ncols) {   // uniform
            const C* c = cb[jj & 1];
            const int jn = jj + 1 < kPanel ? jj + 1 : jj;
            const bool upd = row_ok && rel > jj && rel - jj <= S.bw;
            C l = czero<C>();
            if (upd) {
                l = cmulT(a[jj], c[kPanel]);
                a[jj] = l;
                if (jj + 1 < kPanel) cfmsT(a[jn], l, c[jn]);
            }
            if (jj + 1 < ncols) publish(cb[(jj + 1) & 1], jj + 1, a[jn]);
            if (upd) {
#pragma unroll
                for (int k = jj + 2; k < kPanel; ++k) cfmsT(a[k], l, c[k]);
            }
            __syncthreads();
        }
    }
    if (pivot && blockIdx.x != 0) return;
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        const bool ok = row_ok && k < ncols && rel >= k && rel - k <= S.bw;
        if (ok) Fs[(int64_t)(k0 + k) * ld + (rel - k)] = a[k];
    }
}

// ---- trailing update ---------------------------------------------------------
// Contributions of the npan panels starting at k0 (columns [k0, k0 + 32
// npan)) to the window columns [c0, c1), rows [c0, wend), wend = min(n,
// k0 + 32 npan + bw), lower triangle: C[i, j] -= sum_k l_ik d_k l_jk.
// strip == 0: blockIdx.x is a lower-triangular index of 64 x 64 tiles
// (bi >= bj) from (c0, c0); strip != 0: the row tile of the single tile
// column at c0 (c1 - c0 <= 64).  blockIdx.y: system.  Wave w forms D(j, i)
// for the tile's 16 columns j of block w and all 64 rows i (four 16-row
// blocks): A = W_j = l_jk d_k, B = l_ik, each panel's 32 columns staged in
// LDS in turn with lanes running down band columns; the result registers
// run down a column of C, so the single read-modify-write per tile is
// coalesced.  Entries a panel does not reach (past its band) are zero.
// WPE: waves per SIMD the registers must allow (four work-groups per CU fit
// the FP32 operands' LDS, two the FP64 ones').
template <typename C, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_wb_update(const BandSys* __restrict__ sys, C* F, int k0, int npan,
                                                   int c0, int c1, int strip) {
    using V = typename Mma<C>::V;
    __shared__ C Wi[64][kPanel + 1];
    __shared__ C Wj[64][kPanel + 1];
    const BandSys S = sys[blockIdx.y];
    const int wend = min(S.n, k0 + kPanel * npan + S.bw);
    const int cend = min(c1, wend);
    if (c0 >= cend) return;
    const int x = blockIdx.x;
    int bi = x, bj = 0;
    if (!strip) {
        bi = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
        while ((bi + 1) * (bi + 2) / 2 <= x) ++bi;
        while (bi * (bi + 1) / 2 > x) --bi;
        bj = x - bi * (bi + 1) / 2;
    }
    const int i0 = c0 + 64 * bi, j0 = c0 + 64 * bj;
    if (i0 >= wend || j0 >= cend) return;   // uniform
    const int ld = S.bw + 1;
    C* Fs = F + S.off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    V pre[4], pim[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        pre[rb] = V{0, 0, 0, 0};
        pim[rb] = V{0, 0, 0, 0};
    }
    // panel pp's operands go through registers into LDS; the next panel's
    // are loaded while this one's products run
    constexpr int kPer = 64 * kPanel / 256;
    C ri[kPer], rj[kPer];
    auto fetch = [&](int kp) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int idx = threadIdx.x + 256 * q;
            const int r = idx & 63, kk = idx >> 6;
            const int k = kp + kk;
            const int i = i0 + r, j = j0 + r;
            ri[q] = czero<C>();
            rj[q] = czero<C>();
            if (k < S.n) {
                if (i < wend && i - k <= S.bw) ri[q] = Fs[(int64_t)k * ld + (i - k)];
                if (j < cend && j - k <= S.bw) rj[q] = cmulT(Fs[(int64_t)k * ld + (j - k)], Fs[(int64_t)k * ld]);
            }
        }
    };
    fetch(k0);
    for (int pp = 0; pp < npan; ++pp) {
        const int kp = k0 + kPanel * pp;
        if (kp >= S.n) break;   // uniform
        if (pp > 0) __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int idx = threadIdx.x + 256 * q;
            Wi[idx & 63][idx >> 6] = ri[q];
            Wj[idx & 63][idx >> 6] = rj[q];
        }
        __syncthreads();
        if (pp + 1 < npan && kp + kPanel < S.n) fetch(kp + kPanel);
#pragma unroll 2
        for (int st = 0; st < kPanel / 4; ++st) {
            const int kk = 4 * st + (lane >> 4);
            const C a = Wj[wave * 16 + (lane & 15)][kk];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) cmma<C>(a, Wi[rb * 16 + (lane & 15)][kk], pre[rb], pim[rb]);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + wave * 16 + Mma<C>::row(lane, v);
            const int i = i0 + rb * 16 + (lane & 15);
            if (j >= cend || i >= wend || i < j) continue;
            C& c = Fs[(int64_t)j * ld + (i - j)];
            c.x -= pre[rb][v];
            c.y -= pim[rb][v];
        }
}

// ---- blocked sweeps --------------------------------------------------------------
// The solves walk a system's rows in big blocks of kWbBig = 256 rows (in
// order for L y = b, in reverse for L^T x = D^-1 y), each split into eight
// 32-row blocks.  For the 32-row block at rows [i0, i0 + 32):
//   forward:  y_i = b_i - sum_{j < i0} l_ij y_j - sum_{i0 <= j < i} l_ij y_j;
//   backward: x_i = y_i / d_i - sum_{j >= i0 + 32} l_ji x_j - sum_{i < j < i0 + 32} l_ji x_j.
// The coupling to the rows outside the current big block ("far") only needs
// rows solved in earlier big blocks, so it is formed for all eight blocks at
// once by k_wb_far, one work-group per (chunk, block), into a scratch D.  The
// coupling inside the big block ("near", at most 224 rows) and the block's
// triangle are then done in order by k_wb_near, one work-group per chunk.
// A chunk is up to 16 consecutive columns of one system inside one tile of
// the multivector X (element (i, c) at base + i * 64 + lane0 + c).
//
// Coupling products: D(i, c) = sum_k A(i, k) Y(k, c) over 64-row tiles of
// the coupled rows; the L tile is staged in LDS as Lt[k][i] (forward:
// l_{i0+i, j0+k}, read down the factor's columns j; backward:
// l_{j0+k, i0+i}, read down columns i), the next tile prefetched into
// registers; the four waves take interleaved K steps of 4 on the matrix
// cores and their partial D meet in LDS.
constexpr int kWbBig = 256;

template <typename C, bool FWD>
__device__ inline void wb_coupling(const C* __restrict__ Fs, int ld, int bw, int i0, int rows, int jlo,
                                   int jhi, const C* __restrict__ Xc, int cnt, C (*Lt)[33],
                                   C (*part)[32][16]) {
    using V = typename Mma<C>::V;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int cb = lane & 15;
    const bool cok = cb < cnt;
    V re[2], im[2];
    re[0] = re[1] = im[0] = im[1] = V{0, 0, 0, 0};
    auto fetch = [&](int j0, C* v) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = t + 256 * q;
            const int k = FWD ? (e >> 5) : (e & 63);
            const int i = FWD ? (e & 31) : (e >> 6);
            const int j = j0 + k, r = i0 + i;
            v[q] = czero<C>();
            if (FWD) {
                if (j < jhi && i < rows && r - j <= bw) v[q] = Fs[(int64_t)j * ld + (r - j)];
            } else {
                if (j < jhi && i < rows && j - r <= bw) v[q] = Fs[(int64_t)r * ld + (j - r)];
            }
        }
    };
    C nxt[8];
    if (jlo < jhi) fetch(jlo, nxt);
    for (int j0 = jlo; j0 < jhi; j0 += 64) {
        __syncthreads();   // the previous tile has been consumed
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = t + 256 * q;
            const int k = FWD ? (e >> 5) : (e & 63);
            const int i = FWD ? (e & 31) : (e >> 6);
            Lt[k][i] = nxt[q];
        }
        C xb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * (wave + 4 * u) + (lane >> 4);
            xb[u] = (j0 + k < jhi && cok) ? Xc[(int64_t)(j0 + k) * 64 + cb] : czero<C>();
        }
        __syncthreads();
        if (j0 + 64 < jhi) fetch(j0 + 64, nxt);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * (wave + 4 * u) + (lane >> 4);
#pragma unroll
            for (int h = 0; h < 2; ++h) cmma<C>(Lt[k][16 * h + (lane & 15)], xb[u], re[h], im[h]);
        }
    }
    // register v of lane l holds D(16 h + row(l, v), l % 16)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[wave][16 * h + Mma<C>::row(lane, v)][lane & 15] = mkc<C>(re[h][v], im[h][v]);
}

// Far coupling of block blockIdx.y of big block `big` for chunk blockIdx.x,
// the four waves' partials summed into Dfar[chunk][32 y + r][c].
template <typename C, bool FWD>
__global__ __launch_bounds__(256) void k_wb_far(const BandSys* __restrict__ sys,
                                                const WbChunk* __restrict__ chunks, const C* __restrict__ F,
                                                TileGeom geom, const C* __restrict__ X, C* __restrict__ Dfar,
                                                int big) {
    __shared__ C Lt[64][33];
    __shared__ C part[4][32][16];
    const WbChunk ch = chunks[blockIdx.x];
    const BandSys S = sys[ch.sys];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const int b0 = big * kWbBig;
    const int i0 = b0 + 32 * blockIdx.y;
    if (i0 >= n) return;   // uniform
    const int rows = min(32, n - i0);
    const int jlo = FWD ? max(0, i0 - bw) : min(n, b0 + kWbBig);
    const int jhi = FWD ? b0 : min(n, i0 + rows + bw);
    const C* Xc = X + geom.base[ch.tile] + ch.lane0;
    wb_coupling<C, FWD>(F + S.off, ld, bw, i0, rows, jlo, jhi, Xc, ch.cnt, Lt, part);
    __syncthreads();
    C* D = Dfar + ((int64_t)blockIdx.x * kWbBig + 32 * blockIdx.y) * 16;
    for (int e = threadIdx.x; e < 32 * 16; e += 256) {
        const int r = e >> 4, c = e & 15;
        C v = part[0][r][c];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
            v.x += part[w][r][c].x;
            v.y += part[w][r][c].y;
        }
        D[r * 16 + c] = v;
    }
}

// Near coupling and triangles of the eight blocks of big block `big`, in
// order (forward) or reverse (backward), one work-group per chunk.  The
// triangle is solved right-looking by all threads: thread t owns column
// t % 16 and rows t / 16 and t / 16 + 16.
template <typename C, bool FWD>
__global__ __launch_bounds__(256) void k_wb_near(const BandSys* __restrict__ sys,
                                                 const WbChunk* __restrict__ chunks, const C* __restrict__ F,
                                                 TileGeom geom, C* __restrict__ X, const C* __restrict__ Dfar,
                                                 int big) {
    using R = typename Real<C>::T;
    __shared__ C Lt[64][33];
    __shared__ C Ld[32][33];      // Ld[r][q] = l_{i0+r, i0+q}, q < r; Ld[r][r] = d
    __shared__ C part[4][32][16];
    __shared__ C rhs[32][16];
    const WbChunk ch = chunks[blockIdx.x];
    const BandSys S = sys[ch.sys];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const int b0 = big * kWbBig;
    if (b0 >= n) return;   // uniform
    const C* Fs = F + S.off;
    C* Xc = X + geom.base[ch.tile] + ch.lane0;
    const C* Dc = Dfar + (int64_t)blockIdx.x * kWbBig * 16;
    const int t = threadIdx.x;
    const int tc = t & 15, tr = t >> 4;
    const int bend = min(n, b0 + kWbBig);
    const int nb = (bend - b0 + 31) / 32;
    for (int u = 0; u < nb; ++u) {
        const int blk = FWD ? u : nb - 1 - u;
        const int i0 = b0 + 32 * blk;
        const int rows = min(32, n - i0);
        const int jlo = FWD ? max(b0, i0 - bw) : i0 + 32;
        const int jhi = FWD ? i0 : min(bend, i0 + rows + bw);
        wb_coupling<C, FWD>(Fs, ld, bw, i0, rows, jlo, jhi, Xc, ch.cnt, Lt, part);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int col = e >> 5, r = e & 31;
            C v = czero<C>();
            if (r >= col && r < rows && col < rows && r - col <= bw) v = Fs[(int64_t)(i0 + col) * ld + (r - col)];
            Ld[r][col] = v;
        }
        __syncthreads();
        // right-hand side of the block's triangle: b (or y / d) - far - near
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = tr + 16 * h;
            C v = czero<C>();
            if (r < rows && tc < ch.cnt) {
                v = Xc[(int64_t)(i0 + r) * 64 + tc];
                if (!FWD) {
                    const C d = Ld[r][r];
                    const R m2 = d.x * d.x + d.y * d.y;
                    v = cmulT(v, mkc<C>(d.x / m2, -d.y / m2));
                }
                const C f = Dc[(32 * blk + r) * 16 + tc];
                v.x -= f.x;
                v.y -= f.y;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    v.x -= part[w][r][tc].x;
                    v.y -= part[w][r][tc].y;
                }
            }
            rhs[r][tc] = v;
        }
        __syncthreads();
        if (FWD) {
            for (int q = 0; q < rows - 1; ++q) {
                const C yq = rhs[q][tc];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = tr + 16 * h;
                    if (r > q && r < rows) cfmsT(rhs[r][tc], Ld[r][q], yq);
                }
                __syncthreads();
            }
        } else {
            for (int q = rows - 1; q > 0; --q) {
                const C xq = rhs[q][tc];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = tr + 16 * h;
                    if (r < q) cfmsT(rhs[r][tc], Ld[q][r], xq);
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = tr + 16 * h;
            if (r < rows && tc < ch.cnt) Xc[(int64_t)(i0 + r) * 64 + tc] = rhs[r][tc];
        }
        __syncthreads();
    }
}

// ---- precision conversions over chunks ----------------------------------------
// D (FP32) = S (FP64) on the chunks' columns.
__global__ __launch_bounds__(256) void k_wb_narrow(const BandSys* __restrict__ sys,
                                                   const WbChunk* __restrict__ chunks, TileGeom geom,
                                                   const double2* __restrict__ Sx, float2* __restrict__ D) {
    const WbChunk ch = chunks[blockIdx.y];
    const int n = sys[ch.sys].n;
    const int64_t base = geom.base[ch.tile] + ch.lane0;
    const int c = threadIdx.x & 15;
    if (c >= ch.cnt) return;
    for (int i = blockIdx.x * 16 + (threadIdx.x >> 4); i < n; i += gridDim.x * 16) {
        const double2 v = Sx[base + (int64_t)i * 64 + c];
        D[base + (int64_t)i * 64 + c] = make_float2((float)v.x, (float)v.y);
    }
}

// X (FP64) += D (C) on the chunks' columns (set = 1: X = D).
template <typename C>
__global__ __launch_bounds__(256) void k_wb_accumulate(const BandSys* __restrict__ sys,
                                                       const WbChunk* __restrict__ chunks, TileGeom geom,
                                                       const C* __restrict__ D, double2* __restrict__ X,
                                                       int set) {
    const WbChunk ch = chunks[blockIdx.y];
    const int n = sys[ch.sys].n;
    const int64_t base = geom.base[ch.tile] + ch.lane0;
    const int c = threadIdx.x & 15;
    if (c >= ch.cnt) return;
    for (int i = blockIdx.x * 16 + (threadIdx.x >> 4); i < n; i += gridDim.x * 16) {
        const int64_t o = base + (int64_t)i * 64 + c;
        const C d = D[o];
        double2 x = set ? make_double2(0.0, 0.0) : X[o];
        x.x += (double)d.x;
        x.y += (double)d.y;
        X[o] = x;
    }
}

// ---- launchers -----------------------------------------------------------------
template <typename C>
static hipError_t wb_form_t(const DevPencil& P, const BandSys* sys, int nsys, C* F, hipStream_t s) {
    hipLaunchKernelGGL(k_wb_scatter<C>, dim3(64, nsys), dim3(256), 0, s, sys, P.rowptr, P.colind, P.ab, F);
    return hipGetLastError();
}

// One step of two panels: panel k0, the next panel's columns updated with
// it (a 32-column strip), panel k0 + kPanel, then the trailing window from
// k0 + 2 kPanel with both panels (one read-modify-write of the window per
// two panels).
template <typename C>
static hipError_t wb_step_t(const BandSys* sys, int nsys, int bwmax, C* F, int k0, int nmax, int32_t* flag,
                            hipStream_t s) {
    const int chunks = std::max(1, (bwmax + kWbRows - 1) / kWbRows);
    const int T = (bwmax + 63) / 64;
    hipLaunchKernelGGL(k_wb_panel<C>, dim3(chunks, nsys), dim3(256), 0, s, sys, F, k0, flag);
    if (k0 + kPanel >= nmax) return hipGetLastError();
    if (bwmax > 0)
        hipLaunchKernelGGL((k_wb_update<C, sizeof(C) == 8 ? 4 : 2>), dim3(T + 1, nsys), dim3(256), 0, s, sys, F, k0, 1, k0 + kPanel,
                           k0 + 2 * kPanel, 1);
    hipLaunchKernelGGL(k_wb_panel<C>, dim3(chunks, nsys), dim3(256), 0, s, sys, F, k0 + kPanel, flag);
    if (k0 + 2 * kPanel >= nmax || bwmax == 0) return hipGetLastError();
    hipLaunchKernelGGL((k_wb_update<C, sizeof(C) == 8 ? 4 : 2>), dim3(T * (T + 1) / 2, nsys), dim3(256), 0, s, sys, F, k0, 2,
                       k0 + 2 * kPanel, k0 + 2 * kPanel + bwmax, 0);
    return hipGetLastError();
}

template <typename C>
static hipError_t wb_solve_t(const BandSys* sys, const WbChunk* chunks, int nchunks, const C* F,
                             const TileGeom& g, C* X, int nmax, C* Dfar, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const int nbig = (nmax + kWbBig - 1) / kWbBig;
    for (int b = 0; b < nbig; ++b) {
        // (big block 0 has nothing above it: the far kernel writes zeros)
        hipLaunchKernelGGL((k_wb_far<C, true>), dim3(nchunks, kWbBig / 32), dim3(256), 0, s, sys, chunks, F, g,
                           X, Dfar, b);
        hipLaunchKernelGGL((k_wb_near<C, true>), dim3(nchunks), dim3(256), 0, s, sys, chunks, F, g, X, Dfar, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int b = nbig - 1; b >= 0; --b) {
        hipLaunchKernelGGL((k_wb_far<C, false>), dim3(nchunks, kWbBig / 32), dim3(256), 0, s, sys, chunks, F, g,
                           X, Dfar, b);
        hipLaunchKernelGGL((k_wb_near<C, false>), dim3(nchunks), dim3(256), 0, s, sys, chunks, F, g, X, Dfar, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t wb_form(const DevPencil& P, const BandSys* sys, int nsys, void* F, bool fp32, hipStream_t s) {
    return fp32 ? wb_form_t<float2>(P, sys, nsys, (float2*)F, s) : wb_form_t<double2>(P, sys, nsys, (double2*)F, s);
}

hipError_t wb_step(const BandSys* sys, int nsys, int bwmax, void* F, bool fp32, int k0, int nmax,
                   int32_t* flag, hipStream_t s) {
    return fp32 ? wb_step_t<float2>(sys, nsys, bwmax, (float2*)F, k0, nmax, flag, s)
                : wb_step_t<double2>(sys, nsys, bwmax, (double2*)F, k0, nmax, flag, s);
}

hipError_t wb_solve(const BandSys* sys, const WbChunk* chunks, int nchunks, const void* F, bool fp32,
                    const TileGeom& g, void* X, int nmax, void* Dfar, hipStream_t s) {
    return fp32 ? wb_solve_t<float2>(sys, chunks, nchunks, (const float2*)F, g, (float2*)X, nmax, (float2*)Dfar, s)
                : wb_solve_t<double2>(sys, chunks, nchunks, (const double2*)F, g, (double2*)X, nmax,
                                      (double2*)Dfar, s);
}

size_t wb_scratch_bytes(int nchunks) { return sizeof(double2) * (size_t)nchunks * kWbBig * 16; }

hipError_t wb_narrow(const BandSys* sys, const WbChunk* chunks, int nchunks, const TileGeom& g,
                     const double2* Sx, float2* D, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wb_narrow, dim3(64, nchunks), dim3(256), 0, s, sys, chunks, g, Sx, D);
    return hipGetLastError();
}

hipError_t wb_accumulate(const BandSys* sys, const WbChunk* chunks, int nchunks, const TileGeom& g,
                         const void* D, bool fp32, double2* X, int set, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_wb_accumulate<float2>, dim3(64, nchunks), dim3(256), 0, s, sys, chunks, g,
                           (const float2*)D, X, set);
    else
        hipLaunchKernelGGL(k_wb_accumulate<double2>, dim3(64, nchunks), dim3(256), 0, s, sys, chunks, g,
                           (const double2*)D, X, set);
    return hipGetLastError();
}

}  // namespace gep
