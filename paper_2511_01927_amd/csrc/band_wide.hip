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
//   k_wb_update   the whole trailing window C -= W diag(d) W^T, lower
//                 triangle, 64 x 64 tiles on the matrix cores
//                 (v_mfma_f64_16x16x4 or v_mfma_f32_16x16x4).
// Solves on the tiled multivector, one work-group per chunk of at most 16
// columns of one system (k_wb_sweep): 32-row blocks, the block's coupling
// to the rows already solved (forward: the bw rows above; backward: the bw
// rows below) as a matrix-core product whose K dimension runs over those
// rows in 64-row tiles staged through LDS (the forward tile is read down
// the factor's columns, the backward one across them), then a triangular
// solve of the block.  The forward sweep leaves y = L^-1 b; the backward
// sweep divides by d on the fly.
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
// After panel [k0, k0 + kPanel): the window [w0, wend), w0 = k0 + kPanel,
// wend = min(n, w0 + bw), lower triangle, C[i, j] -= sum_k l_ik d_k l_jk.
// blockIdx.x: lower-triangular index of a 64 x 64 tile (bi >= bj);
// blockIdx.y: system.  Wave w forms D(j, i) for the tile's 16 columns j of
// block w and all 64 rows i (four 16-row blocks): A = W_j = l_jk d_k,
// B = l_ik, both staged in LDS with lanes running down band columns; the
// result registers run down a column of C, so the read-modify-write is
// coalesced.
template <typename C>
__global__ __launch_bounds__(256) void k_wb_update(const BandSys* __restrict__ sys, C* F, int k0) {
    using V = typename Mma<C>::V;
    __shared__ C Wi[64][kPanel + 1];
    __shared__ C Wj[64][kPanel + 1];
    const BandSys S = sys[blockIdx.y];
    const int w0 = k0 + kPanel;
    const int wend = min(S.n, k0 + kPanel + S.bw);
    if (w0 >= wend) return;
    const int x = blockIdx.x;
    int bi = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= x) ++bi;
    while (bi * (bi + 1) / 2 > x) --bi;
    const int bj = x - bi * (bi + 1) / 2;
    const int i0 = w0 + 64 * bi, j0 = w0 + 64 * bj;
    if (i0 >= wend) return;   // uniform
    const int ld = S.bw + 1;
    C* Fs = F + S.off;
    for (int idx = threadIdx.x; idx < 64 * kPanel; idx += blockDim.x) {
        const int r = idx & 63, kk = idx >> 6;
        const int k = k0 + kk;
        const int i = i0 + r, j = j0 + r;
        C wi = czero<C>(), wj = czero<C>();
        if (i < wend && i - k <= S.bw) wi = Fs[(int64_t)k * ld + (i - k)];
        if (j < wend && j - k <= S.bw) wj = cmulT(Fs[(int64_t)k * ld + (j - k)], Fs[(int64_t)k * ld]);
        Wi[r][kk] = wi;
        Wj[r][kk] = wj;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    V pre[4], pim[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        pre[rb] = V{0, 0, 0, 0};
        pim[rb] = V{0, 0, 0, 0};
    }
#pragma unroll
    for (int st = 0; st < kPanel / 4; ++st) {
        const int kk = 4 * st + (lane >> 4);
        const C a = Wj[wave * 16 + (lane & 15)][kk];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) cmma<C>(a, Wi[rb * 16 + (lane & 15)][kk], pre[rb], pim[rb]);
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + wave * 16 + Mma<C>::row(lane, v);
            const int i = i0 + rb * 16 + (lane & 15);
            if (j >= wend || i >= wend || i < j) continue;
            C& c = Fs[(int64_t)j * ld + (i - j)];
            c.x -= pre[rb][v];
            c.y -= pim[rb][v];
        }
}

// ---- blocked sweeps --------------------------------------------------------------
// One work-group (4 waves) per chunk: up to 16 consecutive columns of one
// system inside one tile of the multivector X (element (i, c) of the chunk
// at base + i * 64 + lane0 + c, base the tile's).  Blocks of 32 rows, in
// order (forward) or in reverse (backward).  For block rows [i0, i0 + 32):
//   forward:  D(i, c) = sum_{j < i0} l_ij y_jc, then y_i = b_i - D_i -
//             sum_{i0 <= j < i} l_ij y_j;
//   backward: D(i, c) = sum_{j >= i0 + 32} l_ji x_jc, then x_i = y_i / d_i -
//             D_i - sum_{i < j < i0 + 32} l_ji x_j.
// The K dimension of D runs over 64-row tiles of the coupled rows; a tile of
// L (64 x 32) is staged in LDS as Lt[k][i] (forward: l_{i0+i, j0+k}, read
// down the factor's columns j; backward: l_{j0+k, i0+i}, read down columns
// i), and the four waves take interleaved K steps of 4, their partial D
// summed through LDS.  The block's triangle is solved by 16 lanes, one per
// column, from LDS.
template <typename C, bool FWD>
__global__ __launch_bounds__(256) void k_wb_sweep(const BandSys* __restrict__ sys,
                                                  const WbChunk* __restrict__ chunks,
                                                  const C* __restrict__ F, TileGeom geom,
                                                  C* __restrict__ X) {
    using R = typename Real<C>::T;
    using V = typename Mma<C>::V;
    __shared__ C Lt[64][33];
    __shared__ C Ld[32][33];      // Ld[r][q] = l_{i0+r, i0+q}, q < r; Ld[r][r] = d
    __shared__ C part[4][32][16];
    __shared__ C rhs[32][16];
    const WbChunk ch = chunks[blockIdx.x];
    const BandSys S = sys[ch.sys];
    const int n = S.n, bw = S.bw, ld = bw + 1;
    const C* Fs = F + S.off;
    C* Xc = X + geom.base[ch.tile] + ch.lane0;   // element (i, c) at Xc[i * 64 + c]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int cb = lane & 15;
    const bool cok = cb < ch.cnt;
    const int nblk = (n + 31) / 32;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = FWD ? bb : nblk - 1 - bb;
        const int i0 = blk * 32;
        const int rows = min(32, n - i0);
        const int jlo = FWD ? max(0, i0 - bw) : i0 + 32;
        const int jhi = FWD ? i0 : min(n, i0 + rows + bw);
        V re[2], im[2];
        re[0] = re[1] = im[0] = im[1] = V{0, 0, 0, 0};
        for (int j0 = jlo; j0 < jhi; j0 += 64) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = t + 256 * q;
                int k, i;
                if (FWD) {
                    k = e >> 5;
                    i = e & 31;
                } else {
                    i = e >> 6;
                    k = e & 63;
                }
                const int j = j0 + k, r = i0 + i;
                C v = czero<C>();
                if (FWD) {
                    if (j < jhi && i < rows && r - j <= bw) v = Fs[(int64_t)j * ld + (r - j)];
                } else {
                    if (j < jhi && i < rows && j - r <= bw) v = Fs[(int64_t)r * ld + (j - r)];
                }
                Lt[k][i] = v;
            }
            __syncthreads();
#pragma unroll
            for (int s = wave; s < 16; s += 4) {
                const int k = 4 * s + (lane >> 4);
                const C xb = (j0 + k < jhi && cok) ? Xc[(int64_t)(j0 + k) * 64 + cb] : czero<C>();
#pragma unroll
                for (int h = 0; h < 2; ++h) cmma<C>(Lt[k][16 * h + (lane & 15)], xb, re[h], im[h]);
            }
        }
        // A(i, k) = Lt[k][16 h + i], B(k, c) = X rows: register v of lane l
        // holds D(16 h + row(l, v), c = l % 16); the waves' partials go to LDS
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[wave][16 * h + Mma<C>::row(lane, v)][lane & 15] = mkc<C>(re[h][v], im[h][v]);
        // diagonal block and right-hand sides
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int col = e >> 5, r = e & 31;   // Ld[r][col] = l_{i0+r, i0+col}
            C v = czero<C>();
            if (r >= col && r < rows && col < rows && r - col <= bw) v = Fs[(int64_t)(i0 + col) * ld + (r - col)];
            Ld[r][col] = v;
        }
        for (int e = t; e < 32 * 16; e += 256) {
            const int r = e >> 4, c = e & 15;
            rhs[r][c] = (r < rows && c < ch.cnt) ? Xc[(int64_t)(i0 + r) * 64 + c] : czero<C>();
        }
        __syncthreads();
        if (t < 16) {
            const int c = t;
            if (FWD) {
                for (int r = 0; r < rows; ++r) {
                    C v = rhs[r][c];
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        v.x -= part[w][r][c].x;
                        v.y -= part[w][r][c].y;
                    }
                    for (int q = 0; q < r; ++q) cfmsT(v, Ld[r][q], rhs[q][c]);
                    rhs[r][c] = v;
                }
            } else {
                for (int r = rows - 1; r >= 0; --r) {
                    const C d = Ld[r][r];
                    const R m2 = d.x * d.x + d.y * d.y;
                    C v = cmulT(rhs[r][c], mkc<C>(d.x / m2, -d.y / m2));
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        v.x -= part[w][r][c].x;
                        v.y -= part[w][r][c].y;
                    }
                    for (int q = r + 1; q < rows; ++q) cfmsT(v, Ld[q][r], rhs[q][c]);
                    rhs[r][c] = v;
                }
            }
        }
        __syncthreads();
        for (int e = t; e < 32 * 16; e += 256) {
            const int r = e >> 4, c = e & 15;
            if (r < rows && c < ch.cnt) Xc[(int64_t)(i0 + r) * 64 + c] = rhs[r][c];
        }
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

template <typename C>
static hipError_t wb_step_t(const BandSys* sys, int nsys, int bwmax, C* F, int k0, int nmax, int32_t* flag,
                            hipStream_t s) {
    const int chunks = std::max(1, (bwmax + kWbRows - 1) / kWbRows);
    hipLaunchKernelGGL(k_wb_panel<C>, dim3(chunks, nsys), dim3(256), 0, s, sys, F, k0, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || k0 + kPanel >= nmax || bwmax == 0) return e;
    const int T = (bwmax + 63) / 64;
    hipLaunchKernelGGL(k_wb_update<C>, dim3(T * (T + 1) / 2, nsys), dim3(256), 0, s, sys, F, k0);
    return hipGetLastError();
}

template <typename C>
static hipError_t wb_solve_t(const BandSys* sys, const WbChunk* chunks, int nchunks, const C* F,
                             const TileGeom& g, C* X, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_wb_sweep<C, true>), dim3(nchunks), dim3(256), 0, s, sys, chunks, F, g, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_wb_sweep<C, false>), dim3(nchunks), dim3(256), 0, s, sys, chunks, F, g, X);
    return hipGetLastError();
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
                    const TileGeom& g, void* X, hipStream_t s) {
    return fp32 ? wb_solve_t<float2>(sys, chunks, nchunks, (const float2*)F, g, (float2*)X, s)
                : wb_solve_t<double2>(sys, chunks, nchunks, (const double2*)F, g, (double2*)X, s);
}

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
