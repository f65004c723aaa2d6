// Sparse matrix x multivector kernels for the shifted systems of the
// quadrature equation, (z_j B - A) Y_j = B V, on the packed union pattern.
//
// Complex kernels work on the tiled layout: a tile holds 64 columns of an
// n x W multivector, element (i, c) at ((c / 64) * n + i) * 64 + c % 64.
// One wavefront owns one row at a time for one tile: the row's CSR entries
// are wave-uniform (scalar loads), each lane gathers its column's 16-byte
// complex value, so every gather is a fully coalesced 1 KiB segment.
// A x and B x are accumulated separately and combined once per row as
// y = z (B x) - (A x): 8 flops per stored entry and column.
#include "internal.h"

namespace gep {

template <typename VT>
struct CplxTraits;
template <>
struct CplxTraits<double2> {
    using R = double;
    using M = double2;
};
template <>
struct CplxTraits<float2> {
    using R = float;
    using M = float2;
};

template <typename VT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_shifted(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const typename CplxTraits<VT>::M* __restrict__ ab, int n, const double2* __restrict__ shifts,
    const VT* __restrict__ X, VT* __restrict__ Y, const int32_t* __restrict__ tiles,
    const int32_t* __restrict__ n_active, int nrb, int rpb, double2* __restrict__ partial) {
    using R = typename CplxTraits<VT>::R;
    using M = typename CplxTraits<VT>::M;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int slot = lb / nrb;
    const int rb = lb - slot * nrb;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t base = (size_t)tile * (size_t)n * kTile;
    const VT* __restrict__ Xt = X + base;
    VT* __restrict__ Yt = Y + base;
    const double2 zd = shifts[tile * kTile + lane];
    const R zr = (R)zd.x, zi = (R)zd.y;
    const int r0 = rb * rpb;
    const int r1 = min(n, r0 + rpb);
    double dr = 0.0, di = 0.0;
    for (int i = r0 + wave; i < r1; i += kWaves) {
        const int k0 = rowptr[i];
        const int k1 = rowptr[i + 1];
        R ar = 0, ai = 0, br = 0, bi = 0;
        int k = k0;
        for (; k + 4 <= k1; k += 4) {
            const int j0 = colind[k], j1 = colind[k + 1], j2 = colind[k + 2], j3 = colind[k + 3];
            const M v0 = ab[k], v1 = ab[k + 1], v2 = ab[k + 2], v3 = ab[k + 3];
            const VT x0 = Xt[(size_t)j0 * kTile + lane];
            const VT x1 = Xt[(size_t)j1 * kTile + lane];
            const VT x2 = Xt[(size_t)j2 * kTile + lane];
            const VT x3 = Xt[(size_t)j3 * kTile + lane];
            ar = fma(v0.x, x0.x, ar); ai = fma(v0.x, x0.y, ai);
            br = fma(v0.y, x0.x, br); bi = fma(v0.y, x0.y, bi);
            ar = fma(v1.x, x1.x, ar); ai = fma(v1.x, x1.y, ai);
            br = fma(v1.y, x1.x, br); bi = fma(v1.y, x1.y, bi);
            ar = fma(v2.x, x2.x, ar); ai = fma(v2.x, x2.y, ai);
            br = fma(v2.y, x2.x, br); bi = fma(v2.y, x2.y, bi);
            ar = fma(v3.x, x3.x, ar); ai = fma(v3.x, x3.y, ai);
            br = fma(v3.y, x3.x, br); bi = fma(v3.y, x3.y, bi);
        }
        for (; k < k1; ++k) {
            const int j = colind[k];
            const M v = ab[k];
            const VT x = Xt[(size_t)j * kTile + lane];
            ar = fma(v.x, x.x, ar); ai = fma(v.x, x.y, ai);
            br = fma(v.y, x.x, br); bi = fma(v.y, x.y, bi);
        }
        VT y;
        y.x = fma(zr, br, fma(-zi, bi, -ar));
        y.y = fma(zr, bi, fma(zi, br, -ai));
        Yt[(size_t)i * kTile + lane] = y;
        if (DOT) {
            const VT xo = Xt[(size_t)i * kTile + lane];
            dr += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
            di += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
        }
    }
    if (DOT) {
        __shared__ double2 red[kWaves][kTile];
        red[wave][lane] = make_double2(dr, di);
        __syncthreads();
        if (wave == 0) {
            double2 acc = red[0][lane];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) {
                acc.x += red[w][lane].x;
                acc.y += red[w][lane].y;
            }
            partial[((size_t)tile * nrb + rb) * kTile + lane] = acc;
        }
    }
}

template <typename VT>
static hipError_t launch_shifted(const DevPencil& P, const void* ab, const double2* shifts,
                                 const VT* X, VT* Y, const int32_t* tiles,
                                 const int32_t* n_active, int n_active_host, int nrb,
                                 double2* partial, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int n = (int)P.n;
    const int rpb = (n + nrb - 1) / nrb;
    const int grid = pad8(n_active_host * nrb);
    using M = typename CplxTraits<VT>::M;
    if (partial)
        hipLaunchKernelGGL((k_spmm_shifted<VT, true>), dim3(grid), dim3(kBlock), 0, s, P.rowptr,
                           P.colind, (const M*)ab, n, shifts, X, Y, tiles, n_active, nrb, rpb,
                           partial);
    else
        hipLaunchKernelGGL((k_spmm_shifted<VT, false>), dim3(grid), dim3(kBlock), 0, s, P.rowptr,
                           P.colind, (const M*)ab, n, shifts, X, Y, tiles, n_active, nrb, rpb,
                           partial);
    return hipGetLastError();
}

hipError_t launch_spmm_c64(const DevPencil& P, const double2* shifts, const double2* X,
                           double2* Y, const int32_t* tiles, const int32_t* n_active,
                           int n_active_host, int nrb, double2* partial, hipStream_t s) {
    return launch_shifted<double2>(P, P.ab, shifts, X, Y, tiles, n_active, n_active_host, nrb,
                                   partial, s);
}

hipError_t launch_spmm_c32(const DevPencil& P, const double2* shifts, const float2* X, float2* Y,
                           const int32_t* tiles, const int32_t* n_active, int n_active_host,
                           int nrb, double2* partial, hipStream_t s) {
    return launch_shifted<float2>(P, P.ab32, shifts, X, Y, tiles, n_active, n_active_host, nrb,
                                  partial, s);
}

// Real multivector product on row-major n x k blocks (leading dimension ld):
// YA = A X, YB = B X.  The work-group's waves take consecutive rows of one
// 64-column chunk.
__global__ __launch_bounds__(kBlock) void k_spmm_real(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const double2* __restrict__ ab, int row0,
                                                      int n, const double* __restrict__ X, int k,
                                                      int64_t ld, double* __restrict__ YA,
                                                      double* __restrict__ YB, int nrb, int rpb) {
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int chunk = lb / nrb;
    const int rb = lb - chunk * nrb;
    const int nchunks = (k + kTile - 1) / kTile;
    if (chunk >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = chunk * kTile + lane;
    const bool ok = col < k;
    const int r0 = rb * rpb;
    const int r1 = min(n, r0 + rpb);
    for (int i = r0 + wave; i < r1; i += kWaves) {
        const int k0 = rowptr[row0 + i];
        const int k1 = rowptr[row0 + i + 1];
        double sa = 0.0, sb = 0.0;
        for (int e = k0; e < k1; ++e) {
            const int j = colind[e] - row0;
            const double2 v = ab[e];
            const double x = ok ? X[(size_t)j * ld + col] : 0.0;
            sa = fma(v.x, x, sa);
            sb = fma(v.y, x, sb);
        }
        if (ok) {
            if (YA) YA[(size_t)i * ld + col] = sa;
            if (YB) YB[(size_t)i * ld + col] = sb;
        }
    }
}

hipError_t launch_spmm_real(const DevPencil& P, const double* X, int64_t k, int64_t ld,
                            double* YA, double* YB, hipStream_t s, int64_t row0, int64_t nloc) {
    const int n = (int)(nloc < 0 ? P.n : nloc);
    if (k <= 0 || n <= 0) return hipSuccess;
    const int nchunks = (int)((k + kTile - 1) / kTile);
    int nrb = (2048 + nchunks - 1) / nchunks;
    nrb = max(1, min(nrb, (n + 15) / 16));
    const int rpb = (n + nrb - 1) / nrb;
    const int grid = pad8(nchunks * nrb);
    hipLaunchKernelGGL(k_spmm_real, dim3(grid), dim3(kBlock), 0, s, P.rowptr, P.colind, P.ab,
                       (int)row0, n, X, (int)k, ld, YA, YB, nrb, rpb);
    return hipGetLastError();
}

}  // namespace gep
