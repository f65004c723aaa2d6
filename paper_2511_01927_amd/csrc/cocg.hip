// Batched Jacobi-preconditioned COCG for the complex symmetric shifted
// systems (z_j B - A) y = b of the quadrature equation (paper Appendix,
// "Numerical Quadrature": the N_q shifted solves are the dominant cost and
// are independent).  Every column of the tiled multivector is its own
// system (one node z_c, one right-hand side); all columns advance together.
//
// Conjugate-orthogonal CG (bilinear form x^T y) is carried in "u-form": the
// preconditioned residual u = D^-1 r is stored instead of r
// (D = z diag(B) - diag(A)), so r^T u = sum D u^2 and ||r|| = ||D u|| need
// no division.  One iteration is two streaming kernels:
//
//   A  p' = u + beta p (formed on the fly for every gathered neighbour),
//      q = K p' (K = z B - A), store p', partials of p'^T q      [3 passes]
//   B  recompute K p' (gather p'), x += alpha p', u -= alpha D^-1 K p',
//      partials of D u^2 and |D u|^2                              [5 passes]
//
// Both walk the pencil in row groups (see group_walk below) so that
// neighbours shared by consecutive rows are gathered once.
//
// plus three tiny kernels: alpha = rho / p'^T q; beta = rho'/rho with the
// per-column convergence test ||r|| <= tol ||b||; active-tile compaction.
// p is double-buffered because neighbours gather the old p while p' is
// written.  Dot products: each lane owns one column, a wave sums its rows in
// registers, the work-group's waves combine in LDS, and per-tile partials
// over row blocks are summed in a fixed order (deterministic).
//
// The kernels are templated on the storage type: double2 (FP64 path) or
// float2 (mixed path, FP32 recurrence; FP64 scalars, dots and the residual
// replacement of cocg32 kernels below).
#include "internal.h"

namespace gep {

template <typename VT>
struct Cx;
template <>
struct Cx<double2> {
    using R = double;
    using M = double2;
};
template <>
struct Cx<float2> {
    using R = float;
    using M = float2;
};

__device__ inline double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

struct BlockMap {
    int slot, rb, tile, lane, wave, r0, r1, row0;
    int64_t base;   // element offset of the tile's row 0
    int64_t goff;   // base - row0 * 64: offset of global row j is goff + j * 64
};

// Work-group -> (active tile, row block).  Rows are local to the tile's
// pencil; row blocks past the tile's row count run with an empty range so
// that every partial slot is written.
__device__ inline bool map_block(const int32_t* tiles, const int32_t* n_active, int nrb, int rpb,
                                 const TileGeom& g, BlockMap& m) {
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    m.slot = lb / nrb;
    m.rb = lb - m.slot * nrb;
    if (m.slot >= n_active[0]) return false;
    m.tile = tiles[m.slot];
    m.lane = threadIdx.x & 63;
    m.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nt = g.n[m.tile];
    m.row0 = g.row0[m.tile];
    m.base = g.base[m.tile];
    m.goff = m.base - (int64_t)m.row0 * kTile;
    m.r0 = min(nt, m.rb * rpb);
    m.r1 = min(nt, m.r0 + rpb);
    return true;
}

// Sum a per-lane double2 and double over the work-group's waves and store the partials.
__device__ inline void block_partials(const BlockMap& m, int nrb, double2 c, double d,
                                      double2* part_c, double* part_r) {
    __shared__ double2 rc[kWaves][kTile];
    __shared__ double rd[kWaves][kTile];
    rc[m.wave][m.lane] = c;
    rd[m.wave][m.lane] = d;
    __syncthreads();
    if (m.wave == 0) {
        double2 ac = rc[0][m.lane];
        double ad = rd[0][m.lane];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            ac.x += rc[w][m.lane].x;
            ac.y += rc[w][m.lane].y;
            ad += rd[w][m.lane];
        }
        const size_t o = ((size_t)m.tile * nrb + m.rb) * kTile + m.lane;
        part_c[o] = ac;
        if (part_r) part_r[o] = ad;
    }
}

template <typename R>
__device__ inline void cfma_acc(R va, R vb, R xr, R xi, R& ar, R& ai, R& br, R& bi) {
    ar = fma(va, xr, ar);
    ai = fma(va, xi, ai);
    br = fma(vb, xr, br);
    bi = fma(vb, xi, bi);
}

// x = 0, u = D^-1 b, p = 0 (with beta = 0 the first kernel A forms p' = u);
// partials of rho = b^T u and ||b||^2.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_init(TileGeom geom, const double* __restrict__ dA,
                                                 const double* __restrict__ dB,
                                                 const double2* __restrict__ shifts,
                                                 const int64_t* __restrict__ bsrc,
                                                 const double* __restrict__ BV, int64_t ldbv,
                                                 VT* __restrict__ x, VT* __restrict__ u,
                                                 VT* __restrict__ p,
                                                 const int32_t* __restrict__ tiles,
                                                 const int32_t* __restrict__ n_active, int nrb,
                                                 int rpb, double2* part_c, double* part_r) {
    using R = typename Cx<VT>::R;
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, geom, m)) return;
    const int col = m.tile * kTile + m.lane;
    const int64_t bs = bsrc[col];
    const double2 z = shifts[col];
    const int64_t base = m.base;
    double2 rho = make_double2(0.0, 0.0);
    double bb = 0.0;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const int g = m.row0 + i;
        const double b = bs >= 0 ? BV[bs + (int64_t)i * ldbv] : 0.0;
        const double2 D = make_double2(z.x * dB[g] - dA[g], z.y * dB[g]);
        const double2 uv = cdiv(make_double2(b, 0.0), D);
        const size_t o = base + (size_t)i * kTile + m.lane;
        VT zero;
        zero.x = (R)0;
        zero.y = (R)0;
        VT us;
        us.x = (R)uv.x;
        us.y = (R)uv.y;
        x[o] = zero;
        u[o] = us;
        p[o] = zero;
        rho.x += b * uv.x;
        rho.y += b * uv.y;
        bb += b * b;
    }
    block_partials(m, nrb, rho, bb, part_c, part_r);
}

// Row groups.  The pencil is also stored as a sequence of groups of R
// consecutive rows (never crossing a pencil of a batch): group k holds the
// sorted union of its rows' column indices, gcol[gptr[k] .. gptr[k+1]), and
// an R-wide coefficient block gab[c * R + r] = (a, b) of row r at column
// gcol[c], zero where row r has no entry.  A wave walks the union once and
// applies every gathered neighbour to all R rows, so a neighbour shared by
// consecutive rows is loaded once instead of once per row (R = 4 halves the
// gathers of a 2D nine-point pattern).  Per row the nonzero terms are added
// in ascending column order, as a CSR walk would, and the zero padding adds
// exact zeros, so every row's K p' is the same for any R (the dot-product
// partials follow the rows each wave owns, so their rounding does not).
// R = 1 is plain CSR.
// Every row holds its diagonal (B has a positive diagonal), so the union of a
// group contains the group's own rows and their values are picked up on the
// way instead of being loaded again.
template <typename VT, int R>
struct GroupAcc {
    using Rt = typename Cx<VT>::R;
    Rt ar[R], ai[R], br[R], bi[R];
    VT own[R];
    __device__ void clear() {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ar[r] = ai[r] = br[r] = bi[r] = 0;
            own[r].x = 0;
            own[r].y = 0;
        }
    }
};

// Chunk of union columns loaded together (more loads in flight per wave).
constexpr int kChunk = 3;

// Streaming (non-temporal) access for vectors that are touched once per
// kernel, so that they do not push the gathered neighbour rows out of L2.
template <typename VT>
__device__ inline VT nt_load(const VT* p) {
    VT v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}
template <typename VT>
__device__ inline void nt_store(VT* p, VT v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Walk group k's union: for each column j, v = fetch(j) (the gathered value),
// accumulate A v and B v into every row of the group, and keep v for the
// group's own rows.  grow is the group's first global row.
template <typename VT, int R, typename F>
__device__ inline void group_walk(const int32_t* __restrict__ gcol,
                                  const typename Cx<VT>::M* __restrict__ gab, int c0, int c1,
                                  int grow, GroupAcc<VT, R>& acc, F fetch) {
    using M = typename Cx<VT>::M;
    for (int c = c0; c < c1; c += kChunk) {
        int j[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) j[t] = gcol[min(c + t, c1 - 1)];
        VT v[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) v[t] = fetch(j[t]);
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const bool ok = c + t < c1;
            const int cc = ok ? c + t : c1 - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                M w = gab[(size_t)cc * R + r];
                if (!ok) w.x = w.y = 0;
                cfma_acc(w.x, w.y, v[t].x, v[t].y, acc.ar[r], acc.ai[r], acc.br[r], acc.bi[r]);
                if (j[t] == grow + r) acc.own[r] = v[t];
            }
        }
    }
}

// Kernel A: p' = u + beta p, q = K p', store p', partials of p'^T q.
template <typename VT, int R>
__global__ __launch_bounds__(kBlock) void k_spmm_dir(
    const int32_t* __restrict__ gptr, const int32_t* __restrict__ gcol,
    const typename Cx<VT>::M* __restrict__ gab, TileGeom geom, const double2* __restrict__ shifts,
    const double2* __restrict__ beta, const VT* __restrict__ U, const VT* __restrict__ P,
    VT* __restrict__ Pn, const int32_t* __restrict__ tiles, const int32_t* __restrict__ n_active,
    int nrb, int rpb, double2* __restrict__ part_c) {
    using Rt = typename Cx<VT>::R;
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, geom, m)) return;
    const int col = m.tile * kTile + m.lane;
    // offsets below are global row indices of the concatenated pencil
    const VT* __restrict__ Ut = U + m.goff;
    const VT* __restrict__ Pt = P + m.goff;
    VT* __restrict__ Pnt = Pn + m.goff;
    const double2 zd = shifts[col];
    const double2 bd = beta[col];
    const Rt zr = (Rt)zd.x, zi = (Rt)zd.y, br_ = (Rt)bd.x, bi_ = (Rt)bd.y;
    const int gbase = geom.g0[m.tile];
    double dr = 0.0, di = 0.0;
    // r0 is a multiple of R except for row blocks past the pencil's end,
    // where r0 = r1 = n and the range below is empty
    const int k_end = (m.r1 + R - 1) / R;
    for (int k = (m.r0 + R - 1) / R + m.wave; k < k_end; k += kWaves) {
        const int gk = gbase + k;
        const int grow = m.row0 + k * R;
        GroupAcc<VT, R> acc;
        acc.clear();
        group_walk<VT, R>(gcol, gab, gptr[gk], gptr[gk + 1], grow, acc, [&](int j) {
            const VT uj = Ut[(size_t)j * kTile + m.lane], pj = Pt[(size_t)j * kTile + m.lane];
            VT x;
            x.x = uj.x + br_ * pj.x - bi_ * pj.y;
            x.y = uj.y + br_ * pj.y + bi_ * pj.x;
            return x;
        });
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (k * R + r >= m.r1) break;
            const VT pn = acc.own[r];
            nt_store(&Pnt[(size_t)(grow + r) * kTile + m.lane], pn);
            const Rt qr = fma(zr, acc.br[r], fma(-zi, acc.bi[r], -acc.ar[r]));
            const Rt qi = fma(zr, acc.bi[r], fma(zi, acc.br[r], -acc.ai[r]));
            dr += (double)pn.x * (double)qr - (double)pn.y * (double)qi;
            di += (double)pn.x * (double)qi + (double)pn.y * (double)qr;
        }
    }
    block_partials(m, nrb, make_double2(dr, di), 0.0, part_c, nullptr);
}

// Kernel B: q = K p (recomputed), x += alpha p, u -= alpha D^-1 q,
// partials of rho' = sum D u^2 and ||D u||^2.
template <typename VT, int R>
__global__ __launch_bounds__(kBlock) void k_update(
    const int32_t* __restrict__ gptr, const int32_t* __restrict__ gcol,
    const typename Cx<VT>::M* __restrict__ gab, TileGeom geom, const double* __restrict__ dA,
    const double* __restrict__ dB, const double2* __restrict__ shifts,
    const double2* __restrict__ alpha, VT* __restrict__ X, VT* __restrict__ U,
    const VT* __restrict__ P, const int32_t* __restrict__ tiles,
    const int32_t* __restrict__ n_active, int nrb, int rpb, double2* __restrict__ part_c,
    double* __restrict__ part_r) {
    using Rt = typename Cx<VT>::R;
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, geom, m)) return;
    const int col = m.tile * kTile + m.lane;
    VT* __restrict__ Xt = X + m.goff;
    VT* __restrict__ Ut = U + m.goff;
    const VT* __restrict__ Pt = P + m.goff;
    const double2 zd = shifts[col];
    const double2 ad = alpha[col];
    const Rt zr = (Rt)zd.x, zi = (Rt)zd.y, alr = (Rt)ad.x, ali = (Rt)ad.y;
    const int gbase = geom.g0[m.tile];
    double2 rho = make_double2(0.0, 0.0);
    double rr = 0.0;
    // r0 is a multiple of R except for row blocks past the pencil's end,
    // where r0 = r1 = n and the range below is empty
    const int k_end = (m.r1 + R - 1) / R;
    for (int k = (m.r0 + R - 1) / R + m.wave; k < k_end; k += kWaves) {
        const int gk = gbase + k;
        const int grow = m.row0 + k * R;
        GroupAcc<VT, R> acc;
        acc.clear();
        group_walk<VT, R>(gcol, gab, gptr[gk], gptr[gk + 1], grow, acc,
                          [&](int j) { return Pt[(size_t)j * kTile + m.lane]; });
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (k * R + r >= m.r1) break;
            const int g = grow + r;
            const Rt qr = fma(zr, acc.br[r], fma(-zi, acc.bi[r], -acc.ar[r]));
            const Rt qi = fma(zr, acc.bi[r], fma(zi, acc.br[r], -acc.ai[r]));
            const size_t o = (size_t)g * kTile + m.lane;
            const VT pi = acc.own[r];
            VT xv = nt_load(&Xt[o]), uv = nt_load(&Ut[o]);
            xv.x = fma(alr, pi.x, fma(-ali, pi.y, xv.x));
            xv.y = fma(alr, pi.y, fma(ali, pi.x, xv.y));
            // s = alpha q / D, one reciprocal of |D|^2 per row and column
            const double2 D = make_double2(zd.x * dB[g] - dA[g], zd.y * dB[g]);
            const Rt aqr = alr * qr - ali * qi, aqi = alr * qi + ali * qr;
            const double inv = 1.0 / (D.x * D.x + D.y * D.y);
            const double sx = ((double)aqr * D.x + (double)aqi * D.y) * inv;
            const double sy = ((double)aqi * D.x - (double)aqr * D.y) * inv;
            uv.x = uv.x - (Rt)sx;
            uv.y = uv.y - (Rt)sy;
            nt_store(&Xt[o], xv);
            nt_store(&Ut[o], uv);
            // r = D u
            const double ux = (double)uv.x, uy = (double)uv.y;
            const double rx = D.x * ux - D.y * uy, ry = D.x * uy + D.y * ux;
            rho.x += rx * ux - ry * uy;
            rho.y += rx * uy + ry * ux;
            rr += rx * rx + ry * ry;
        }
    }
    block_partials(m, nrb, rho, rr, part_c, part_r);
}

// First level of the per-tile sums: work-group (slot, g) adds row blocks
// [g * chunk, (g + 1) * chunk) of the active tile's partials into part2
// [tile][g][64], so the per-column kernels below only sum G entries.
__global__ __launch_bounds__(kBlock) void k_fold_partials(int nrb, int G,
                                                          const int32_t* __restrict__ tiles,
                                                          const int32_t* __restrict__ n_active,
                                                          const double2* __restrict__ part_c,
                                                          const double* __restrict__ part_r,
                                                          double2* __restrict__ part2_c,
                                                          double* __restrict__ part2_r) {
    __shared__ double2 sc[kWaves][kTile];
    __shared__ double sr[kWaves][kTile];
    const int slot = blockIdx.x / G;
    const int g = blockIdx.x - slot * G;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int chunk = (nrb + G - 1) / G;
    const int r0 = g * chunk, r1 = min(nrb, r0 + chunk);
    double2 a = make_double2(0.0, 0.0);
    double d = 0.0;
    for (int rb = r0 + wave; rb < r1; rb += kWaves) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        const double2 v = part_c[o];
        a.x += v.x;
        a.y += v.y;
        if (part_r) d += part_r[o];
    }
    sc[wave][lane] = a;
    sr[wave][lane] = d;
    __syncthreads();
    if (wave) return;
    for (int w = 1; w < kWaves; ++w) {
        a.x += sc[w][lane].x;
        a.y += sc[w][lane].y;
        d += sr[w][lane];
    }
    const size_t o = ((size_t)tile * G + g) * kTile + lane;
    part2_c[o] = a;
    if (part_r) part2_r[o] = d;
}

// After k_init: rho, ||b||^2, activity per column and per tile.
__global__ __launch_bounds__(kBlock) void k_reduce_init(int nrb, const double2* __restrict__ part_c,
                                                        const double* __restrict__ part_r,
                                                        double2* __restrict__ rho,
                                                        double* __restrict__ bb,
                                                        double* __restrict__ rr,
                                                        double* __restrict__ rmax,
                                                        int32_t* __restrict__ flag,
                                                        double2* __restrict__ beta,
                                                        int32_t* __restrict__ active,
                                                        int32_t* __restrict__ iters,
                                                        double* __restrict__ rbest,
                                                        int32_t* __restrict__ stall,
                                                        int32_t* __restrict__ stalled,
                                                        int32_t* __restrict__ tile_active) {
    __shared__ double2 sc[kWaves][kTile];
    __shared__ double sr[kWaves][kTile];
    __shared__ int cnt;
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 a = make_double2(0.0, 0.0);
    double d = 0.0;
    for (int rb = wave; rb < nrb; rb += kWaves) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        a.x += part_c[o].x;
        a.y += part_c[o].y;
        d += part_r[o];
    }
    sc[wave][lane] = a;
    sr[wave][lane] = d;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w) {
            a.x += sc[w][lane].x;
            a.y += sc[w][lane].y;
            d += sr[w][lane];
        }
        const int col = tile * kTile + lane;
        rho[col] = a;
        bb[col] = d;
        rr[col] = d;
        rmax[col] = d;
        flag[col] = 0;
        rbest[col] = d;
        stall[col] = 0;
        stalled[col] = 0;
        beta[col] = make_double2(0.0, 0.0);
        iters[col] = 0;
        const int act = d > 0.0 ? 1 : 0;
        active[col] = act;
        if (act) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_active[tile] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_reduce_alpha(int nrb, const int32_t* __restrict__ tiles,
                                                         const int32_t* __restrict__ n_active,
                                                         const double2* __restrict__ part_c,
                                                         const double2* __restrict__ rho,
                                                         double2* __restrict__ alpha,
                                                         int32_t* __restrict__ active) {
    __shared__ double2 sc[kWaves][kTile];
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 pq = make_double2(0.0, 0.0);
    for (int rb = wave; rb < nrb; rb += kWaves) {
        const double2 v = part_c[((size_t)tile * nrb + rb) * kTile + lane];
        pq.x += v.x;
        pq.y += v.y;
    }
    sc[wave][lane] = pq;
    __syncthreads();
    if (wave) return;
    for (int w = 1; w < kWaves; ++w) {
        pq.x += sc[w][lane].x;
        pq.y += sc[w][lane].y;
    }
    const int col = tile * kTile + lane;
    double2 a = make_double2(0.0, 0.0);
    if (active[col]) {
        const double m2 = pq.x * pq.x + pq.y * pq.y;
        if (m2 > 0.0 && isfinite(m2)) {
            a = cdiv(rho[col], pq);
        } else {
            active[col] = 0;   // breakdown: p^T K p = 0
        }
    }
    alpha[col] = a;
}

__global__ __launch_bounds__(kBlock) void k_reduce_beta(
    int nrb, const int32_t* __restrict__ tiles, const int32_t* __restrict__ n_active,
    const double2* __restrict__ part_c, const double* __restrict__ part_r,
    double2* __restrict__ rho, double2* __restrict__ beta, const double* __restrict__ bb,
    double* __restrict__ rr, double* __restrict__ rmax, int32_t* __restrict__ flag,
    int32_t* __restrict__ active, int32_t* __restrict__ iters, int32_t* __restrict__ tile_active,
    int32_t* __restrict__ stalled, double tol2, int max_iter, int hold) {
    __shared__ double2 sc[kWaves][kTile];
    __shared__ double sr[kWaves][kTile];
    __shared__ int cnt;
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 rn = make_double2(0.0, 0.0);
    double s = 0.0;
    for (int rb = wave; rb < nrb; rb += kWaves) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        rn.x += part_c[o].x;
        rn.y += part_c[o].y;
        s += part_r[o];
    }
    sc[wave][lane] = rn;
    sr[wave][lane] = s;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w) {
            rn.x += sc[w][lane].x;
            rn.y += sc[w][lane].y;
            s += sr[w][lane];
        }
        const int col = tile * kTile + lane;
        int a = active[col];
        double2 b = make_double2(0.0, 0.0);
        if (a) {
            const int it = iters[col] + 1;
            iters[col] = it;
            rr[col] = s;
            const double2 ro = rho[col];
            const double m2 = ro.x * ro.x + ro.y * ro.y;
            const bool conv = s <= tol2 * bb[col];
            if (hold) {
                // mixed path: ask for a residual replacement once the recursive
                // residual fell by 10x since the last one, or reached tol
                const double mx = fmax(rmax[col], s);
                rmax[col] = mx;
                if (conv || s <= 1e-2 * mx) flag[col] = 1;
            }
            if ((conv && !hold) || it >= max_iter || !(m2 > 0.0) || !isfinite(s)) {
                a = 0;
                active[col] = 0;
                // the FP32 recurrence ran out of iterations or broke down:
                // the FP64 completion takes the column over
                if (hold && !conv) stalled[col] = 1;
            } else {
                b = cdiv(rn, ro);
                rho[col] = rn;
            }
        }
        beta[col] = b;
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_active[tile] = cnt;
}

// Compacts the list of tiles that still have an active column; counts[0] =
// active tiles, counts[1] = active columns.  One work-group of 1024 threads.
__global__ __launch_bounds__(1024) void k_compact(int ntiles, const int32_t* __restrict__ tile_active,
                                                  int32_t* __restrict__ tiles,
                                                  int32_t* __restrict__ counts) {
    __shared__ int scan[1024];
    __shared__ int base_s, cols_s;
    const int t = threadIdx.x;
    if (t == 0) {
        base_s = 0;
        cols_s = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < ntiles; c0 += 1024) {
        const int idx = c0 + t;
        const int cnt = idx < ntiles ? tile_active[idx] : 0;
        const int f = cnt > 0 ? 1 : 0;
        scan[t] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int v = t >= off ? scan[t - off] : 0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        if (f) tiles[base_s + scan[t] - 1] = idx;
        if (cnt) atomicAdd(&cols_s, cnt);
        __syncthreads();
        if (t == 0) base_s += scan[1023];
        __syncthreads();
    }
    if (t == 0) {
        counts[0] = base_s;
        counts[1] = cols_s;
    }
}

// ---- mixed precision: FP64 residual replacement ----------------------------
// (reliable updates: the FP32 recurrence keeps its search direction; every
// few iterations the FP32 correction is folded into the FP64 solution and
// the residual is recomputed in FP64 with the FP64 pencil.)

// x64 += x32, x32 = 0 on the active tiles.
__global__ __launch_bounds__(kBlock) void k_fold(TileGeom geom, double2* __restrict__ X64,
                                                 float2* __restrict__ X32,
                                                 const int32_t* __restrict__ tiles,
                                                 const int32_t* __restrict__ n_active, int nrb,
                                                 int rpb) {
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, geom, m)) return;
    const int64_t base = m.base;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const size_t o = base + (size_t)i * kTile + m.lane;
        const float2 c = X32[o];
        double2 xv = X64[o];
        xv.x += (double)c.x;
        xv.y += (double)c.y;
        X64[o] = xv;
        X32[o] = make_float2(0.f, 0.f);
    }
}

// r = b - K x64 in FP64, u = D^-1 r stored as UT (float2 for the mixed
// replacement, double2 for the FP64 completion) for the flagged columns;
// partials of r^T u and ||r||^2.
template <typename UT>
__global__ __launch_bounds__(kBlock) void k_true_residual(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const double2* __restrict__ ab, TileGeom geom, const double* __restrict__ dA,
    const double* __restrict__ dB, const double2* __restrict__ shifts,
    const int64_t* __restrict__ bsrc, const double* __restrict__ BV, int64_t ldbv,
    const double2* __restrict__ X64, UT* __restrict__ Uo, const int32_t* __restrict__ flag,
    const int32_t* __restrict__ tiles, const int32_t* __restrict__ n_active, int nrb, int rpb,
    double2* part_c, double* part_r) {
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, geom, m)) return;
    const int col = m.tile * kTile + m.lane;
    const bool fl = flag[col] != 0;
    // the decision is uniform over the work-group (all waves see the same 64 columns)
    if (!__any(fl)) {
        block_partials(m, nrb, make_double2(0.0, 0.0), 0.0, part_c, part_r);
        return;
    }
    const int64_t base = m.base;
    const double2* __restrict__ Xt = X64 + m.goff;
    const double2 z = shifts[col];
    const int64_t bs = bsrc[col];
    double2 rho = make_double2(0.0, 0.0);
    double rr = 0.0;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const int g = m.row0 + i;
        const int k0 = rowptr[g];
        const int k1 = rowptr[g + 1];
        double ar = 0, ai = 0, sbr = 0, sbi = 0;
        for (int k = k0; k < k1; ++k) {
            const int j = colind[k];
            const double2 v = ab[k];
            const double2 xj = Xt[(size_t)j * kTile + m.lane];
            cfma_acc(v.x, v.y, xj.x, xj.y, ar, ai, sbr, sbi);
        }
        const double b = bs >= 0 ? BV[bs + (int64_t)i * ldbv] : 0.0;
        const double rx = b - (z.x * sbr - z.y * sbi - ar);
        const double ry = -(z.x * sbi + z.y * sbr - ai);
        const double2 D = make_double2(z.x * dB[g] - dA[g], z.y * dB[g]);
        const double2 uv = cdiv(make_double2(rx, ry), D);
        if (fl) {
            UT us;
            us.x = (decltype(us.x))uv.x;
            us.y = (decltype(us.y))uv.y;
            Uo[base + (size_t)i * kTile + m.lane] = us;
            const double ux = (double)us.x, uy = (double)us.y;
            rho.x += rx * ux - ry * uy;
            rho.y += rx * uy + ry * ux;
            rr += rx * rx + ry * ry;
        }
    }
    block_partials(m, nrb, rho, rr, part_c, part_r);
}

// Replacements in a row without progress of the true residual after which a
// column leaves the FP32 recurrence for the FP64 completion.
constexpr int kStallLimit = 3;

// rho <- true r^T u, beta rescaled to rho_true / rho_old, convergence on the
// true residual.
__global__ __launch_bounds__(kBlock) void k_reduce_replace(
    int nrb, const int32_t* __restrict__ tiles, const int32_t* __restrict__ n_active,
    const double2* __restrict__ part_c, const double* __restrict__ part_r,
    double2* __restrict__ rho, double2* __restrict__ beta, const double* __restrict__ bb,
    double* __restrict__ rr, double* __restrict__ rmax, int32_t* __restrict__ flag,
    int32_t* __restrict__ active, int32_t* __restrict__ tile_active, double* __restrict__ rbest,
    int32_t* __restrict__ stall, int32_t* __restrict__ stalled, double tol2) {
    __shared__ double2 sc[kWaves][kTile];
    __shared__ double sr[kWaves][kTile];
    __shared__ int cnt;
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 rn = make_double2(0.0, 0.0);
    double s = 0.0;
    for (int rb = wave; rb < nrb; rb += kWaves) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        rn.x += part_c[o].x;
        rn.y += part_c[o].y;
        s += part_r[o];
    }
    sc[wave][lane] = rn;
    sr[wave][lane] = s;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w) {
            rn.x += sc[w][lane].x;
            rn.y += sc[w][lane].y;
            s += sr[w][lane];
        }
        const int col = tile * kTile + lane;
        int a = active[col];
        if (a && flag[col]) {
            flag[col] = 0;
            rr[col] = s;
            rmax[col] = s;
            const double2 rec = rho[col];
            const double m2 = rec.x * rec.x + rec.y * rec.y;
            // progress of the true residual between replacements: the FP32
            // recurrence is given up after kStallLimit replacements in a row
            // that did not reduce ||r||^2 by 4x below its best
            int st = stall[col];
            if (s < 0.25 * rbest[col]) {
                rbest[col] = s;
                st = 0;
            } else {
                ++st;
            }
            stall[col] = st;
            const bool done = s <= tol2 * bb[col];
            if (done || !isfinite(s) || !(m2 > 0.0) || st >= kStallLimit) {
                a = 0;
                active[col] = 0;
                beta[col] = make_double2(0.0, 0.0);
                if (!done) stalled[col] = 1;
            } else {
                // beta = rho_rec / rho_old was set by k_reduce_beta; rescale
                const double2 f = cdiv(rn, rec);
                const double2 b = beta[col];
                beta[col] = make_double2(b.x * f.x - b.y * f.y, b.x * f.y + b.y * f.x);
                rho[col] = rn;
            }
        }
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_active[tile] = cnt;
}


// FP64 completion: the stalled columns restart from their true residual
// (rho = r^T u, beta = 0) and become active again; everything else stays
// inactive.
__global__ __launch_bounds__(kBlock) void k_reduce_restart(
    int nrb, const int32_t* __restrict__ tiles, const int32_t* __restrict__ n_active,
    const double2* __restrict__ part_c, const double* __restrict__ part_r,
    double2* __restrict__ rho, double2* __restrict__ beta, const double* __restrict__ bb,
    double* __restrict__ rr, int32_t* __restrict__ stalled, int32_t* __restrict__ active,
    int32_t* __restrict__ tile_active, double tol2) {
    __shared__ double2 sc[kWaves][kTile];
    __shared__ double sr[kWaves][kTile];
    __shared__ int cnt;
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2 rn = make_double2(0.0, 0.0);
    double s = 0.0;
    for (int rb = wave; rb < nrb; rb += kWaves) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        rn.x += part_c[o].x;
        rn.y += part_c[o].y;
        s += part_r[o];
    }
    sc[wave][lane] = rn;
    sr[wave][lane] = s;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w) {
            rn.x += sc[w][lane].x;
            rn.y += sc[w][lane].y;
            s += sr[w][lane];
        }
        const int col = tile * kTile + lane;
        int a = 0;
        if (stalled[col]) {
            stalled[col] = 0;
            rr[col] = s;
            beta[col] = make_double2(0.0, 0.0);
            const double m2 = rn.x * rn.x + rn.y * rn.y;
            if (s > tol2 * bb[col] && isfinite(s) && m2 > 0.0) {
                a = 1;
                rho[col] = rn;
            }
        }
        active[col] = a;
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_active[tile] = cnt;
}

template <typename VT>
hipError_t launch_init_t(const DevPencil& P, CocgState& S, VT* x, VT* u, VT* p, const double* BV,
                         int64_t ldbv, int nrb, hipStream_t s) {
    const int rpb = S.rpb;
    const int grid = pad8(S.ntiles * nrb);
    hipLaunchKernelGGL((k_init<VT>), dim3(grid), dim3(kBlock), 0, s, S.geom, P.dA, P.dB, S.shifts,
                       S.bsrc, BV, ldbv, x, u, p, S.tiles, S.counts, nrb, rpb, S.part_c, S.part_r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_init, dim3(S.ntiles), dim3(kBlock), 0, s, nrb, S.part_c, S.part_r,
                       S.rho, S.bb, S.rr, S.rmax, S.flag, S.beta, S.active, S.iters, S.rbest,
                       S.stall, S.stalled, S.tile_active);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cocg_compact(S, s);
}

hipError_t cocg_init(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv, int nrb,
                     hipStream_t s) {
    return launch_init_t<double2>(P, S, S.x, S.u, S.p, BV, ldbv, nrb, s);
}

template <typename VT>
hipError_t launch_spmm_dir_t(const DevPencil& P, const void* gab, CocgState& S, const VT* u,
                             const VT* p, VT* pn, int n_active_host, int nrb, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int rpb = S.rpb;
    const int grid = pad8(n_active_host * nrb);
    using M = typename Cx<VT>::M;
    if (P.grp == 4)
        hipLaunchKernelGGL((k_spmm_dir<VT, 4>), dim3(grid), dim3(kBlock), 0, s, P.gptr, P.gcol,
                           (const M*)gab, S.geom, S.shifts, S.beta, u, p, pn, S.tiles, S.counts,
                           nrb, rpb, S.part_c);
    else
        hipLaunchKernelGGL((k_spmm_dir<VT, 1>), dim3(grid), dim3(kBlock), 0, s, P.gptr, P.gcol,
                           (const M*)gab, S.geom, S.shifts, S.beta, u, p, pn, S.tiles, S.counts,
                           nrb, rpb, S.part_c);
    return hipGetLastError();
}

template <typename VT>
hipError_t launch_update_t(const DevPencil& P, const void* gab, CocgState& S, VT* x, VT* u,
                           const VT* p, int n_active_host, int nrb, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int rpb = S.rpb;
    const int grid = pad8(n_active_host * nrb);
    using M = typename Cx<VT>::M;
    if (P.grp == 4)
        hipLaunchKernelGGL((k_update<VT, 4>), dim3(grid), dim3(kBlock), 0, s, P.gptr, P.gcol,
                           (const M*)gab, S.geom, P.dA, P.dB, S.shifts, S.alpha, x, u, p,
                           S.tiles, S.counts, nrb, rpb, S.part_c, S.part_r);
    else
        hipLaunchKernelGGL((k_update<VT, 1>), dim3(grid), dim3(kBlock), 0, s, P.gptr, P.gcol,
                           (const M*)gab, S.geom, P.dA, P.dB, S.shifts, S.alpha, x, u, p,
                           S.tiles, S.counts, nrb, rpb, S.part_c, S.part_r);
    return hipGetLastError();
}

hipError_t cocg_spmm_dir(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                         hipStream_t s) {
    return launch_spmm_dir_t<double2>(P, P.gab, S, S.u, S.p, S.pn, n_active_host, nrb, s);
}

hipError_t cocg_update(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                       hipStream_t s) {
    return launch_update_t<double2>(P, P.gab, S, S.x, S.u, S.pn, n_active_host, nrb, s);
}

hipError_t cocg32_init(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv, int nrb,
                       hipStream_t s) {
    return launch_init_t<float2>(P, S, S.x32, S.u32, S.p32, BV, ldbv, nrb, s);
}

hipError_t cocg32_spmm_dir(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                           hipStream_t s) {
    return launch_spmm_dir_t<float2>(P, P.gab32, S, S.u32, S.p32, S.pn32, n_active_host, nrb, s);
}

hipError_t cocg32_update(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                         hipStream_t s) {
    return launch_update_t<float2>(P, P.gab32, S, S.x32, S.u32, S.pn32, n_active_host, nrb, s);
}

hipError_t cocg32_fold(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                       hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int rpb = S.rpb;
    const int grid = pad8(n_active_host * nrb);
    hipLaunchKernelGGL(k_fold, dim3(grid), dim3(kBlock), 0, s, S.geom, S.x, S.x32, S.tiles,
                       S.counts, nrb, rpb);
    return hipGetLastError();
}

static hipError_t fold_partials(CocgState& S, int n_active_host, int nrb, bool with_r,
                                const double2*& pc, const double*& pr, int& cnt, hipStream_t s);

hipError_t cocg32_replace(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv,
                          int n_active_host, int nrb, double tol2, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    hipError_t e = cocg32_fold(P, S, n_active_host, nrb, s);
    if (e != hipSuccess) return e;
    const int rpb = S.rpb;
    const int grid = pad8(n_active_host * nrb);
    hipLaunchKernelGGL((k_true_residual<float2>), dim3(grid), dim3(kBlock), 0, s, P.rowptr, P.colind, P.ab,
                       S.geom, P.dA, P.dB, S.shifts, S.bsrc, BV, ldbv, S.x, S.u32, S.flag,
                       S.tiles, S.counts, nrb, rpb, S.part_c, S.part_r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double2* pc;
    const double* pr;
    int cnt;
    e = fold_partials(S, n_active_host, nrb, true, pc, pr, cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_replace, dim3(n_active_host), dim3(kBlock), 0, s, cnt, S.tiles,
                       S.counts, pc, pr, S.rho, S.beta, S.bb, S.rr, S.rmax, S.flag,
                       S.active, S.tile_active, S.rbest, S.stall, S.stalled, tol2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cocg_compact(S, s);
}

hipError_t cocg64_restart(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv,
                          int nrb, double tol2, hipStream_t s) {
    const int n_all = S.ntiles;
    const int rpb = S.rpb;
    const int grid = pad8(n_all * nrb);
    hipLaunchKernelGGL((k_true_residual<double2>), dim3(grid), dim3(kBlock), 0, s, P.rowptr,
                       P.colind, P.ab, S.geom, P.dA, P.dB, S.shifts, S.bsrc, BV, ldbv, S.x, S.u,
                       S.stalled, S.tiles, S.counts, nrb, rpb, S.part_c, S.part_r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double2* pc;
    const double* pr;
    int cnt;
    e = fold_partials(S, n_all, nrb, true, pc, pr, cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_restart, dim3(n_all), dim3(kBlock), 0, s, cnt, S.tiles, S.counts,
                       pc, pr, S.rho, S.beta, S.bb, S.rr, S.stalled, S.active, S.tile_active,
                       tol2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cocg_compact(S, s);
}

// Folds the partials of the active tiles to G entries when that pays;
// returns the partial arrays and their row-block count to sum.
static hipError_t fold_partials(CocgState& S, int n_active_host, int nrb, bool with_r,
                                const double2*& pc, const double*& pr, int& cnt, hipStream_t s) {
    pc = S.part_c;
    pr = S.part_r;
    cnt = nrb;
    if (S.G <= 0 || nrb <= 2 * S.G) return hipSuccess;
    hipLaunchKernelGGL(k_fold_partials, dim3(n_active_host * S.G), dim3(kBlock), 0, s, nrb, S.G,
                       S.tiles, S.counts, S.part_c, with_r ? S.part_r : nullptr, S.part2_c,
                       S.part2_r);
    pc = S.part2_c;
    pr = S.part2_r;
    cnt = S.G;
    return hipGetLastError();
}

hipError_t cocg_reduce_alpha(CocgState& S, int n_active_host, int nrb, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const double2* pc;
    const double* pr;
    int cnt;
    hipError_t e = fold_partials(S, n_active_host, nrb, false, pc, pr, cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_alpha, dim3(n_active_host), dim3(kBlock), 0, s, cnt, S.tiles,
                       S.counts, pc, S.rho, S.alpha, S.active);
    return hipGetLastError();
}

hipError_t cocg_reduce_beta(CocgState& S, int n_active_host, int nrb, double tol2, int max_iter,
                            int hold, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const double2* pc;
    const double* pr;
    int cnt;
    hipError_t e = fold_partials(S, n_active_host, nrb, true, pc, pr, cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_beta, dim3(n_active_host), dim3(kBlock), 0, s, cnt, S.tiles,
                       S.counts, pc, pr, S.rho, S.beta, S.bb, S.rr, S.rmax, S.flag,
                       S.active, S.iters, S.tile_active, S.stalled, tol2, max_iter, hold);
    return hipGetLastError();
}

hipError_t cocg_compact(CocgState& S, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, S.ntiles, S.tile_active, S.tiles,
                       S.counts);
    return hipGetLastError();
}

}  // namespace gep
