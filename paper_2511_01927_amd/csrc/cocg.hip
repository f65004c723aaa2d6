// Batched Jacobi-preconditioned COCG for the complex symmetric shifted
// systems (z_j B - A) y = b of the quadrature equation (paper Appendix,
// "Numerical Quadrature": the N_q shifted solves are the dominant cost and
// are independent).  Every column of the tiled multivector is its own
// system (one node z_c, one right-hand side); all columns advance together.
//
// Per iteration (conjugate-orthogonal CG, bilinear form x^T y):
//   q = K p                      (spmm.hip, fused p^T q partials)
//   alpha = rho / p^T q          (k_reduce_alpha)
//   x += alpha p, r -= alpha q, u = D^-1 r, rho' = r^T u, ||r||^2
//                                (k_update, D = z diag(B) - diag(A))
//   beta = rho'/rho, convergence ||r|| <= tol ||b||   (k_reduce_beta)
//   active-tile compaction       (k_compact)
//   p = u + beta p               (k_direction)
// Dot products: each lane owns one column, so a wave sums its rows in
// registers, the 4 waves of a work-group combine in LDS, and per-tile
// partials over row blocks are summed in a fixed order (deterministic).
#include "internal.h"

namespace gep {

__device__ inline double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct BlockMap {
    int slot, rb, tile, lane, wave, r0, r1;
};

__device__ inline bool map_block(const int32_t* tiles, const int32_t* n_active, int nrb, int rpb,
                                 int n, BlockMap& m) {
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    m.slot = lb / nrb;
    m.rb = lb - m.slot * nrb;
    if (m.slot >= n_active[0]) return false;
    m.tile = tiles[m.slot];
    m.lane = threadIdx.x & 63;
    m.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    m.r0 = m.rb * rpb;
    m.r1 = min(n, m.r0 + rpb);
    return true;
}

// Sum a per-lane double2 and double over the 4 waves and store the partials.
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

// x = 0, r = b, p = u = D^-1 b; partials of rho = b^T u and ||b||^2.
__global__ __launch_bounds__(kBlock) void k_init(int n, const double* __restrict__ dA,
                                                 const double* __restrict__ dB,
                                                 const double2* __restrict__ shifts,
                                                 const int32_t* __restrict__ bcol,
                                                 const double* __restrict__ BV, int64_t ldbv,
                                                 double2* __restrict__ x, double2* __restrict__ r,
                                                 double2* __restrict__ p,
                                                 const int32_t* __restrict__ tiles,
                                                 const int32_t* __restrict__ n_active, int nrb,
                                                 int rpb, double2* part_c, double* part_r) {
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, n, m)) return;
    const int col = m.tile * kTile + m.lane;
    const int bc = bcol[col];
    const double2 z = shifts[col];
    const size_t base = (size_t)m.tile * (size_t)n * kTile;
    double2 rho = make_double2(0.0, 0.0);
    double bb = 0.0;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const double b = bc >= 0 ? BV[(size_t)i * ldbv + bc] : 0.0;
        const double2 D = make_double2(z.x * dB[i] - dA[i], z.y * dB[i]);
        const double2 u = cdiv(make_double2(b, 0.0), D);
        const size_t o = base + (size_t)i * kTile + m.lane;
        x[o] = make_double2(0.0, 0.0);
        r[o] = make_double2(b, 0.0);
        p[o] = u;
        rho.x += b * u.x;
        rho.y += b * u.y;
        bb += b * b;
    }
    block_partials(m, nrb, rho, bb, part_c, part_r);
}

// After k_init: rho, ||b||^2, activity per column and per tile.
__global__ void k_reduce_init(int ntiles, int nrb, const double2* __restrict__ part_c,
                              const double* __restrict__ part_r, double2* __restrict__ rho,
                              double* __restrict__ bb, double* __restrict__ rr,
                              int32_t* __restrict__ active, int32_t* __restrict__ iters,
                              int32_t* __restrict__ tile_active) {
    const int tile = blockIdx.x;
    const int lane = threadIdx.x;
    const int col = tile * kTile + lane;
    double2 sc = make_double2(0.0, 0.0);
    double sr = 0.0;
    for (int rb = 0; rb < nrb; ++rb) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        sc.x += part_c[o].x;
        sc.y += part_c[o].y;
        sr += part_r[o];
    }
    rho[col] = sc;
    bb[col] = sr;
    rr[col] = sr;
    iters[col] = 0;
    const int a = sr > 0.0 ? 1 : 0;
    active[col] = a;
    __shared__ int cnt;
    if (lane == 0) cnt = 0;
    __syncthreads();
    if (a) atomicAdd(&cnt, 1);
    __syncthreads();
    if (lane == 0) tile_active[tile] = cnt;
}

__global__ void k_reduce_alpha(int nrb, const int32_t* __restrict__ tiles,
                               const int32_t* __restrict__ n_active,
                               const double2* __restrict__ part_c, const double2* __restrict__ rho,
                               double2* __restrict__ alpha, int32_t* __restrict__ active) {
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x;
    const int col = tile * kTile + lane;
    double2 pq = make_double2(0.0, 0.0);
    for (int rb = 0; rb < nrb; ++rb) {
        const double2 v = part_c[((size_t)tile * nrb + rb) * kTile + lane];
        pq.x += v.x;
        pq.y += v.y;
    }
    double2 a = make_double2(0.0, 0.0);
    if (active[col]) {
        const double m2 = pq.x * pq.x + pq.y * pq.y;
        if (m2 > 0.0 && isfinite(m2)) {
            a = cdiv(rho[col], pq);
        } else {
            active[col] = 0;   // breakdown: p^T q = 0
        }
    }
    alpha[col] = a;
}

// x += alpha p, r -= alpha q, u = D^-1 r; partials rho' = r^T u, ||r||^2.
__global__ __launch_bounds__(kBlock) void k_update(int n, const double* __restrict__ dA,
                                                   const double* __restrict__ dB,
                                                   const double2* __restrict__ shifts,
                                                   const double2* __restrict__ alpha,
                                                   double2* __restrict__ x,
                                                   double2* __restrict__ r,
                                                   const double2* __restrict__ p,
                                                   const double2* __restrict__ q,
                                                   const int32_t* __restrict__ tiles,
                                                   const int32_t* __restrict__ n_active, int nrb,
                                                   int rpb, double2* part_c, double* part_r) {
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, n, m)) return;
    const int col = m.tile * kTile + m.lane;
    const double2 a = alpha[col];
    const double2 z = shifts[col];
    const size_t base = (size_t)m.tile * (size_t)n * kTile;
    double2 rho = make_double2(0.0, 0.0);
    double rr = 0.0;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const size_t o = base + (size_t)i * kTile + m.lane;
        const double2 pv = p[o], qv = q[o];
        double2 xv = x[o], rv = r[o];
        xv.x = fma(a.x, pv.x, fma(-a.y, pv.y, xv.x));
        xv.y = fma(a.x, pv.y, fma(a.y, pv.x, xv.y));
        rv.x = fma(-a.x, qv.x, fma(a.y, qv.y, rv.x));
        rv.y = fma(-a.x, qv.y, fma(-a.y, qv.x, rv.y));
        x[o] = xv;
        r[o] = rv;
        const double2 D = make_double2(z.x * dB[i] - dA[i], z.y * dB[i]);
        const double2 u = cdiv(rv, D);
        rho.x += rv.x * u.x - rv.y * u.y;
        rho.y += rv.x * u.y + rv.y * u.x;
        rr += rv.x * rv.x + rv.y * rv.y;
    }
    block_partials(m, nrb, rho, rr, part_c, part_r);
}

__global__ void k_reduce_beta(int nrb, const int32_t* __restrict__ tiles,
                              const int32_t* __restrict__ n_active,
                              const double2* __restrict__ part_c, const double* __restrict__ part_r,
                              double2* __restrict__ rho, double2* __restrict__ beta,
                              const double* __restrict__ bb, double* __restrict__ rr,
                              int32_t* __restrict__ active, int32_t* __restrict__ iters,
                              int32_t* __restrict__ tile_active, double tol2, int max_iter) {
    const int slot = blockIdx.x;
    if (slot >= n_active[0]) return;
    const int tile = tiles[slot];
    const int lane = threadIdx.x;
    const int col = tile * kTile + lane;
    double2 rn = make_double2(0.0, 0.0);
    double s = 0.0;
    for (int rb = 0; rb < nrb; ++rb) {
        const size_t o = ((size_t)tile * nrb + rb) * kTile + lane;
        rn.x += part_c[o].x;
        rn.y += part_c[o].y;
        s += part_r[o];
    }
    int a = active[col];
    double2 b = make_double2(0.0, 0.0);
    if (a) {
        const int it = iters[col] + 1;
        iters[col] = it;
        rr[col] = s;
        const double2 ro = rho[col];
        const double m2 = ro.x * ro.x + ro.y * ro.y;
        if (s <= tol2 * bb[col] || it >= max_iter || !(m2 > 0.0) || !isfinite(s)) {
            a = 0;
            active[col] = 0;
        } else {
            b = cdiv(rn, ro);
            rho[col] = rn;
        }
    }
    beta[col] = b;
    __shared__ int cnt;
    if (lane == 0) cnt = 0;
    __syncthreads();
    if (a) atomicAdd(&cnt, 1);
    __syncthreads();
    if (lane == 0) tile_active[tile] = cnt;
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

// p = D^-1 r + beta p
__global__ __launch_bounds__(kBlock) void k_direction(int n, const double* __restrict__ dA,
                                                      const double* __restrict__ dB,
                                                      const double2* __restrict__ shifts,
                                                      const double2* __restrict__ beta,
                                                      const double2* __restrict__ r,
                                                      double2* __restrict__ p,
                                                      const int32_t* __restrict__ tiles,
                                                      const int32_t* __restrict__ n_active,
                                                      int nrb, int rpb) {
    BlockMap m;
    if (!map_block(tiles, n_active, nrb, rpb, n, m)) return;
    const int col = m.tile * kTile + m.lane;
    const double2 b = beta[col];
    const double2 z = shifts[col];
    const size_t base = (size_t)m.tile * (size_t)n * kTile;
    for (int i = m.r0 + m.wave; i < m.r1; i += kWaves) {
        const size_t o = base + (size_t)i * kTile + m.lane;
        const double2 D = make_double2(z.x * dB[i] - dA[i], z.y * dB[i]);
        const double2 u = cdiv(r[o], D);
        const double2 pv = p[o];
        p[o] = make_double2(u.x + b.x * pv.x - b.y * pv.y, u.y + b.x * pv.y + b.y * pv.x);
    }
}

static inline int rows_per_block(int64_t n, int nrb) { return (int)((n + nrb - 1) / nrb); }

// k_init runs over all tiles: the caller fills `tiles` with 0..ntiles-1 and
// counts[0] = ntiles first.
hipError_t cocg_init(const DevPencil& P, CocgState& S, const double* BV, int64_t ldbv, int nrb,
                     hipStream_t s) {
    const int rpb = rows_per_block(P.n, nrb);
    const int grid = pad8(S.ntiles * nrb);
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, (int)P.n, P.dA, P.dB, S.shifts,
                       S.bcol, BV, ldbv, S.x, S.r, S.p, S.tiles, S.counts, nrb, rpb, S.part_c,
                       S.part_r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_init, dim3(S.ntiles), dim3(kTile), 0, s, S.ntiles, nrb, S.part_c,
                       S.part_r, S.rho, S.bb, S.rr, S.active, S.iters, S.tile_active);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cocg_compact(S, s);
}

hipError_t cocg_reduce_alpha(CocgState& S, int n_active_host, int nrb, hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_alpha, dim3(n_active_host), dim3(kTile), 0, s, nrb, S.tiles,
                       S.counts, S.part_c, S.rho, S.alpha, S.active);
    return hipGetLastError();
}

hipError_t cocg_update(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                       hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int rpb = rows_per_block(P.n, nrb);
    const int grid = pad8(n_active_host * nrb);
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(kBlock), 0, s, (int)P.n, P.dA, P.dB, S.shifts,
                       S.alpha, S.x, S.r, S.p, S.q, S.tiles, S.counts, nrb, rpb, S.part_c,
                       S.part_r);
    return hipGetLastError();
}

hipError_t cocg_reduce_beta(CocgState& S, int n_active_host, int nrb, double tol2, int max_iter,
                            hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_beta, dim3(n_active_host), dim3(kTile), 0, s, nrb, S.tiles,
                       S.counts, S.part_c, S.part_r, S.rho, S.beta, S.bb, S.rr, S.active, S.iters,
                       S.tile_active, tol2, max_iter);
    return hipGetLastError();
}

hipError_t cocg_compact(CocgState& S, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, S.ntiles, S.tile_active, S.tiles,
                       S.counts);
    return hipGetLastError();
}

hipError_t cocg_direction(const DevPencil& P, CocgState& S, int n_active_host, int nrb,
                          hipStream_t s) {
    if (n_active_host <= 0) return hipSuccess;
    const int rpb = rows_per_block(P.n, nrb);
    const int grid = pad8(n_active_host * nrb);
    hipLaunchKernelGGL(k_direction, dim3(grid), dim3(kBlock), 0, s, (int)P.n, P.dA, P.dB,
                       S.shifts, S.beta, S.r, S.p, S.tiles, S.counts, nrb, rpb);
    return hipGetLastError();
}

}  // namespace gep
