// Multi-shift COCG: the shifted systems (z_j B - A) y_j = B v of every node
// of every contour share one Krylov space when B = beta I, since then the
// matrices differ by multiples of the identity: (z_j beta I - A) y_j = beta v.
// The paper leaves the linear solver open (appendix on numerical quadrature:
// the N_q shifted solves are the dominant cost); this is the shifted form of
// COCG (Frommer's collinear-residual construction for shifted Krylov
// families, here with the complex-symmetric bilinear form): one seed system
// K_s = sigma_s I - A is iterated, and every other shift sigma_c keeps its
// solution and search vector, with residual r / pi_c collinear to the seed's.
// No preconditioner (a preconditioner shared by all shifts would have to be
// shift-invariant).
//
// Layouts: the seed vectors r, p_s, q are tiles of 64 columns, one seed
// column per right-hand side (a contour's block column), element (i, s) at
// ((s / 64) * n + i) * 64 + s % 64; the shifted solutions X and search
// vectors P are the tiled multivector of the solve, element (i, c) at
// base[tile] + i * 64 + lane with c = tile * 64 + lane, column c shifting
// seed column col_l[c].
#include "internal.h"

namespace gep {

// r -= alpha q per seed column; partials of rho = r^T r (bilinear) and of
// ||r||^2 per seed tile (blockIdx.y), row block (blockIdx.x) and column
// (lane), at (tile * nrb + block) * 64 + lane.
__global__ __launch_bounds__(kBlock) void k_ms_seed_update(int n, int rpb, const double2* __restrict__ alpha,
                                                          const double2* __restrict__ q, double2* __restrict__ r,
                                                          double2* __restrict__ part_rho,
                                                          double* __restrict__ part_nrm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.x * rpb, i1 = min(n, i0 + rpb);
    const size_t tb = (size_t)blockIdx.y * n * kTile;
    const double2 a = alpha[blockIdx.y * kTile + lane];
    double2 rho = make_double2(0.0, 0.0);
    double nrm = 0.0;
    for (int i = i0 + wave; i < i1; i += kWaves) {
        const size_t o = tb + (size_t)i * kTile + lane;
        const double2 qv = q[o];
        double2 rv = r[o];
        rv.x -= a.x * qv.x - a.y * qv.y;
        rv.y -= a.x * qv.y + a.y * qv.x;
        r[o] = rv;
        rho.x += rv.x * rv.x - rv.y * rv.y;
        rho.y += 2.0 * rv.x * rv.y;
        nrm += rv.x * rv.x + rv.y * rv.y;
    }
    __shared__ double2 sr[kWaves][kTile];
    __shared__ double sn[kWaves][kTile];
    sr[wave][lane] = rho;
    sn[wave][lane] = nrm;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w) {
            rho.x += sr[w][lane].x;
            rho.y += sr[w][lane].y;
            nrm += sn[w][lane];
        }
        const size_t po = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kTile + lane;
        part_rho[po] = rho;
        part_nrm[po] = nrm;
    }
}

// Every active shifted column c: x_c += alpha_c p_c, p_c = r_s / pi_c + beta_c p_c
// (s = col_l[c], its seed column; coef[c] = {alpha_c, beta_c, 1 / pi_c};
// inactive columns are left as they are).  blockIdx.y is the tile,
// blockIdx.x a row block; n_seed is the seed's row count.
__global__ __launch_bounds__(kBlock) void k_ms_shift_update(TileGeom geom, const int32_t* __restrict__ col_l,
                                                           const int32_t* __restrict__ active,
                                                           const double2* __restrict__ coef,
                                                           const double2* __restrict__ r, double2* __restrict__ X,
                                                           double2* __restrict__ P, int rpb, int n_seed) {
    const int tile = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = tile * kTile + lane;
    const int l = col_l[c];
    if (l < 0 || !active[c]) return;   // per lane: no barrier below
    const double2* __restrict__ rs = r + (size_t)(l / kTile) * n_seed * kTile + (l % kTile);
    const int n = geom.n[tile];
    const int64_t base = geom.base[tile];
    const double2 al = coef[3 * c], be = coef[3 * c + 1], ip = coef[3 * c + 2];
    const int i0 = blockIdx.x * rpb, i1 = min(n, i0 + rpb);
    for (int i = i0 + wave; i < i1; i += kWaves) {
        const int64_t o = base + (int64_t)i * kTile + lane;
        const double2 pv = P[o], rv = rs[(size_t)i * kTile];
        double2 xv = X[o];
        xv.x += al.x * pv.x - al.y * pv.y;
        xv.y += al.x * pv.y + al.y * pv.x;
        X[o] = xv;
        double2 pn;
        pn.x = rv.x * ip.x - rv.y * ip.y + be.x * pv.x - be.y * pv.y;
        pn.y = rv.x * ip.y + rv.y * ip.x + be.x * pv.y + be.y * pv.x;
        P[o] = pn;
    }
}

// p_s = r + beta p_s per seed column (blockIdx.y: seed tile).
__global__ __launch_bounds__(kBlock) void k_ms_seed_p(int n, const double2* __restrict__ beta,
                                                     const double2* __restrict__ r, double2* __restrict__ ps) {
    const int lane = threadIdx.x & 63;
    const size_t tb = (size_t)blockIdx.y * n * kTile;
    const double2 b = beta[blockIdx.y * kTile + lane];
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += gridDim.x * kWaves) {
        const size_t o = tb + (size_t)i * kTile + lane;
        const double2 rv = r[o], pv = ps[o];
        ps[o] = make_double2(rv.x + b.x * pv.x - b.y * pv.y, rv.y + b.x * pv.y + b.y * pv.x);
    }
}

hipError_t ms_seed_update(int n, int nseed_tiles, int nrb, const double2* alpha, const double2* q, double2* r,
                          double2* part_rho, double* part_nrm, hipStream_t s) {
    const int rpb = (n + nrb - 1) / nrb;
    hipLaunchKernelGGL(k_ms_seed_update, dim3(nrb, nseed_tiles), dim3(kBlock), 0, s, n, rpb, alpha, q, r, part_rho,
                       part_nrm);
    return hipGetLastError();
}

hipError_t ms_shift_update(const TileGeom& g, int ntiles, int64_t nmax, int n_seed, const int32_t* col_l,
                           const int32_t* active, const double2* coef, const double2* r, double2* X, double2* P,
                           hipStream_t s) {
    const int nrb = (int)std::max<int64_t>(1, std::min<int64_t>(256, (nmax + 255) / 256));
    const int rpb = (int)((nmax + nrb - 1) / nrb);
    hipLaunchKernelGGL(k_ms_shift_update, dim3(nrb, ntiles), dim3(kBlock), 0, s, g, col_l, active, coef, r, X, P,
                       rpb, n_seed);
    return hipGetLastError();
}

hipError_t ms_seed_p(int n, int nseed_tiles, const double2* beta, const double2* r, double2* ps, hipStream_t s) {
    hipLaunchKernelGGL(k_ms_seed_p, dim3(256, nseed_tiles), dim3(kBlock), 0, s, n, beta, r, ps);
    return hipGetLastError();
}

}  // namespace gep
