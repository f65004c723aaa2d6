// Right-hand-side block and moment accumulation.
//
// * k_gaussian: the random block V of the CI pipeline (Alg. "Standard CI
//   pipeline", draw a random block), real N(0,1) entries from a
//   counter-based generator: SplitMix64 (Steele, Lea, Flood 2014) at counter
//   e = l*n + i, a uniform in (0,1] from its top 53 bits, Box-Muller on the
//   counter pair (e & ~1, e | 1), cosine branch for even e, sine for odd.
// * k_moments: S_m = (1/2 pi i) * contour integral of zeta^m (zB - A)^-1 B V dz by the
//   trapezoid rule over the nodes in the upper half plane; the lower-half
//   nodes are the complex conjugates for a real pencil, so each node
//   contributes 2 Re(w_j zeta_j^m Y_j).  coef[k][j][m] = 2 w_j zeta_j^m.
#include "internal.h"

namespace gep {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double uniform_at(uint64_t seed, uint64_t c) {
    return ((double)(splitmix64_at(seed, c) >> 11) + 1.0) * 0x1.0p-53;
}

__global__ void k_gaussian(uint64_t seed, int64_t n, int64_t L, double* __restrict__ V) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * L) return;
    const int64_t i = t / L;
    const int64_t l = t - i * L;
    const uint64_t e = (uint64_t)(l * n + i);
    const uint64_t p = e >> 1;
    const double u1 = uniform_at(seed, 2 * p);
    const double u2 = uniform_at(seed, 2 * p + 1);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = (2.0 * M_PI) * u2;
    V[t] = (e & 1ull) ? rad * sin(ang) : rad * cos(ang);
}

hipError_t launch_gaussian(uint64_t seed, int64_t n, int64_t L, double* V, hipStream_t s) {
    const int64_t total = n * L;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_gaussian, dim3((unsigned)blocks), dim3(256), 0, s, seed, n, L, V);
    return hipGetLastError();
}

constexpr int kMaxMoments = 16;

__global__ __launch_bounds__(256) void k_moments(const double2* __restrict__ X, TileGeom g, int NH,
                                                 int L, int M, const int64_t* __restrict__ coff,
                                                 const int32_t* __restrict__ cn,
                                                 const int64_t* __restrict__ soff,
                                                 const double2* __restrict__ coef,
                                                 double* __restrict__ S) {
    const int k = blockIdx.y;
    const int64_t n = cn[k];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * L) return;
    const int64_t i = e / L;
    const int l = (int)(e - i * L);
    double acc[kMaxMoments];
#pragma unroll
    for (int m = 0; m < kMaxMoments; ++m) acc[m] = 0.0;
    for (int j = 0; j < NH; ++j) {
        const int64_t col = coff[k] + (int64_t)j * L + l;
        const int64_t t = col / kTile;
        const double2 xv = X[g.base[t] + i * kTile + (col % kTile)];
        const double2* cj = coef + ((int64_t)k * NH + j) * M;
#pragma unroll
        for (int m = 0; m < kMaxMoments; ++m)
            if (m < M) acc[m] += cj[m].x * xv.x - cj[m].y * xv.y;
    }
    double* Sk = S + soff[k] + i * ((int64_t)L * M);
#pragma unroll
    for (int m = 0; m < kMaxMoments; ++m)
        if (m < M) Sk[(int64_t)m * L + l] = acc[m];
}

hipError_t launch_moments(const double2* X, const TileGeom& g, int64_t nmax, int K, int NH, int L,
                          int M, const int64_t* coff, const int32_t* cn, const int64_t* soff,
                          const double2* coef, double* S, hipStream_t s) {
    if (M > kMaxMoments) return hipErrorInvalidValue;
    if (K <= 0 || nmax <= 0) return hipSuccess;
    const int64_t blocks = (nmax * L + 255) / 256;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)blocks, K), dim3(256), 0, s, X, g, NH, L, M, coff,
                       cn, soff, coef, S);
    return hipGetLastError();
}

}  // namespace gep
