// FP64 matrix-core (MFMA) kernels for the dense tall-skinny products of the
// orthonormalisation and Rayleigh-Ritz steps (Alg. "Standard CI pipeline":
// Q <- orth(Y), A_k = Q^T A Q, B_k = Q^T B Q, x = Q u).
//
// Both kernels use v_mfma_f64_16x16x4_f64: per wavefront D(16x16) += A(16x4)
// B(4x16) with lane l supplying A[l % 16][l / 16] and B[l / 16][l % 16],
// and holding D[(l / 16) + 4 v][l % 16] in accumulator element v.
#include "internal.h"

#include <mutex>

namespace gep {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---- Gram: G = X^T Y, X n x k1 (ld1), Y n x k2 (ld2), row-major -----------
// Work-group: 64 x 64 output tile, 4 waves each 32 x 32 (2 x 2 MFMA tiles),
// split-K over row chunks; partial tiles go to work[split][k1][k2].
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ X, int64_t ld1,
                                              const double* __restrict__ Y, int64_t ld2,
                                              int64_t n, int k1, int k2, int tm, int tn,
                                              int64_t chunk, double* __restrict__ work) {
    const int b = blockIdx.x;
    const int tiles = tm * tn;
    const int split = b / tiles;
    const int t = b - split * tiles;
    const int bm = t / tn, bn = t - (t / tn) * tn;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = bm * 64 + (wave & 1) * 32;
    const int n0 = bn * 64 + (wave >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t rs = (int64_t)split * chunk;
    const int64_t re = min(n, rs + chunk);
    f64x4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    const int ca0 = m0 + li, ca1 = m0 + 16 + li;
    const int cb0 = n0 + li, cb1 = n0 + 16 + li;
    const bool oka0 = ca0 < k1, oka1 = ca1 < k1, okb0 = cb0 < k2, okb1 = cb1 < k2;
    for (int64_t r = rs; r < re; r += 4) {
        const int64_t row = r + lk;
        const bool okr = row < re;
        const double* xr = X + row * ld1;
        const double* yr = Y + row * ld2;
        const double a0 = (okr && oka0) ? xr[ca0] : 0.0;
        const double a1 = (okr && oka1) ? xr[ca1] : 0.0;
        const double b0 = (okr && okb0) ? yr[cb0] : 0.0;
        const double b1 = (okr && okb1) ? yr[cb1] : 0.0;
        acc00 = mfma16x16x4(a0, b0, acc00);
        acc01 = mfma16x16x4(a0, b1, acc01);
        acc10 = mfma16x16x4(a1, b0, acc10);
        acc11 = mfma16x16x4(a1, b1, acc11);
    }
    double* W = work + (int64_t)split * k1 * k2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ri = lk + 4 * v;
        const int r0 = m0 + ri, r1 = m0 + 16 + ri;
        if (r0 < k1 && okb0) W[(int64_t)r0 * k2 + cb0] = acc00[v];
        if (r0 < k1 && okb1) W[(int64_t)r0 * k2 + cb1] = acc01[v];
        if (r1 < k1 && okb0) W[(int64_t)r1 * k2 + cb0] = acc10[v];
        if (r1 < k1 && okb1) W[(int64_t)r1 * k2 + cb1] = acc11[v];
    }
}

__global__ void k_sum_splits(const double* __restrict__ work, int splits, int64_t elems,
                             double* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= elems) return;
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += work[(int64_t)p * elems + e];
    G[e] = s;
}

static void gram_plan(int64_t n, int64_t k1, int64_t k2, int& tm, int& tn, int& splits,
                      int64_t& chunk) {
    tm = (int)((k1 + 63) / 64);
    tn = (int)((k2 + 63) / 64);
    if (n <= 0) {
        splits = 0;
        chunk = 0;
        return;
    }
    int want = (1024 + tm * tn - 1) / (tm * tn);
    int64_t maxs = (n + 63) / 64;   // at least 64 rows per split
    splits = (int)std::max<int64_t>(1, std::min<int64_t>(want, maxs));
    chunk = (n + splits - 1) / splits;
    chunk = (chunk + 3) & ~int64_t(3);
    splits = (int)((n + chunk - 1) / chunk);
    if (splits < 1) splits = 1;
}

size_t gram_work_elems(int64_t n, int64_t k1, int64_t k2) {
    int tm, tn, splits;
    int64_t chunk;
    gram_plan(n, k1, k2, tm, tn, splits, chunk);
    return (size_t)splits * (size_t)k1 * (size_t)k2;
}

hipError_t launch_gram(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n,
                       int64_t k1, int64_t k2, double* G, double* work, size_t work_elems,
                       hipStream_t s) {
    if (k1 <= 0 || k2 <= 0) return hipSuccess;
    int tm, tn, splits;
    int64_t chunk;
    gram_plan(n, k1, k2, tm, tn, splits, chunk);
    if ((size_t)splits * k1 * k2 > work_elems) return hipErrorInvalidValue;
    if (splits > 0)
        hipLaunchKernelGGL(k_gram, dim3(splits * tm * tn), dim3(256), 0, s, X, ld1, Y, ld2, n,
                       (int)k1, (int)k2, tm, tn, chunk, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t elems = k1 * k2;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, work,
                       splits, elems, G);
    return hipGetLastError();
}

// ---- allocation-free Gram (gep_gram_noalloc) --------------------------------
// The split-K partial tiles of k_gram normally live in a buffer allocated per
// call.  For callers that cannot allocate, they go to this file-scope device
// array instead: kGramScratchElems doubles (64 MiB) per GPU, held from module
// load until the process ends.  Its host-side name is only a stand-in for the
// symbol; kernels get the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.  Every call on one GPU
// shares the array: calls that overlap on one GPU (different streams or
// threads) race on it.  Each call overwrites every partial it later sums, so
// nothing has to be cleared between calls.
constexpr size_t kGramScratchElems = size_t(8) << 20;
static __device__ __align__(256) double scratch[kGramScratchElems];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t gram_scratch_elems() { return kGramScratchElems; }

// Device address of `scratch` on the current device (looked up on the first
// call per device).
hipError_t gram_scratch(double** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

// ---- tall GEMM: C = X T, X n x k (ldx), T k x m (ldt), C n x m (ldc) -----
// Work-group: 64 rows x 64 columns; wave w owns rows 16w..16w+15 and four
// 16-column MFMA tiles.
__global__ __launch_bounds__(256) void k_gemm_tall(const double* __restrict__ X, int64_t ldx,
                                                   const double* __restrict__ T, int64_t ldt,
                                                   int64_t n, int k, int m,
                                                   double* __restrict__ C, int64_t ldc) {
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int n0 = blockIdx.y * 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t arow = row0 + wave * 16 + li;
    const bool okrow = arow < n;
    const double* xr = X + arow * ldx;
    f64x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f64x4{0, 0, 0, 0};
    for (int kk = 0; kk < k; kk += 4) {
        const int ka = kk + lk;
        const bool okk = ka < k;
        const double a = (okrow && okk) ? xr[ka] : 0.0;
        const double* tr = T + (int64_t)ka * ldt;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = n0 + c * 16 + li;
            const double bv = (okk && col < m) ? tr[col] : 0.0;
            acc[c] = mfma16x16x4(a, bv, acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int col = n0 + c * 16 + li;
        if (col >= m) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t orow = row0 + wave * 16 + lk + 4 * v;
            if (orow < n) C[orow * ldc + col] = acc[c][v];
        }
    }
}

hipError_t launch_gemm_tall(const double* X, int64_t ldx, const double* T, int64_t ldt, int64_t n,
                            int64_t k, int64_t m, double* C, int64_t ldc, hipStream_t s) {
    if (n <= 0 || m <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
    hipLaunchKernelGGL(k_gemm_tall, grid, dim3(256), 0, s, X, ldx, T, ldt, n, (int)k, (int)m, C,
                       ldc);
    return hipGetLastError();
}

}  // namespace gep
