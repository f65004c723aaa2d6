// Spectral-density network: a small MLP that maps a downsampled coefficient
// field to an eigenvalue-density histogram over a target window, the learned
// spectral prior that drives contour construction (paper Sec. 4.1, "Neural
// Operator for Rapid Spectral Prediction"; the paper regresses eigenvalues
// with an FNO backbone, here the output is a histogram and the network is a
// GEMM-shaped MLP).
//
//   H1 = GELU(X W1 + b1), H2 = GELU(H1 W2 + b2), Y = H2 W3 + b3
//   loss = mean((Y - T)^2)  (the paper trains with a mean squared error)
//
// Every GEMM (forward and backward) runs on BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; master weights, Adam
// moments, biases, pre-activations and the loss are FP32.  GELU is the exact
// erf form.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gep_ci.h"
#include "internal.h"

namespace gep {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// C[m][n] (+)= sum_k A(m, k) B(k, n); A(m, k) = A[m * sam + k * sak] (bf16),
// B(k, n) = B[k * sbk + n * sbn] (bf16), C row-major fp32 with ldc.
// Work-group: 4 waves, each one 16 x 16 output tile of a 32 x 32 block.
// Lane l supplies A[l % 16][8 (l / 16) .. +7] and B[8 (l / 16) .. +7][l % 16]
// and holds C[4 (l / 16) + v][l % 16] in accumulator element v.
__global__ __launch_bounds__(256) void k_gemm_bf16(const __bf16* __restrict__ A, int64_t sam,
                                                   int64_t sak, const __bf16* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, float* __restrict__ C,
                                                   int64_t ldc, int M, int N, int K, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 32 + (wave & 1) * 16;
    const int n0 = blockIdx.x * 32 + (wave >> 1) * 16;
    const int li = lane & 15, lk = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int am = m0 + li, bn = n0 + li;
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + 8 * lk + e;
            a[e] = (am < M && k < K) ? A[(int64_t)am * sam + (int64_t)k * sak] : to_bf16(0.f);
            b[e] = (bn < N && k < K) ? B[(int64_t)k * sbk + (int64_t)bn * sbn] : to_bf16(0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = m0 + 4 * lk + v, c = n0 + li;
        if (r < M && c < N) {
            float* p = C + (int64_t)r * ldc + c;
            *p = accumulate ? *p + acc[v] : acc[v];
        }
    }
}

static hipError_t gemm_bf16(const __bf16* A, int64_t sam, int64_t sak, const __bf16* B, int64_t sbk,
                            int64_t sbn, float* C, int64_t ldc, int M, int N, int K, hipStream_t s) {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, 0);
    return hipGetLastError();
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z += b (in place), H = GELU(Z) or Z (last layer) into bf16 and fp32 copies
__global__ void k_bias_act(float* __restrict__ Z, const float* __restrict__ b, int rows, int cols,
                           int act, __bf16* __restrict__ Hb, float* __restrict__ Hf) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const float z = Z[e] + b[e % cols];
    Z[e] = z;
    const float h = act ? gelu(z) : z;
    if (Hb) Hb[e] = to_bf16(h);
    if (Hf) Hf[e] = h;
}

// dY = 2 (Y - T) / (rows cols); loss partials
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t total,
                      float* __restrict__ dY, __bf16* __restrict__ dYb, double* __restrict__ loss) {
    __shared__ double red[256];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (e < total) {
        const float d = Y[e] - T[e];
        const float g = 2.f * d / (float)total;
        dY[e] = g;
        dYb[e] = to_bf16(g);
        l = (double)d * d / (double)total;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// dZ = dH * GELU'(Z) (bf16 copy for the next GEMMs, fp32 copy for the bias)
__global__ void k_act_bwd(const float* __restrict__ dH, const float* __restrict__ Z, int64_t total,
                          float* __restrict__ dZ, __bf16* __restrict__ dZb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const float g = dH[e] * gelu_d(Z[e]);
    dZ[e] = g;
    dZb[e] = to_bf16(g);
}

// db[c] = sum_r dZ[r][c]
__global__ void k_colsum(const float* __restrict__ dZ, int rows, int cols, float* __restrict__ db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += dZ[(int64_t)r * cols + c];
    db[c] = s;
}

// Adam (Kingma and Ba 2015) with bias correction; refreshes the bf16 copy.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, __bf16* __restrict__ wb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[e] = wi;
    if (wb) wb[e] = to_bf16(wi);
}

__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, __bf16* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = to_bf16(x[e]);
}

static inline dim3 blocks1d(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace gep

using namespace gep;

// Three-layer MLP, parameters: W1 (din x dh), b1, W2 (dh x dh), b2, W3 (dh x dout), b3.
struct gep_density {
    int din = 0, dh = 0, dout = 0;
    int bmax = 0;
    std::vector<int64_t> psize;            // sizes of the 6 parameter tensors
    float* w[6] = {nullptr};               // fp32 master parameters
    float* g[6] = {nullptr};               // gradients
    float* m[6] = {nullptr};
    float* v[6] = {nullptr};
    __bf16* wb[3] = {nullptr};             // bf16 copies of W1..W3
    // activations for a batch of up to bmax rows
    __bf16* xb = nullptr;                  // bmax x din
    float *z1 = nullptr, *z2 = nullptr, *y = nullptr;
    __bf16 *h1b = nullptr, *h2b = nullptr;
    float *dy = nullptr, *dh2 = nullptr, *dz2 = nullptr, *dh1 = nullptr, *dz1 = nullptr;
    __bf16 *dyb = nullptr, *dz2b = nullptr, *dz1b = nullptr;
    double* loss = nullptr;
    long step = 0;
    std::vector<void*> owned;
    ~gep_density() {
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

template <typename T>
T* dalloc(gep_density* N, int64_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<int64_t>(count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    N->owned.push_back(p);
    return (T*)p;
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int fwd(gep_density* N, const float* X, int B, hipStream_t s) {
    if (B <= 0 || B > N->bmax) {
        set_error("batch size out of range");
        return GEP_EINVAL;
    }
    const int din = N->din, dh = N->dh, dout = N->dout;
    hipLaunchKernelGGL(k_to_bf16, blocks1d((int64_t)B * din), dim3(256), 0, s, X, (int64_t)B * din, N->xb);
    // Z1 = X W1
    if (gemm_bf16(N->xb, din, 1, N->wb[0], dh, 1, N->z1, dh, B, dh, din, s) != hipSuccess) return GEP_EDEVICE;
    hipLaunchKernelGGL(k_bias_act, blocks1d((int64_t)B * dh), dim3(256), 0, s, N->z1, N->w[1], B, dh, 1, N->h1b,
                       (float*)nullptr);
    if (gemm_bf16(N->h1b, dh, 1, N->wb[1], dh, 1, N->z2, dh, B, dh, dh, s) != hipSuccess) return GEP_EDEVICE;
    hipLaunchKernelGGL(k_bias_act, blocks1d((int64_t)B * dh), dim3(256), 0, s, N->z2, N->w[3], B, dh, 1, N->h2b,
                       (float*)nullptr);
    if (gemm_bf16(N->h2b, dh, 1, N->wb[2], dout, 1, N->y, dout, B, dout, dh, s) != hipSuccess) return GEP_EDEVICE;
    hipLaunchKernelGGL(k_bias_act, blocks1d((int64_t)B * dout), dim3(256), 0, s, N->y, N->w[5], B, dout, 0,
                       (__bf16*)nullptr, (float*)nullptr);
    return hipGetLastError() == hipSuccess ? GEP_OK : GEP_EDEVICE;
}

}  // namespace

// Block averages of a 3D (or, with nz = 1, 2D) row-major field [z][y][x]
// onto a side^3 (side^2) grid: cell (cz, cy, cx) averages the entries whose
// index along each axis a maps to c = floor(a * side / n_axis).  One thread
// per output cell; the sum runs over the cell's index ranges in order.
__global__ void k_downsample(const float* __restrict__ g, int nz, int ny, int nx, int sz, int side,
                             float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int cells = sz * side * side;
    if (c >= cells) return;
    const int cz = c / (side * side), cy = (c / side) % side, cx = c % side;
    // index ranges [lo, hi) of each axis mapping to the cell
    auto range = [](int cidx, int n, int sd, int& lo, int& hi) {
        lo = (int)(((int64_t)cidx * n + sd - 1) / sd);
        hi = (int)(((int64_t)(cidx + 1) * n + sd - 1) / sd);
    };
    int z0, z1, y0, y1, x0, x1;
    range(cz, nz, sz, z0, z1);
    range(cy, ny, side, y0, y1);
    range(cx, nx, side, x0, x1);
    double acc = 0.0;
    int64_t cnt = 0;
    for (int z = z0; z < z1; ++z)
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                acc += g[((int64_t)z * ny + y) * nx + x];
                ++cnt;
            }
    out[c] = cnt ? (float)(acc / (double)cnt) : 0.0f;
}

extern "C" {

int gep_field_downsample(const float* g, int nz, int ny, int nx, int side, float* out, void* stream) {
    if (!g || !out || nz < 1 || ny < 1 || nx < 1 || side < 1 || side > ny || side > nx ||
        (nz > 1 && side > nz)) {
        set_error("bad downsample arguments");
        return GEP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int sz = nz > 1 ? side : 1;
    const int cells = sz * side * side;
    hipLaunchKernelGGL(k_downsample, dim3((cells + 255) / 256), dim3(256), 0, s, g, nz, ny, nx, sz, side, out);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("downsample kernel failed");
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_density_create(int din, int dhidden, int dout, int max_batch, uint64_t seed, gep_density** out) {
    if (!out || din <= 0 || dhidden <= 0 || dout <= 0 || max_batch <= 0) {
        set_error("bad density-net sizes");
        return GEP_EINVAL;
    }
    *out = nullptr;
    auto* N = new gep_density();
    N->din = din;
    N->dh = dhidden;
    N->dout = dout;
    N->bmax = max_batch;
    N->psize = {(int64_t)din * dhidden, dhidden, (int64_t)dhidden * dhidden, dhidden, (int64_t)dhidden * dout, dout};
    bool ok = true;
    for (int i = 0; i < 6; ++i) {
        N->w[i] = dalloc<float>(N, N->psize[i]);
        N->g[i] = dalloc<float>(N, N->psize[i]);
        N->m[i] = dalloc<float>(N, N->psize[i]);
        N->v[i] = dalloc<float>(N, N->psize[i]);
        ok = ok && N->w[i] && N->g[i] && N->m[i] && N->v[i];
    }
    for (int i = 0; i < 3; ++i) {
        N->wb[i] = dalloc<__bf16>(N, N->psize[2 * i]);
        ok = ok && N->wb[i];
    }
    const int64_t B = max_batch;
    N->xb = dalloc<__bf16>(N, B * din);
    N->z1 = dalloc<float>(N, B * dhidden);
    N->z2 = dalloc<float>(N, B * dhidden);
    N->y = dalloc<float>(N, B * dout);
    N->h1b = dalloc<__bf16>(N, B * dhidden);
    N->h2b = dalloc<__bf16>(N, B * dhidden);
    N->dy = dalloc<float>(N, B * dout);
    N->dh2 = dalloc<float>(N, B * dhidden);
    N->dz2 = dalloc<float>(N, B * dhidden);
    N->dh1 = dalloc<float>(N, B * dhidden);
    N->dz1 = dalloc<float>(N, B * dhidden);
    N->dyb = dalloc<__bf16>(N, B * dout);
    N->dz2b = dalloc<__bf16>(N, B * dhidden);
    N->dz1b = dalloc<__bf16>(N, B * dhidden);
    N->loss = dalloc<double>(N, 1);
    ok = ok && N->xb && N->z1 && N->z2 && N->y && N->h1b && N->h2b && N->dy && N->dh2 && N->dz2 && N->dh1 &&
         N->dz1 && N->dyb && N->dz2b && N->dz1b && N->loss;
    if (!ok) {
        delete N;
        set_error("hipMalloc failed for the density net");
        return GEP_ENOMEM;
    }
    // Glorot-uniform weights from SplitMix64, zero biases and Adam moments
    uint64_t st = seed;
    const int fan[3][2] = {{din, dhidden}, {dhidden, dhidden}, {dhidden, dout}};
    for (int i = 0; i < 6; ++i) {
        std::vector<float> h(N->psize[i], 0.f);
        if (i % 2 == 0) {
            const double lim = std::sqrt(6.0 / (fan[i / 2][0] + fan[i / 2][1]));
            for (auto& x : h) x = (float)(((double)(splitmix(st) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * lim);
        }
        std::vector<float> zero(N->psize[i], 0.f);
        if (hipMemcpy(N->w[i], h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(N->m[i], zero.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(N->v[i], zero.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess) {
            delete N;
            set_error("copy of initial density-net parameters failed");
            return GEP_EDEVICE;
        }
    }
    for (int i = 0; i < 3; ++i)
        hipLaunchKernelGGL(k_to_bf16, blocks1d(N->psize[2 * i]), dim3(256), 0, 0, N->w[2 * i], N->psize[2 * i],
                           N->wb[i]);
    if (hipDeviceSynchronize() != hipSuccess) {
        delete N;
        set_error("density-net initialisation failed");
        return GEP_EDEVICE;
    }
    *out = N;
    return GEP_OK;
}

void gep_density_free(gep_density* N) { delete N; }

int gep_density_forward(gep_density* N, const float* X, int B, float* Y, void* stream) {
    if (!N || !X || !Y) return GEP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = fwd(N, X, B, s);
    if (st) return st;
    if (hipMemcpyAsync(Y, N->y, sizeof(float) * B * N->dout, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("density forward copy failed");
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_density_grads(gep_density* N, const float* X, const float* T, int B, double* loss, void* stream) {
    if (!N || !X || !T) return GEP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = fwd(N, X, B, s);
    if (st) return st;
    const int din = N->din, dh = N->dh, dout = N->dout;
    const int64_t ny = (int64_t)B * dout, nh = (int64_t)B * dh;
    bool ok = hipMemsetAsync(N->loss, 0, sizeof(double), s) == hipSuccess;
    hipLaunchKernelGGL(k_mse, blocks1d(ny), dim3(256), 0, s, N->y, T, ny, N->dy, N->dyb, N->loss);
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = dY W3^T
    ok = ok && gemm_bf16(N->h2b, 1, dh, N->dyb, dout, 1, N->g[4], dout, dh, dout, B, s) == hipSuccess;
    hipLaunchKernelGGL(k_colsum, blocks1d(dout), dim3(256), 0, s, N->dy, B, dout, N->g[5]);
    ok = ok && gemm_bf16(N->dyb, dout, 1, N->wb[2], 1, dout, N->dh2, dh, B, dh, dout, s) == hipSuccess;
    hipLaunchKernelGGL(k_act_bwd, blocks1d(nh), dim3(256), 0, s, N->dh2, N->z2, nh, N->dz2, N->dz2b);
    // layer 2
    ok = ok && gemm_bf16(N->h1b, 1, dh, N->dz2b, dh, 1, N->g[2], dh, dh, dh, B, s) == hipSuccess;
    hipLaunchKernelGGL(k_colsum, blocks1d(dh), dim3(256), 0, s, N->dz2, B, dh, N->g[3]);
    ok = ok && gemm_bf16(N->dz2b, dh, 1, N->wb[1], 1, dh, N->dh1, dh, B, dh, dh, s) == hipSuccess;
    hipLaunchKernelGGL(k_act_bwd, blocks1d(nh), dim3(256), 0, s, N->dh1, N->z1, nh, N->dz1, N->dz1b);
    // layer 1
    ok = ok && gemm_bf16(N->xb, 1, din, N->dz1b, dh, 1, N->g[0], dh, din, dh, B, s) == hipSuccess;
    hipLaunchKernelGGL(k_colsum, blocks1d(dh), dim3(256), 0, s, N->dz1, B, dh, N->g[1]);
    ok = ok && hipGetLastError() == hipSuccess;
    if (loss) ok = ok && hipMemcpyAsync(loss, N->loss, sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        set_error("density backward failed");
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_density_adam(gep_density* N, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!N) return GEP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    N->step += 1;
    const float c1 = 1.f - std::pow(beta1, (float)N->step), c2 = 1.f - std::pow(beta2, (float)N->step);
    for (int i = 0; i < 6; ++i)
        hipLaunchKernelGGL(k_adam, blocks1d(N->psize[i]), dim3(256), 0, s, N->w[i], N->g[i], N->m[i], N->v[i],
                           N->psize[i], lr, beta1, beta2, eps, c1, c2, (i % 2 == 0) ? N->wb[i / 2] : (__bf16*)nullptr);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("Adam step failed");
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_density_param(gep_density* N, int which, int grad, float* host, int set) {
    if (!N || which < 0 || which >= 6 || !host) return GEP_EINVAL;
    float* d = grad ? N->g[which] : N->w[which];
    const size_t bytes = sizeof(float) * N->psize[which];
    hipError_t e = set ? hipMemcpy(d, host, bytes, hipMemcpyHostToDevice) : hipMemcpy(host, d, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && set && !grad && which % 2 == 0) {
        hipLaunchKernelGGL(k_to_bf16, blocks1d(N->psize[which]), dim3(256), 0, 0, N->w[which], N->psize[which],
                           N->wb[which / 2]);
        e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        set_error(std::string("density parameter copy failed: ") + hipGetErrorString(e));
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_gemm_bf16(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk, int64_t sbn,
                  float* C, int64_t ldc, int M, int N, int K, void* stream) {
    if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0) return GEP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (gemm_bf16((const __bf16*)A, sam, sak, (const __bf16*)B, sbk, sbn, C, ldc, M, N, K, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("bf16 gemm failed");
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

}  // extern "C"
