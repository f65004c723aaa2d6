// Small dense FP64 kernels for the reduced problems of the CI pipeline
// (orthonormalisation and the reduced GEP A_k u = lambda B_k u, Alg.
// "Standard CI pipeline").  Matrices are k x k, k <= 1024, row-major, one
// work-group per matrix of a batch.
#include "internal.h"

namespace gep {

constexpr int kDenseThreads = 1024;

__device__ inline double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int off = blockDim.x >> 1; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// ---- symmetric eigensolver: cyclic Jacobi, parallel (round-robin) order --
// Each sweep visits all k(k-1)/2 pairs in kp-1 steps of kp/2 disjoint pairs
// (kp = k rounded up to even; the padding index never rotates).  A rotation
// (c, s) zeroes a_pq with t = sgn(tau)/(|tau| + sqrt(1 + tau^2)),
// tau = (a_qq - a_pp)/(2 a_pq) (Golub and Van Loan, symmetric Schur 2x2);
// rows then columns of A, and columns of V, are rotated.  Stops when the
// off-diagonal Frobenius norm is <= 1e-15 ||A||_F or after 40 sweeps.
__global__ __launch_bounds__(kDenseThreads) void k_jacobi(double* __restrict__ Aall,
                                                          double* __restrict__ wout,
                                                          double* __restrict__ Vout,
                                                          double* __restrict__ Vwork, int kmax,
                                                          const int32_t* __restrict__ ks) {
    __shared__ double red[kDenseThreads];
    __shared__ int pp[kDenseThreads / 2], qq[kDenseThreads / 2];
    __shared__ double cs[kDenseThreads / 2], sn[kDenseThreads / 2];
    __shared__ double wl[kDenseThreads];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int k = ks ? ks[b] : kmax;   // matrix b is k x k, stored with stride kmax * kmax
    double* A = Aall + (int64_t)b * kmax * kmax;
    double* V = Vwork + (int64_t)b * kmax * kmax;
    if (k <= 0) return;
    const int kp = k + (k & 1);
    const int np = kp / 2;
    for (int e = t; e < k * k; e += nt) V[e] = (e / k == e % k) ? 1.0 : 0.0;
    double f = 0.0;
    for (int e = t; e < k * k; e += nt) f += A[e] * A[e];
    __syncthreads();
    const double fro2 = block_sum(f, red);
    for (int sweep = 0; sweep < 40 && k > 1; ++sweep) {
        double off = 0.0;
        for (int e = t; e < k * k; e += nt)
            if (e / k != e % k) off += A[e] * A[e];
        const double off2 = block_sum(off, red);
        if (!(off2 > 1e-30 * fro2)) break;
        for (int step = 0; step < kp - 1; ++step) {
            if (t < np) {
                int p, q;
                if (t == 0) {
                    p = kp - 1;
                    q = step;
                } else {
                    p = (step + t) % (kp - 1);
                    q = (step - t + (kp - 1)) % (kp - 1);
                }
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, s = 0.0;
                if (q < k) {
                    const double apq = A[(int64_t)p * k + q];
                    if (apq != 0.0) {
                        const double diff = A[(int64_t)q * k + q] - A[(int64_t)p * k + p];
                        double tt;
                        if (fabs(diff) > 1e150 * fabs(apq)) {
                            tt = apq / diff;
                        } else {
                            const double tau = diff / (2.0 * apq);
                            tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        }
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[t] = p;
                qq[t] = q;
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            // rows p, q of A
            for (int e = t; e < np * k; e += nt) {
                const int pr = e / k, j = e - pr * k;
                const int p = pp[pr], q = qq[pr];
                if (q >= k || sn[pr] == 0.0) continue;
                const double c = cs[pr], s = sn[pr];
                const double ap = A[(int64_t)p * k + j], aq = A[(int64_t)q * k + j];
                A[(int64_t)p * k + j] = c * ap - s * aq;
                A[(int64_t)q * k + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p, q of A and V
            for (int e = t; e < np * k; e += nt) {
                const int i = e / np, pr = e - i * np;
                const int p = pp[pr], q = qq[pr];
                if (q >= k || sn[pr] == 0.0) continue;
                const double c = cs[pr], s = sn[pr];
                const double ap = A[(int64_t)i * k + p], aq = A[(int64_t)i * k + q];
                A[(int64_t)i * k + p] = c * ap - s * aq;
                A[(int64_t)i * k + q] = s * ap + c * aq;
                const double vp = V[(int64_t)i * k + p], vq = V[(int64_t)i * k + q];
                V[(int64_t)i * k + p] = c * vp - s * vq;
                V[(int64_t)i * k + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // ascending order by rank (ties broken by index)
    for (int j = t; j < k; j += nt) wl[j] = A[(int64_t)j * k + j];
    __syncthreads();
    for (int j = t; j < k; j += nt) {
        const double wj = wl[j];
        int rank = 0;
        for (int i = 0; i < k; ++i) rank += (wl[i] < wj) || (wl[i] == wj && i < j);
        wout[(int64_t)b * kmax + rank] = wj;
        double* Vo = Vout + (int64_t)b * kmax * kmax;
        for (int i = 0; i < k; ++i) Vo[(int64_t)i * k + rank] = V[(int64_t)i * k + j];
    }
}

hipError_t launch_sym_eig(double* A, double* w, double* V, int64_t kmax, int batch,
                          const int32_t* ks, double* work, hipStream_t s) {
    if (kmax <= 0 || batch <= 0) return hipSuccess;
    if (kmax > kDenseThreads) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi, dim3(batch), dim3(kDenseThreads), 0, s, A, w, V, work, (int)kmax,
                       ks);
    return hipGetLastError();
}

// ---- Cholesky G = L L^T and LinvT = L^-T ---------------------------------
__global__ __launch_bounds__(kDenseThreads) void k_chol_inv(const double* __restrict__ Gall,
                                                            double* __restrict__ Tall,
                                                            double* __restrict__ Wall, int kmax,
                                                            const int32_t* __restrict__ ks,
                                                            int32_t* __restrict__ status) {
    __shared__ int fail;
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const int k = ks ? ks[b] : kmax;   // matrix b is k x k (leading dimension k), stride kmax^2
    const double* G = Gall + (int64_t)b * kmax * kmax;
    double* W = Wall + (int64_t)b * kmax * kmax;   // holds L (lower)
    double* T = Tall + (int64_t)b * kmax * kmax;   // receives L^-T
    for (int e = t; e < k * k; e += nt) W[e] = G[e];
    if (t == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            const double d = W[(int64_t)j * k + j];
            if (!(d > 0.0) || !isfinite(d)) {
                fail = j + 1;
            } else {
                W[(int64_t)j * k + j] = sqrt(d);
            }
        }
        __syncthreads();
        if (fail) break;
        const double djj = W[(int64_t)j * k + j];
        for (int i = j + 1 + t; i < k; i += nt) W[(int64_t)i * k + j] /= djj;
        __syncthreads();
        const int m = k - j - 1;
        for (int e = t; e < m * m; e += nt) {
            const int i = j + 1 + e / m, l = j + 1 + e % m;
            if (l <= i) W[(int64_t)i * k + l] -= W[(int64_t)i * k + j] * W[(int64_t)l * k + j];
        }
        __syncthreads();
    }
    if (t == 0) status[b] = fail;
    if (fail) return;
    // column c of L^-1 by forward substitution, stored transposed in T
    for (int c = t; c < k; c += nt) {
        for (int i = 0; i < c; ++i) T[(int64_t)c * k + i] = 0.0;
        T[(int64_t)c * k + c] = 1.0 / W[(int64_t)c * k + c];
        for (int i = c + 1; i < k; ++i) {
            double s = 0.0;
            for (int u = c; u < i; ++u) s += W[(int64_t)i * k + u] * T[(int64_t)c * k + u];
            T[(int64_t)c * k + i] = -s / W[(int64_t)i * k + i];
        }
    }
    // T currently holds row c = column c of L^-1, i.e. T = (L^-1)^T = L^-T.
}

hipError_t launch_chol_inv(const double* G, double* LinvT, int64_t kmax, int batch,
                           const int32_t* ks, double* work, int32_t* status, hipStream_t s) {
    if (kmax <= 0 || batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chol_inv, dim3(batch), dim3(kDenseThreads), 0, s, G, LinvT, work,
                       (int)kmax, ks, status);
    return hipGetLastError();
}

// ---- C = op(A) op(B), small row-major ------------------------------------
__global__ void k_small_gemm(const double* __restrict__ A, int ta, const double* __restrict__ B,
                             int tb, double* __restrict__ C, int m, int n, int kk, int64_t lda,
                             int64_t ldb, int64_t ldc) {
    const int i = blockIdx.y * 16 + threadIdx.y;
    const int j = blockIdx.x * 16 + threadIdx.x;
    if (i >= m || j >= n) return;
    double s = 0.0;
    for (int u = 0; u < kk; ++u) {
        const double a = ta ? A[(int64_t)u * lda + i] : A[(int64_t)i * lda + u];
        const double bv = tb ? B[(int64_t)j * ldb + u] : B[(int64_t)u * ldb + j];
        s = fma(a, bv, s);
    }
    C[(int64_t)i * ldc + j] = s;
}

hipError_t launch_small_gemm(const double* A, int ta, const double* B, int tb, double* C,
                             int64_t m, int64_t n, int64_t kk, int64_t lda, int64_t ldb,
                             int64_t ldc, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 15) / 16), (unsigned)((m + 15) / 16));
    hipLaunchKernelGGL(k_small_gemm, grid, dim3(16, 16), 0, s, A, ta, B, tb, C, (int)m, (int)n,
                       (int)kk, lda, ldb, ldc);
    return hipGetLastError();
}

__global__ void k_symmetrise(double* __restrict__ A, int k) {
    const int i = blockIdx.y * 16 + threadIdx.y;
    const int j = blockIdx.x * 16 + threadIdx.x;
    if (i >= k || j >= k || j <= i) return;
    const double v = 0.5 * (A[(int64_t)i * k + j] + A[(int64_t)j * k + i]);
    A[(int64_t)i * k + j] = v;
    A[(int64_t)j * k + i] = v;
}

hipError_t launch_symmetrise(double* A, int64_t k, hipStream_t s) {
    if (k <= 1) return hipSuccess;
    dim3 grid((unsigned)((k + 15) / 16), (unsigned)((k + 15) / 16));
    hipLaunchKernelGGL(k_symmetrise, grid, dim3(16, 16), 0, s, A, (int)k);
    return hipGetLastError();
}

__global__ void k_svqb_scale(const double* __restrict__ U, const double* __restrict__ w, int k,
                             int r, double* __restrict__ T) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * r) return;
    const int i = e / r, j = e - (e / r) * r;
    const int src = k - r + j;
    T[e] = U[(int64_t)i * k + src] / sqrt(w[src]);
}

hipError_t launch_svqb_scale(const double* U, const double* w, int64_t k, int64_t r, double* T,
                             hipStream_t s) {
    if (k <= 0 || r <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_svqb_scale, dim3((unsigned)((k * r + 255) / 256)), dim3(256), 0, s, U, w,
                       (int)k, (int)r, T);
    return hipGetLastError();
}

// ---- residual norms over row-major n x k blocks ---------------------------
__global__ __launch_bounds__(256) void k_resid_part(const double* __restrict__ AX,
                                                    const double* __restrict__ BX,
                                                    const double* __restrict__ X,
                                                    const double* __restrict__ th, int64_t n,
                                                    int k, int nrb, int64_t rpb,
                                                    double* __restrict__ work) {
    const int nch = (k + 63) / 64;
    const int chunk = blockIdx.x % nch;
    const int rb = blockIdx.x / nch;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = chunk * 64 + lane;
    const bool ok = col < k;
    const double tc = ok ? th[col] : 0.0;
    const int64_t r0 = (int64_t)rb * rpb;
    const int64_t r1 = min(n, r0 + rpb);
    double sn = 0.0, sd = 0.0;
    if (ok) {
        for (int64_t i = r0 + wave; i < r1; i += 4) {
            const int64_t o = i * k + col;
            const double rv = AX[o] - tc * BX[o];
            sn += rv * rv;
            sd += X[o] * X[o];
        }
    }
    __shared__ double ra[4][64], rd[4][64];
    ra[wave][lane] = sn;
    rd[wave][lane] = sd;
    __syncthreads();
    if (wave == 0 && ok) {
        const double a = ra[0][lane] + ra[1][lane] + ra[2][lane] + ra[3][lane];
        const double d = rd[0][lane] + rd[1][lane] + rd[2][lane] + rd[3][lane];
        work[((int64_t)rb * k + col) * 2] = a;
        work[((int64_t)rb * k + col) * 2 + 1] = d;
    }
}

__global__ void k_resid_final(const double* __restrict__ work, int nrb, int k,
                              double* __restrict__ num, double* __restrict__ den) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= k) return;
    double a = 0.0, d = 0.0;
    for (int rb = 0; rb < nrb; ++rb) {
        a += work[((int64_t)rb * k + col) * 2];
        d += work[((int64_t)rb * k + col) * 2 + 1];
    }
    num[col] = sqrt(a);
    den[col] = sqrt(d);
}

hipError_t launch_resid_norms(const double* AX, const double* BX, const double* X,
                              const double* theta, int64_t n, int64_t k, double* num, double* den,
                              double* work, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    const int nch = (int)((k + 63) / 64);
    int nrb = (int)std::min<int64_t>(std::max<int64_t>(1, 1024 / nch), std::max<int64_t>(1, n / 64));
    const int64_t rpb = (n + nrb - 1) / nrb;
    hipLaunchKernelGGL(k_resid_part, dim3(nch * nrb), dim3(256), 0, s, AX, BX, X, theta, n, (int)k,
                       nrb, rpb, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid_final, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, work, nrb,
                       (int)k, num, den);
    return hipGetLastError();
}

// ---- gather + sign normalisation -------------------------------------------
__global__ __launch_bounds__(256) void k_gather_cols(const double* __restrict__ X, int64_t n,
                                                     int k, const int32_t* __restrict__ sel,
                                                     double* __restrict__ out) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    const int t = threadIdx.x;
    const int c = sel[blockIdx.x];
    double best = -1.0;
    int64_t idx = 0;
    for (int64_t i = t; i < n; i += 256) {
        const double a = fabs(X[i * k + c]);
        if (a > best) {
            best = a;
            idx = i;
        }
    }
    bv[t] = best;
    bi[t] = idx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            const double o = bv[t + off];
            const int64_t oi = bi[t + off];
            if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
                bv[t] = o;
                bi[t] = oi;
            }
        }
        __syncthreads();
    }
    const double sgn = X[bi[0] * k + c] < 0.0 ? -1.0 : 1.0;
    double* o = out + (int64_t)blockIdx.x * n;
    for (int64_t i = t; i < n; i += 256) o[i] = sgn * X[i * k + c];
}

hipError_t launch_gather_cols(const double* X, int64_t n, int64_t k, const int32_t* sel, int m,
                              double* out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_cols, dim3(m), dim3(256), 0, s, X, n, (int)k, sel, out);
    return hipGetLastError();
}

}  // namespace gep
