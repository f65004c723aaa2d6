// Small dense FP64 kernels for the reduced problems of the CI pipeline
// (orthonormalisation and the reduced GEP A_k u = lambda B_k u, Alg.
// "Standard CI pipeline").  Matrices are k x k, k <= 1024, row-major, one
// work-group per matrix of a batch.
#include <algorithm>
#include <vector>

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

// ---- symmetric eigensolver: block Jacobi, parallel (round-robin) order ---
// Two-sided block Jacobi with blocks of kBJ = 32 indices (Golub and Van Loan,
// block Jacobi for the symmetric eigenproblem).  The nbp blocks (k / 32
// rounded up, plus one empty block when odd) are paired round robin: a sweep
// is nbp - 1 rounds of nbp / 2 disjoint block pairs.  In a round every pair
// (I, J) runs one cyclic sweep of element rotations on its 64 x 64 subproblem
// S = A[I u J, I u J] in LDS (all index pairs in the first round of a sweep,
// the pairs coupling I with J in the others) and accumulates the rotation R; then A[P, Q] <- R_P^T A[P, Q] R_Q for every two pairs P, Q of the round
// (the diagonal blocks take S itself) and V[:, P] <- V[:, P] R_P.  An element
// rotation zeroes s_pq with t = sgn(tau)/(|tau| + sqrt(1 + tau^2)),
// tau = (s_qq - s_pp)/(2 s_pq) (symmetric Schur 2 x 2); s_pq, s_qp are set to
// zero and s_pp -= t s_pq, s_qq += t s_pq.  Indices past k are padding: their
// rows and columns are zero and never rotate.  Sweeps stop when the
// off-diagonal Frobenius norm is <= 1e-15 ||A||_F, after at most 60 sweeps
// (graded spectra converge linearly, about one decade per sweep).
constexpr int kBJ = 32;
constexpr int kBJ2 = 2 * kBJ;
constexpr int kBJThreads = 256;
typedef double bj_f64x4 __attribute__((ext_vector_type(4)));
static_assert(kBJThreads == 256 && kBJ2 == 64, "four waves, one 16-column block each");
constexpr int kBJMaxSweeps = 60;

__device__ inline void bj_pair(int nbp, int r, int t, int& I, int& J) {
    if (t == 0) {
        I = nbp - 1;
        J = r;
    } else {
        I = (r + t) % (nbp - 1);
        J = (r - t + (nbp - 1)) % (nbp - 1);
    }
    if (I > J) {
        const int x = I;
        I = J;
        J = x;
    }
}

// global index of local index s of block pair (I, J)
__device__ inline int bj_index(int I, int J, int s) { return s < kBJ ? I * kBJ + s : J * kBJ + (s - kBJ); }

// Frobenius norm squared (whole or off-diagonal) of each matrix.
__global__ __launch_bounds__(kDenseThreads) void k_bj_norm(const double* __restrict__ Aall, int kmax,
                                                           const int32_t* __restrict__ ks, int offdiag,
                                                           double* __restrict__ out) {
    __shared__ double red[kDenseThreads];
    const int b = blockIdx.x;
    const int k = ks ? ks[b] : kmax;
    const double* A = Aall + (int64_t)b * kmax * kmax;
    double f = 0.0;
    for (int i = threadIdx.y; i < k; i += blockDim.y)
        for (int j = threadIdx.x; j < k; j += blockDim.x)
            if (!offdiag || i != j) f += A[(int64_t)i * k + j] * A[(int64_t)i * k + j];
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    red[t] = f;
    __syncthreads();
    for (int o = kDenseThreads / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    if (t == 0) out[b] = red[0];
}

__global__ __launch_bounds__(kDenseThreads) void k_bj_identity(double* __restrict__ Vall, int kmax,
                                                               const int32_t* __restrict__ ks) {
    const int b = blockIdx.x;
    const int k = ks ? ks[b] : kmax;
    double* V = Vall + (int64_t)b * kmax * kmax;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) V[e] = (e / k == e % k) ? 1.0 : 0.0;
}

// Index pair (p < q) of rotation r in step `step` of a sweep on a block
// pair's subproblem: round robin over all 64 indices when full, else local
// index r paired with 32 + (r + step) mod 32.
__device__ inline void bj_step_pair(int full, int step, int r, int& p, int& q) {
    if (!full) {
        p = r;
        q = kBJ + (r + step) % kBJ;
    } else if (r == 0) {
        p = kBJ2 - 1;
        q = step;
    } else {   // 0 <= step < 63, 1 <= r < 32: one conditional subtraction reduces mod 63
        p = step + r;
        p -= p >= kBJ2 - 1 ? kBJ2 - 1 : 0;
        q = step - r + (kBJ2 - 1);
        q -= q >= kBJ2 - 1 ? kBJ2 - 1 : 0;
    }
    if (p > q) {
        const int x = p;
        p = q;
        q = x;
    }
}

// One rotation sweep on the subproblem of block pair blockIdx.x of round r of
// matrix blockIdx.y; R and S of the pair go to Rall and Sall.  full != 0:
// all 64 * 63 / 2 index pairs (63 steps of 32 disjoint pairs, round robin);
// else only the 32 * 32 pairs that couple I with J (step s pairs local index
// p with 32 + (p + s) mod 32).  A sweep uses full on its first round, so that
// every index pair of the matrix is visited at least once per sweep.
//
// The 32 rotations of a step are disjoint, so S <- J^T S J splits into 2 x 2
// blocks: block (a, b) = rows {p_a, q_a} x columns {p_b, q_b} takes rotation
// a on its rows and then rotation b on its columns (the same operations, in
// the same order, as rotating all rows first and all columns after), and the
// diagonal blocks take the 2 x 2 result.  Thread t owns column pair
// b = t mod 32 (whose rotation every lane computes itself) and the row pairs
// a = t / 32 + 8m, so each entry of S and R has one owner per step: two
// barriers per step, one LDS read and write of S and R.
__global__ __launch_bounds__(kBJThreads) void k_bj_solve(const double* __restrict__ Aall, int kmax,
                                                         const int32_t* __restrict__ ks, int nbp, int r,
                                                         int full, double* __restrict__ Rall,
                                                         double* __restrict__ Sall) {
    constexpr int kBlk = kBJ * kBJ / kBJThreads;    // 2 x 2 blocks of S per thread (4)
    constexpr int kRrow = kBJ2 * kBJ / kBJThreads;  // rows of R per thread (8)
    constexpr int kStride = kBJThreads / kBJ;       // between a thread's row pairs (8)
    __shared__ double S[kBJ2][kBJ2 + 1];
    __shared__ double Rm[kBJ2][kBJ2 + 1];
    __shared__ double cs[kBJ], sn[kBJ];
    const int b = blockIdx.y;
    const int k = ks ? ks[b] : kmax;
    const int t = threadIdx.x;
    int I, J;
    bj_pair(nbp, r, blockIdx.x, I, J);
    const double* A = Aall + (int64_t)b * kmax * kmax;
    for (int e = t; e < kBJ2 * kBJ2; e += kBJThreads) {
        const int s1 = e / kBJ2, s2 = e % kBJ2;
        const int g1 = bj_index(I, J, s1), g2 = bj_index(I, J, s2);
        S[s1][s2] = (g1 < k && g2 < k) ? A[(int64_t)g1 * k + g2] : 0.0;
        Rm[s1][s2] = s1 == s2 ? 1.0 : 0.0;
    }
    __syncthreads();
    const int rb = t % kBJ, ra0 = t / kBJ;
    const int nsteps = full ? kBJ2 - 1 : kBJ;
    for (int step = 0; step < nsteps; ++step) {
        // rotation rb from the step's S (symmetric Schur 2 x 2)
        int p, q;
        bj_step_pair(full, step, rb, p, q);
        double c = 1.0, sv = 0.0, tt = 0.0;
        const double apq = S[p][q], app = S[p][p], aqq = S[q][q];
        if (apq != 0.0) {
            const double diff = aqq - app;
            if (fabs(diff) > 1e150 * fabs(apq)) {
                tt = apq / diff;
            } else {
                const double tau = diff / (2.0 * apq);
                tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            }
            c = 1.0 / sqrt(1.0 + tt * tt);
            sv = tt * c;
        }
        const double dpp = app - tt * apq, dqq = aqq + tt * apq;
        if (t < kBJ) {
            cs[t] = c;
            sn[t] = sv;
        }
        __syncthreads();   // every rotation has read its entries before any is rewritten
#pragma unroll
        for (int m = 0; m < kBlk; ++m) {
            const int a = ra0 + kStride * m;
            int pa, qa;
            bj_step_pair(full, step, a, pa, qa);
            const double ca = cs[a], sa = sn[a];
            const double x00 = S[pa][p], x01 = S[pa][q], x10 = S[qa][p], x11 = S[qa][q];
            const double y00 = ca * x00 - sa * x10, y10 = sa * x00 + ca * x10;
            const double y01 = ca * x01 - sa * x11, y11 = sa * x01 + ca * x11;
            double z00 = c * y00 - sv * y01, z01 = sv * y00 + c * y01;
            double z10 = c * y10 - sv * y11, z11 = sv * y10 + c * y11;
            if (a == rb) {
                z00 = dpp;
                z01 = z10 = 0.0;
                z11 = dqq;
            }
            S[pa][p] = z00;
            S[pa][q] = z01;
            S[qa][p] = z10;
            S[qa][q] = z11;
        }
#pragma unroll
        for (int m = 0; m < kRrow; ++m) {
            const int i = ra0 + kStride * m;
            const double rp = Rm[i][p], rq = Rm[i][q];
            Rm[i][p] = c * rp - sv * rq;
            Rm[i][q] = sv * rp + c * rq;
        }
        __syncthreads();
    }
    const int64_t off = ((int64_t)b * (nbp / 2) + blockIdx.x) * kBJ2 * kBJ2;
    for (int e = t; e < kBJ2 * kBJ2; e += kBJThreads) {
        Rall[off + e] = Rm[e / kBJ2][e % kBJ2];
        Sall[off + e] = S[e / kBJ2][e % kBJ2];
    }
}

// C (64 x 64 per work-group, 4 x 4 per thread) = X^T Y or X Y for LDS tiles.
template <bool TRANS_X>
__device__ inline void bj_tile_product(const double (*X)[kBJ2 + 1], const double (*Y)[kBJ2 + 1],
                                       double (&acc)[4][4]) {
    // C = op(X) Y on the FP64 matrix cores: wave w forms columns [16 w, 16 w
    // + 16) of all four 16-row blocks; v_mfma_f64_16x16x4 lane l holds
    // A(l % 16, l / 16), B(l / 16, l % 16) and result register v is row
    // l / 16 + 4 v, column l % 16 of its block (bj_row / bj_col below)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bj_f64x4 c[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) c[rb] = bj_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int q = 0; q < kBJ2 / 4; ++q) {
        const int u = 4 * q + (lane >> 4);
        const double yv = Y[u][16 * wave + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int i = 16 * rb + (lane & 15);
            const double xv = TRANS_X ? X[u][i] : X[i][u];
            c[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, yv, c[rb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[rb][v] = c[rb][v];
}
// row and column of acc[rb][v] in the 64 x 64 product
__device__ inline int bj_row(int rb, int v) { return 16 * rb + ((threadIdx.x & 63) >> 4) + 4 * v; }
__device__ inline int bj_col() { return 16 * (threadIdx.x >> 6) + (threadIdx.x & 15); }

// Apply the round's rotations.  Work-groups [0, nA) take the pair blocks
// (P <= Q) of A: A[P, Q] <- R_P^T A[P, Q] R_Q and A[Q, P] its transpose, or S
// when P == Q; the rest take 64-row chunks of V: V[c, P] <- V[c, P] R_P.
__global__ __launch_bounds__(kBJThreads) void k_bj_apply(double* __restrict__ Aall,
                                                         double* __restrict__ Vall, int kmax,
                                                         const int32_t* __restrict__ ks, int nbp,
                                                         int r, const double* __restrict__ Rall,
                                                         const double* __restrict__ Sall) {
    __shared__ double X[kBJ2][kBJ2 + 1];
    __shared__ double Y[kBJ2][kBJ2 + 1];
    __shared__ double Z[kBJ2][kBJ2 + 1];
    const int b = blockIdx.y;
    const int k = ks ? ks[b] : kmax;
    const int npair = nbp / 2;
    const int nA = npair * (npair + 1) / 2;
    const int t = threadIdx.x;
    double* A = Aall + (int64_t)b * kmax * kmax;
    const double* Rb = Rall + (int64_t)b * npair * kBJ2 * kBJ2;
    int w = blockIdx.x;
    if (w < nA) {
        int P = 0;
        while (w >= npair - P) {   // upper-triangular enumeration of (P, Q)
            w -= npair - P;
            ++P;
        }
        const int Q = P + w;
        int I1, J1, I2, J2;
        bj_pair(nbp, r, P, I1, J1);
        bj_pair(nbp, r, Q, I2, J2);
        if (P == Q) {
            const double* Sp = Sall + ((int64_t)b * npair + P) * kBJ2 * kBJ2;
            for (int e = t; e < kBJ2 * kBJ2; e += kBJThreads) {
                const int g1 = bj_index(I1, J1, e / kBJ2), g2 = bj_index(I1, J1, e % kBJ2);
                if (g1 < k && g2 < k) A[(int64_t)g1 * k + g2] = Sp[e];
            }
            return;
        }
        const double* R1 = Rb + (int64_t)P * kBJ2 * kBJ2;
        const double* R2 = Rb + (int64_t)Q * kBJ2 * kBJ2;
        for (int e = t; e < kBJ2 * kBJ2; e += kBJThreads) {
            const int s1 = e / kBJ2, s2 = e % kBJ2;
            const int g1 = bj_index(I1, J1, s1), g2 = bj_index(I2, J2, s2);
            X[s1][s2] = R1[e];
            Y[s1][s2] = (g1 < k && g2 < k) ? A[(int64_t)g1 * k + g2] : 0.0;
            Z[s1][s2] = R2[e];
        }
        __syncthreads();
        double acc[4][4];
        bj_tile_product<true>(X, Y, acc);   // R_P^T A[P, Q]
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) Y[bj_row(a, q)][bj_col()] = acc[a][q];
        __syncthreads();
        bj_tile_product<false>(Y, Z, acc);   // (R_P^T A[P, Q]) R_Q
        const int g2 = bj_index(I2, J2, bj_col());
        if (g2 < k) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int g1 = bj_index(I1, J1, bj_row(a, q));
                    if (g1 >= k) continue;
                    A[(int64_t)g1 * k + g2] = acc[a][q];
                    A[(int64_t)g2 * k + g1] = acc[a][q];
                }
        }
        return;
    }
    w -= nA;
    const int P = w % npair;
    const int r0 = (w / npair) * kBJ2;
    if (r0 >= k) return;
    int I, J;
    bj_pair(nbp, r, P, I, J);
    double* V = Vall + (int64_t)b * kmax * kmax;
    const double* R = Rb + (int64_t)P * kBJ2 * kBJ2;
    for (int e = t; e < kBJ2 * kBJ2; e += kBJThreads) {
        const int i = e / kBJ2, s2 = e % kBJ2;
        const int g = bj_index(I, J, s2);
        X[i][s2] = (g < k && r0 + i < k) ? V[(int64_t)(r0 + i) * k + g] : 0.0;
        Y[i][s2] = R[e];
    }
    __syncthreads();
    double acc[4][4];
    bj_tile_product<false>(X, Y, acc);
    const int g = bj_index(I, J, bj_col());
    if (g < k) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = r0 + bj_row(a, q);
                if (i < k) V[(int64_t)i * k + g] = acc[a][q];
            }
    }
}

// Eigenvalues ascending by rank (ties broken by index), eigenvector columns with them.
__global__ __launch_bounds__(kDenseThreads) void k_bj_sort(const double* __restrict__ Aall,
                                                           const double* __restrict__ Vall,
                                                           double* __restrict__ wout,
                                                           double* __restrict__ Vout, int kmax,
                                                           const int32_t* __restrict__ ks) {
    __shared__ double wl[kDenseThreads];
    const int b = blockIdx.x;
    const int k = ks ? ks[b] : kmax;
    const double* A = Aall + (int64_t)b * kmax * kmax;
    const double* V = Vall + (int64_t)b * kmax * kmax;
    for (int j = threadIdx.x; j < k; j += blockDim.x) wl[j] = A[(int64_t)j * k + j];
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const double wj = wl[j];
        int rank = 0;
        for (int i = 0; i < k; ++i) rank += (wl[i] < wj) || (wl[i] == wj && i < j);
        wout[(int64_t)b * kmax + rank] = wj;
        double* Vo = Vout + (int64_t)b * kmax * kmax;
        for (int i = 0; i < k; ++i) Vo[(int64_t)i * k + rank] = V[(int64_t)i * k + j];
    }
}

size_t sym_eig_work_elems(int64_t kmax, int batch) {
    const int64_t nb = (kmax + kBJ - 1) / kBJ;
    const int64_t nbp = std::max<int64_t>(2, nb + (nb & 1));
    return (size_t)batch * kmax * kmax + 2 * (size_t)batch * (nbp / 2) * kBJ2 * kBJ2 + 2 * (size_t)batch;
}

hipError_t launch_sym_eig(double* A, double* w, double* V, int64_t kmax, int batch,
                          const int32_t* ks, double* work, hipStream_t s) {
    if (kmax <= 0 || batch <= 0) return hipSuccess;
    if (kmax > kDenseThreads) return hipErrorInvalidValue;
    const int nb = (int)((kmax + kBJ - 1) / kBJ);
    const int nbp = std::max(2, nb + (nb & 1));
    const int npair = nbp / 2;
    const int nA = npair * (npair + 1) / 2;
    const int nV = npair * (int)((kmax + kBJ2 - 1) / kBJ2);
    double* Vw = work;
    double* Rw = Vw + (size_t)batch * kmax * kmax;
    double* Sw = Rw + (size_t)batch * npair * kBJ2 * kBJ2;
    double* fro = Sw + (size_t)batch * npair * kBJ2 * kBJ2;
    double* off = fro + batch;
    hipLaunchKernelGGL(k_bj_identity, dim3(batch), dim3(kDenseThreads), 0, s, Vw, (int)kmax, ks);
    hipLaunchKernelGGL(k_bj_norm, dim3(batch), dim3(32, 32), 0, s, A, (int)kmax, ks, 0, fro);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::vector<double> fh(batch), oh(batch);
    e = hipMemcpyAsync(fh.data(), fro, sizeof(double) * batch, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    for (int sweep = 0; sweep < kBJMaxSweeps; ++sweep) {
        hipLaunchKernelGGL(k_bj_norm, dim3(batch), dim3(32, 32), 0, s, A, (int)kmax, ks, 1, off);
        e = hipMemcpyAsync(oh.data(), off, sizeof(double) * batch, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        bool done = true;
        for (int b = 0; b < batch; ++b) done &= !(oh[b] > 1e-30 * fh[b]);
        if (done) break;
        for (int r = 0; r < nbp - 1; ++r) {
            hipLaunchKernelGGL(k_bj_solve, dim3(npair, batch), dim3(kBJThreads), 0, s, A, (int)kmax, ks,
                               nbp, r, (int)(r == 0), Rw, Sw);
            hipLaunchKernelGGL(k_bj_apply, dim3(nA + nV, batch), dim3(kBJThreads), 0, s, A, Vw, (int)kmax,
                               ks, nbp, r, Rw, Sw);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bj_sort, dim3(batch), dim3(kDenseThreads), 0, s, A, Vw, w, V, (int)kmax, ks);
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
// Column sel[b] of X (n x k, row-major) -> out[b] (n), with the sign that
// makes its largest-modulus entry positive.  Entries within a relative 1e-4
// of the largest modulus count as tied and the lowest index among them
// decides (mirror-symmetric eigenvectors have exactly tied pairs whose
// computed moduli differ by the eigenvector's error, about 1e-7 for pairs
// accepted at residual 1e-8).  Two kernels: the gather, then the sign rule
// on the contiguous copies.

// out (n x m, column-major) = the columns sel of X: 64 x 64 tiles through
// LDS, so that both the reads along X's rows and the writes down out's
// columns are coalesced.  pmax[j * nrt + row tile] = max |entry| of column j
// over the tile's rows.
__global__ __launch_bounds__(256) void k_gather_tile(const double* __restrict__ X, int64_t n, int k,
                                                     const int32_t* __restrict__ sel, int m,
                                                     double* __restrict__ out, double* __restrict__ pmax) {
    __shared__ double tl[64][65];
    __shared__ double mx[4][64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int j = j0 + lane;
    const int c = j < m ? sel[j] : 0;
    double best = 0.0;
    for (int r = wave; r < 64; r += 4) {
        const int64_t i = i0 + r;
        const double x = (i < n && j < m) ? X[i * k + c] : 0.0;
        tl[r][lane] = x;
        best = fmax(best, fabs(x));
    }
    mx[wave][lane] = best;
    __syncthreads();
    if (wave == 0 && j < m)
        pmax[(int64_t)j * gridDim.x + blockIdx.x] = fmax(fmax(mx[0][lane], mx[1][lane]), fmax(mx[2][lane], mx[3][lane]));
    for (int q = wave; q < 64; q += 4) {
        const int jj = j0 + q;
        const int64_t i = i0 + lane;
        if (jj < m && i < n) out[(int64_t)jj * n + i] = tl[lane][q];
    }
}

// Sign of each gathered column (one work-group per column): the largest
// modulus from the row tiles' maxima, then the first row tile that reaches
// the tie threshold and, inside it, the first such row; sgn[j] = -1 when
// that entry is negative.
__global__ __launch_bounds__(256) void k_sign_cols(int64_t n, int nrt, const double* __restrict__ pmax,
                                                   const double* __restrict__ out, double* __restrict__ sgn) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int t = threadIdx.x;
    const double* pm = pmax + (int64_t)blockIdx.x * nrt;
    double best = 0.0;
    for (int b = t; b < nrt; b += 256) best = fmax(best, pm[b]);
    bv[t] = best;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) bv[t] = fmax(bv[t], bv[t + off]);
        __syncthreads();
    }
    const double thr = (1.0 - 1e-4) * bv[0];
    int fb = nrt;
    for (int b = t; b < nrt; b += 256)
        if (pm[b] >= thr) {
            fb = b;
            break;
        }
    bi[t] = fb;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) bi[t] = min(bi[t], bi[t + off]);
        __syncthreads();
    }
    const int b0 = bi[0] < nrt ? bi[0] : 0;
    __syncthreads();   // every thread has read bi[0]
    const double* o = out + (int64_t)blockIdx.x * n;
    const int64_t i = (int64_t)b0 * 64 + t;
    bi[t] = (t < 64 && i < n && fabs(o[i]) >= thr) ? t : 64;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) bi[t] = min(bi[t], bi[t + off]);
        __syncthreads();
    }
    if (t == 0) {
        const int64_t at = (int64_t)b0 * 64 + (bi[0] < 64 ? bi[0] : 0);
        sgn[blockIdx.x] = (at < n && o[at] < 0.0) ? -1.0 : 1.0;
    }
}

// out[:, j] *= sgn[j] where sgn[j] < 0.
__global__ __launch_bounds__(256) void k_flip_cols(int64_t n, const double* __restrict__ sgn,
                                                   double* __restrict__ out) {
    const int j = blockIdx.y;
    if (sgn[j] > 0.0) return;   // uniform over the work-group
    double* o = out + (int64_t)j * n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) o[i] = -o[i];
}

size_t gather_cols_work(int64_t n, int m) { return (size_t)((n + 63) / 64) * m + m; }

hipError_t launch_gather_cols(const double* X, int64_t n, int64_t k, const int32_t* sel, int m,
                              double* out, double* work, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int nrt = (int)((n + 63) / 64);
    double* pmax = work;
    double* sg = work + (size_t)nrt * m;
    hipLaunchKernelGGL(k_gather_tile, dim3((unsigned)nrt, (unsigned)((m + 63) / 64)), dim3(256), 0, s, X, n,
                       (int)k, sel, m, out, pmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sign_cols, dim3(m), dim3(256), 0, s, n, nrt, pmax, out, sg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_flip_cols, dim3((unsigned)std::min<int64_t>(64, (n + 255) / 256), m), dim3(256), 0, s, n,
                       sg, out);
    return hipGetLastError();
}

}  // namespace gep
