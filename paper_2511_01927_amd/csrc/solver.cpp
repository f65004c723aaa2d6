// Host orchestrator and C ABI of the contour-integral eigensolver.
//
// Pipeline per wave of contours (paper Appendix, Alg. "Standard CI pipeline
// with contour partitioning and orthogonalization", moment matrices S_m):
//   pack pencil -> V, B V -> batched COCG over (contour, node, rhs) columns
//   -> moments -> SVQB + Cholesky B-orthonormalisation -> Rayleigh-Ritz ->
//   residuals -> keep-window selection -> optional FEAST-type refinement ->
//   merge.  All arithmetic on the pencil-sized data runs in the HIP kernels
//   of this library; the host validates, plans memory, launches, and makes
//   the O(r)-sized decisions (rank cut, window selection, merge).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/gep_ci.h"
#include "internal.h"

namespace gep {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

struct Fail {
    int code;
};

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                 \
            throw Fail{GEP_EDEVICE};                                                      \
        }                                                                                 \
    } while (0)

[[noreturn]] static void fail(int code, const std::string& msg) {
    set_error(msg);
    throw Fail{code};
}

// Device workspace kept by a packed pencil across its solves.  A solve of
// the same shapes as an earlier one then takes every buffer from here instead
// of calling hipMalloc / hipFree (tens of GB per solve on the 2D headline,
// whose per-solve allocation made the solve time erratic).  The pool is a
// best-fit allocator over the chunks it has obtained from hipMalloc: a
// request is carved from the smallest free range that holds it (256-byte
// granules), a freed range merges with its free neighbours in its chunk,
// and a new chunk is allocated only when no free range is large enough.
// Chunks are kept until the pencil is freed (memory given back with
// hipFree was measured not to become allocatable again right away, so a
// multi-wave solve whose waves have different shapes must reuse it).  A
// buffer handed back is first made idle with a device synchronisation, the
// same wait that hipFree performs, so a later request can never reuse
// memory that queued work still touches.
struct DevPool {
    std::mutex mu;
    std::map<char*, size_t> chunks;              // hipMalloc'd regions: start -> bytes
    std::map<char*, size_t> free_at;             // free ranges: start -> bytes
    std::multimap<size_t, char*> free_by_size;   // the same ranges by size
    size_t idle_bytes = 0;   // in free ranges
    size_t live_bytes = 0;   // handed out and not given back
    long reused = 0, allocated = 0;
    int verbose = 0;   // > 1: log requests of 1 GB and more on stderr
    static constexpr size_t kGranule = 256;

    void erase_free(char* a, size_t sz) {
        free_at.erase(a);
        auto r = free_by_size.equal_range(sz);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == a) {
                free_by_size.erase(it);
                break;
            }
        idle_bytes -= sz;
    }
    void insert_free(char* a, size_t sz) {
        free_at[a] = sz;
        free_by_size.emplace(sz, a);
        idle_bytes += sz;
    }
    // start of the chunk holding address a
    char* chunk_of(char* a) const {
        auto it = chunks.upper_bound(a);
        return std::prev(it)->first;
    }
    size_t largest_free() {
        std::lock_guard<std::mutex> lk(mu);
        return free_by_size.empty() ? 0 : free_by_size.rbegin()->first;
    }
    // One chunk of `bytes` unless a free range that large exists already
    // (called at the start of a solve with what its largest wave needs, so
    // that every wave is carved from one region).  Failure is not an error:
    // requests then get chunks of their own.
    void reserve(size_t bytes) {
        bytes = (bytes + kGranule - 1) / kGranule * kGranule;
        if (bytes == 0 || largest_free() >= bytes) return;
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        std::lock_guard<std::mutex> lk(mu);
        chunks[(char*)q] = bytes;
        insert_free((char*)q, bytes);
        ++allocated;
    }
    // top != 0: carve from the top end of the highest free range that holds
    // the request (buffers that outlive a wave stay out of the way of the
    // next wave's large requests)
    void* take(size_t bytes, size_t& cap, bool top = false) {
        const size_t need = (std::max<size_t>(bytes, 1) + kGranule - 1) / kGranule * kGranule;
        if (top) {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = free_at.rbegin(); it != free_at.rend(); ++it) {
                if (it->second < need) continue;
                char* start = it->first;
                const size_t sz = it->second;
                erase_free(start, sz);
                if (sz > need) insert_free(start, sz - need);
                cap = need;
                live_bytes += need;
                ++reused;
                return start + (sz - need);
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free_by_size.lower_bound(need);
            if (verbose > 1 && need >= (size_t(1) << 30))
                std::fprintf(stderr, "[gep] pool take %.2f GB: %s (live %.2f GB, free ranges %.2f GB, largest %.2f GB)\n",
                             need / 1e9, it != free_by_size.end() ? "reuse" : "new chunk", live_bytes / 1e9,
                             idle_bytes / 1e9, free_by_size.empty() ? 0.0 : free_by_size.rbegin()->first / 1e9);
            if (it != free_by_size.end()) {
                char* a = it->second;
                const size_t sz = it->first;
                erase_free(a, sz);
                if (sz > need) insert_free(a + need, sz - need);
                cap = need;
                live_bytes += need;
                ++reused;
                return a;
            }
        }
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, need);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            trim();
            e = hipMalloc(&q, need);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            size_t fb = 0, tb = 0;
            (void)hipMemGetInfo(&fb, &tb);
            fail(e == hipErrorOutOfMemory ? GEP_ENOMEM : GEP_EDEVICE,
                 "hipMalloc of " + std::to_string(need) + " bytes failed: " + hipGetErrorString(e) +
                     " (workspace pool: " + std::to_string(live_bytes) + " bytes in use, " +
                     std::to_string(idle_bytes) + " free in its chunks; device free " + std::to_string(fb) + ")");
        }
        std::lock_guard<std::mutex> lk(mu);
        chunks[(char*)q] = need;
        cap = need;
        live_bytes += need;
        ++allocated;
        return q;
    }
    void give(void* q, size_t cap) {
        (void)hipDeviceSynchronize();
        std::lock_guard<std::mutex> lk(mu);
        char* a = (char*)q;
        size_t sz = cap;
        live_bytes -= cap;
        char* c0 = chunk_of(a);
        char* c1 = c0 + chunks[c0];
        // merge with the free range after it and the one before it (same chunk)
        auto nx = free_at.find(a + sz);
        if (nx != free_at.end() && nx->first < c1) {
            const size_t s2 = nx->second;
            erase_free(nx->first, s2);
            sz += s2;
        }
        auto pv = free_at.lower_bound(a);
        if (pv != free_at.begin()) {
            --pv;
            if (pv->first >= c0 && pv->first + pv->second == a) {
                char* pa = pv->first;
                const size_t s2 = pv->second;
                erase_free(pa, s2);
                a = pa;
                sz += s2;
            }
        }
        insert_free(a, sz);
    }
    // give back to the runtime every chunk that is entirely free
    void trim() {
        (void)hipDeviceSynchronize();
        if (verbose > 1) std::fprintf(stderr, "[gep] pool trim (free ranges %.2f GB)\n", idle_bytes / 1e9);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = chunks.begin(); it != chunks.end();) {
                auto f = free_at.find(it->first);
                if (f != free_at.end() && f->second == it->second) {
                    erase_free(it->first, it->second);
                    (void)hipFree(it->first);
                    it = chunks.erase(it);
                } else {
                    ++it;
                }
            }
        }
        (void)hipDeviceSynchronize();
    }
    ~DevPool() { trim(); }
};

// Pool that DBuf allocations of the calling thread use (set for the duration
// of a solve on a packed pencil; null: plain hipMalloc / hipFree).
static thread_local DevPool* t_pool = nullptr;
static thread_local bool t_pool_top = false;
struct PoolScope {
    DevPool* prev;
    explicit PoolScope(DevPool* p) : prev(t_pool) { t_pool = p; }
    ~PoolScope() { t_pool = prev; }
};
// Buffers allocated in this scope outlive the current wave of a solve.
struct LongLived {
    bool prev;
    LongLived() : prev(t_pool_top) { t_pool_top = true; }
    ~LongLived() { t_pool_top = prev; }
};

// RAII device buffer (from the thread's current pool when one is set)
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DevPool* pool = nullptr;
    size_t cap = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    void alloc(size_t count) {
        release();
        n = count;
        if (!count) return;
        if (t_pool) {
            pool = t_pool;
            p = static_cast<T*>(pool->take(count * sizeof(T), cap, t_pool_top));
            return;
        }
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(e == hipErrorOutOfMemory ? GEP_ENOMEM : GEP_EDEVICE,
                 "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " +
                     hipGetErrorString(e) + " (outside the workspace pool)");
        }
    }
    void release() {
        if (p) {
            if (pool)
                pool->give(p, cap);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        pool = nullptr;
        n = 0;
        cap = 0;
    }
    ~DBuf() { release(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    T* get() const { return p; }
};

// Host copy of the packed pencil (needed for validation and the merge).
// A batch of pencils is stored as one block-diagonal pencil: problem p owns
// rows [prob_row0[p], prob_row0[p] + prob_n[p]) and its column indices are
// global.
struct HostPencil {
    int64_t n = 0, nnz = 0;
    std::vector<int32_t> rowptr, colind;
    std::vector<double> a, b;
    std::vector<double> dA, dB;
    double a_inf = 0.0;
    int max_row = 0;
    std::vector<int64_t> prob_row0, prob_n;
    std::vector<double> prob_ainf;
    std::vector<int32_t> prob_g4;   // first 4-row group of each problem (set by upload)
    // lower bands of the problems (set by upload): half bandwidth, element
    // offset of the (a, b) band on the device, -1 when no band is kept
    std::vector<int32_t> prob_bw;
    std::vector<int64_t> prob_boff;
};

static void append_pencil(HostPencil& dst, const HostPencil& src) {
    const int64_t r0 = dst.n;
    const int32_t e0 = dst.rowptr.empty() ? 0 : dst.rowptr.back();
    if (dst.rowptr.empty()) dst.rowptr.push_back(0);
    for (int64_t i = 0; i < src.n; ++i) dst.rowptr.push_back(e0 + src.rowptr[i + 1]);
    for (int32_t c : src.colind) dst.colind.push_back((int32_t)(c + r0));
    dst.a.insert(dst.a.end(), src.a.begin(), src.a.end());
    dst.b.insert(dst.b.end(), src.b.begin(), src.b.end());
    dst.dA.insert(dst.dA.end(), src.dA.begin(), src.dA.end());
    dst.dB.insert(dst.dB.end(), src.dB.begin(), src.dB.end());
    dst.n += src.n;
    dst.nnz += src.nnz;
    dst.a_inf = std::max(dst.a_inf, src.a_inf);
    dst.max_row = std::max(dst.max_row, src.max_row);
    dst.prob_row0.push_back(r0);
    dst.prob_n.push_back(src.n);
    dst.prob_ainf.push_back(src.a_inf);
}

// ---- per-kernel-class timing with HIP events -----------------------------
struct Timer {
    bool on = false;
    hipStream_t s = nullptr;
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    static constexpr int kClasses = 13;
    double ms[kClasses] = {0};
    long count[kClasses] = {0};   // timed brackets
    long seen[kClasses] = {0};    // all brackets
    int stride[kClasses] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};   // time every stride-th bracket
    // per-class totals: the timed mean times the number of brackets
    double total_ms(int c) const { return count[c] ? ms[c] * (double)seen[c] / (double)count[c] : 0.0; }
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        return e;
    }
    int open_cls = -1;
    hipEvent_t open_a = nullptr;
    hipStream_t open_s = nullptr;
    // begin / end bracket one launch (or a run of launches) on stream st
    // (the solver's stream by default)
    void begin(int cls, hipStream_t st = nullptr) {
        if (!on) return;
        if (seen[cls]++ % stride[cls] != 0) {
            open_cls = -1;
            return;
        }
        open_cls = cls;
        open_s = st ? st : s;
        open_a = get();
        HIPCHK(hipEventRecord(open_a, open_s));
    }
    void end() {
        if (!on || open_cls < 0) return;
        hipEvent_t b = get();
        HIPCHK(hipEventRecord(b, open_s));
        pending.push_back({open_cls, open_a, b});
    }
    // Events to attach to the next dispatch of class cls (hipExtLaunchKernel
    // start / stop: the kernel's own execution), or null when this dispatch
    // is not sampled.
    void kernel_pair(int cls, hipEvent_t& a, hipEvent_t& b) {
        a = b = nullptr;
        if (!on || seen[cls]++ % stride[cls] != 0) return;
        a = get();
        b = get();
        pending.push_back({cls, a, b});
    }
    // call after a stream synchronisation
    void flush() {
        for (auto& r : pending) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            count[r.cls] += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    ~Timer() {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
enum { T_SPMM = 0, T_UPDATE, T_REPLACE, T_REDUCE, T_MOMENTS, T_GRAM, T_GEMM, T_DENSE, T_BAND_PANEL,
       T_BAND_UPDATE, T_BAND_SOLVE, T_BAND_NEXT, T_BAND_WIDE };
static const char* kTimerNames[Timer::kClasses] = {"cocg_spmm_dir", "cocg_update", "cocg_replace",
                                                   "cocg_reduce", "moments", "gram",
                                                   "gemm_tall", "dense_small", "band_panel",
                                                   "band_update", "band_solve", "band_update_next",
                                                   "band_factor_wide"};

// Algorithmic real flops of the banded L D L^T of one n x n complex
// symmetric system of half bandwidth bw, split between the panel kernel
// (column scaling, 6 flops per complex product, and the updates inside a
// panel) and the trailing-window kernel (8 flops per complex multiply-add
// l_ik d_k l_jk, counted only where l_ik is inside the band).
// update: the contributions to the two columns panels after each panel
// (strip updates, next) and to the rest of its window (rest).
static void band_factor_flops(int64_t n, int64_t bw, double& panel, double& next, double& rest) {
    panel = next = rest = 0.0;
    for (int64_t k0 = 0; k0 < n; k0 += kPanel) {
        const int64_t nc = std::min<int64_t>(kPanel, n - k0);
        for (int64_t jj = 0; jj < nc; ++jj) {
            const int64_t e = std::min<int64_t>(bw, n - 1 - (k0 + jj));
            panel += 6.0 * e;
            const int64_t left = std::min<int64_t>(nc - 1 - jj, e);
            for (int64_t t = 1; t <= left; ++t) panel += 8.0 * (e - t + 1);
        }
        const int64_t w0 = k0 + kPanel, wend = std::min<int64_t>(n, k0 + kPanel + bw);
        for (int64_t i = w0; i < wend; ++i) {
            const int64_t kmin = std::max<int64_t>(k0, i - bw);
            const int64_t c = std::max<int64_t>(0, k0 + kPanel - kmin);
            const int64_t cols = i - w0 + 1;   // target columns w0 .. i
            const int64_t near = std::min<int64_t>(cols, 2 * kPanel);
            next += 8.0 * (double)c * (double)near;
            rest += 8.0 * (double)c * (double)(cols - near);
        }
    }
}

// Algorithmic real flops of one forward + backward band solve of one column.
static double band_solve_flops(int64_t n, int64_t bw) {
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) f += 16.0 * (double)std::min<int64_t>(bw, n - 1 - i) + 9.0;
    return f;
}

}  // namespace gep

using namespace gep;

struct gep_pencil {
    HostPencil h;
    DevPencil d;
    std::vector<void*> owned;
    gep::DevPool pool;   // solve workspace kept between solves
    // second stream and events of the band factorisation's lookahead and the
    // pinned read-back words of the COCG loop, created on first use and kept
    // for later solves
    hipStream_t aux = nullptr;
    hipEvent_t ev_panel = nullptr, ev_rest[2] = {nullptr, nullptr};
    // the banded factorisation's launches as a graph, for the layout in the key
    hipGraphExec_t band_graph = nullptr;
    std::vector<int64_t> band_graph_key;
    int band_graph_steps = 0;
    int32_t* counts_h = nullptr;
    ~gep_pencil() {
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (band_graph) (void)hipGraphExecDestroy(band_graph);
        if (ev_panel) (void)hipEventDestroy(ev_panel);
        for (hipEvent_t e : ev_rest)
            if (e) (void)hipEventDestroy(e);
        if (counts_h) (void)hipHostFree(counts_h);
        pool.trim();
        for (void* p : owned) (void)hipFree(p);
    }
};

struct gep_result {
    int64_t n = 0, m = 0;
    std::vector<double> evals, resid;
    std::unique_ptr<gep::DBuf<double>> dvecs;   // eigenvectors on the device, n x m column-major
    mutable bool copy_enqueued = false;           // a device copy of dvecs may be in flight
    std::vector<int32_t> cid;
    std::vector<uint8_t> conv;
    std::vector<uint8_t> csat;   // per contour: subspace saturated
    std::vector<double> filt;    // per pair: quadrature filter value at its eigenvalue
    std::string stats;
};

namespace gep {

// ---- validation and packing ---------------------------------------------
static void fetch_csr(const gep_csr* M, bool on_dev, std::vector<int64_t>& rp,
                      std::vector<int32_t>& ci, std::vector<double>& v, const char* name) {
    if (!M || !M->rowptr || !M->colind || !M->val) fail(GEP_EINVAL, std::string(name) + ": NULL pointer");
    if (M->n <= 0 || M->nnz < 0) fail(GEP_EINVAL, std::string(name) + ": n <= 0 or nnz < 0");
    if (M->n >= (1ll << 31) - 1 || M->nnz >= (1ll << 31) - 1)
        fail(GEP_EINVAL, std::string(name) + ": n or nnz >= 2^31");
    rp.resize(M->n + 1);
    ci.resize(M->nnz);
    v.resize(M->nnz);
    if (on_dev) {
        HIPCHK(hipMemcpy(rp.data(), M->rowptr, sizeof(int64_t) * (M->n + 1), hipMemcpyDeviceToHost));
        if (M->nnz) {
            HIPCHK(hipMemcpy(ci.data(), M->colind, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(v.data(), M->val, sizeof(double) * M->nnz, hipMemcpyDeviceToHost));
        }
    } else {
        std::memcpy(rp.data(), M->rowptr, sizeof(int64_t) * (M->n + 1));
        if (M->nnz) {
            std::memcpy(ci.data(), M->colind, sizeof(int32_t) * M->nnz);
            std::memcpy(v.data(), M->val, sizeof(double) * M->nnz);
        }
    }
    if (rp[0] != 0 || rp[M->n] != M->nnz) fail(GEP_EINVAL, std::string(name) + ": rowptr ends wrong");
    for (int64_t i = 0; i < M->n; ++i) {
        if (rp[i + 1] < rp[i]) fail(GEP_EINVAL, std::string(name) + ": rowptr not monotone");
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= M->n) fail(GEP_EINVAL, std::string(name) + ": column index out of range");
            if (e > rp[i] && ci[e] <= ci[e - 1])
                fail(GEP_EINVAL, std::string(name) + ": column indices not strictly ascending");
            if (!std::isfinite(v[e])) fail(GEP_EINVAL, std::string(name) + ": non-finite value");
        }
    }
}

static double csr_get(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                      const std::vector<double>& v, int64_t i, int32_t j) {
    auto b = ci.begin() + rp[i], e = ci.begin() + rp[i + 1];
    auto it = std::lower_bound(b, e, j);
    if (it != e && *it == j) return v[it - ci.begin()];
    return 0.0;
}

static void check_sym(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                      const std::vector<double>& v, int64_t n, const char* name) {
    double amax = 0.0;
    for (double x : v) amax = std::max(amax, std::fabs(x));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const double t = csr_get(rp, ci, v, ci[e], (int32_t)i);
            if (std::fabs(v[e] - t) > 1e-12 * amax)
                fail(GEP_ENOTSYM, std::string(name) + " is not symmetric at (" + std::to_string(i) +
                                      "," + std::to_string(ci[e]) + ")");
        }
}

static void pack(const gep_csr* A, const gep_csr* B, bool on_dev, HostPencil& H) {
    std::vector<int64_t> ra, rb;
    std::vector<int32_t> ca, cb;
    std::vector<double> va, vb;
    fetch_csr(A, on_dev, ra, ca, va, "A");
    fetch_csr(B, on_dev, rb, cb, vb, "B");
    if (A->n != B->n) fail(GEP_EINVAL, "A and B differ in size");
    const int64_t n = A->n;
    check_sym(ra, ca, va, n, "A");
    check_sym(rb, cb, vb, n, "B");
    H.n = n;
    H.rowptr.assign(n + 1, 0);
    H.colind.clear();
    H.a.clear();
    H.b.clear();
    H.dA.assign(n, 0.0);
    H.dB.assign(n, 0.0);
    H.a_inf = 0.0;
    H.max_row = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t ea = ra[i], eb = rb[i];
        double rowsum = 0.0;
        while (ea < ra[i + 1] || eb < rb[i + 1]) {
            const int32_t ja = ea < ra[i + 1] ? ca[ea] : INT32_MAX;
            const int32_t jb = eb < rb[i + 1] ? cb[eb] : INT32_MAX;
            const int32_t j = std::min(ja, jb);
            const double av = (ja == j) ? va[ea++] : 0.0;
            const double bv = (jb == j) ? vb[eb++] : 0.0;
            H.colind.push_back(j);
            H.a.push_back(av);
            H.b.push_back(bv);
            rowsum += std::fabs(av);
            if (j == i) {
                H.dA[i] = av;
                H.dB[i] = bv;
            }
        }
        H.rowptr[i + 1] = (int32_t)H.colind.size();
        H.max_row = std::max(H.max_row, H.rowptr[i + 1] - H.rowptr[i]);
        H.a_inf = std::max(H.a_inf, rowsum);
        if (!(H.dB[i] > 0.0)) fail(GEP_ENOTSPD, "B has a non-positive diagonal entry at row " + std::to_string(i));
    }
    H.nnz = (int64_t)H.colind.size();
    if (H.nnz >= (1ll << 31) - 1) fail(GEP_EINVAL, "union pattern nnz >= 2^31");
    H.prob_row0 = {0};
    H.prob_n = {n};
    H.prob_ainf = {H.a_inf};
}

static void upload(const HostPencil& H, gep_pencil* P) {
    DevPencil& D = P->d;
    D.n = H.n;
    D.nnz = H.nnz;
    D.a_inf = H.a_inf;
    D.max_row_nnz = H.max_row;
    auto dalloc = [&](size_t bytes) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(e == hipErrorOutOfMemory ? GEP_ENOMEM : GEP_EDEVICE,
                 std::string("hipMalloc failed while packing the pencil: ") + hipGetErrorString(e));
        }
        P->owned.push_back(p);
        return p;
    };
    D.rowptr = (int32_t*)dalloc(sizeof(int32_t) * (H.n + 1));
    D.colind = (int32_t*)dalloc(sizeof(int32_t) * H.nnz);
    D.ab = (double2*)dalloc(sizeof(double2) * H.nnz);
    D.ab32 = (float2*)dalloc(sizeof(float2) * H.nnz);
    D.dA = (double*)dalloc(sizeof(double) * H.n);
    D.dB = (double*)dalloc(sizeof(double) * H.n);
    std::vector<double2> ab(H.nnz);
    std::vector<float2> ab32(H.nnz);
    for (int64_t e = 0; e < H.nnz; ++e) {
        ab[e] = make_double2(H.a[e], H.b[e]);
        ab32[e] = make_float2((float)H.a[e], (float)H.b[e]);
    }
    HIPCHK(hipMemcpy(D.rowptr, H.rowptr.data(), sizeof(int32_t) * (H.n + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.colind, H.colind.data(), sizeof(int32_t) * H.nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.ab, ab.data(), sizeof(double2) * H.nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.ab32, ab32.data(), sizeof(float2) * H.nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.dA, H.dA.data(), sizeof(double) * H.n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.dB, H.dB.data(), sizeof(double) * H.n, hipMemcpyHostToDevice));
    // 4-row groups of each problem: sorted union of the rows' columns and a
    // 4-wide coefficient block per union column (zero where a row has no entry)
    constexpr int G = 4;
    std::vector<int32_t> gptr(1, 0), gcol, cols;
    std::vector<double2> gab;
    std::vector<int32_t> g0;
    for (size_t pi = 0; pi < H.prob_row0.size(); ++pi) {
        g0.push_back((int32_t)(gptr.size() - 1));
        const int64_t r0 = H.prob_row0[pi], r1 = r0 + H.prob_n[pi];
        for (int64_t gr = r0; gr < r1; gr += G) {
            const int64_t ge = std::min(r1, gr + G);
            cols.clear();
            for (int64_t i = gr; i < ge; ++i)
                cols.insert(cols.end(), H.colind.begin() + H.rowptr[i], H.colind.begin() + H.rowptr[i + 1]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            int32_t cur[G];
            for (int r = 0; r < G; ++r) cur[r] = gr + r < ge ? H.rowptr[gr + r] : 0;
            for (int32_t c : cols) {
                gcol.push_back(c);
                for (int r = 0; r < G; ++r) {
                    double2 v = make_double2(0.0, 0.0);
                    if (gr + r < ge && cur[r] < H.rowptr[gr + r + 1] && H.colind[cur[r]] == c) {
                        v = make_double2(H.a[cur[r]], H.b[cur[r]]);
                        ++cur[r];
                    }
                    gab.push_back(v);
                }
            }
            if ((int64_t)gcol.size() >= (1ll << 31) - 1) fail(GEP_EINVAL, "row-group pattern >= 2^31");
            gptr.push_back((int32_t)gcol.size());
        }
    }
    P->h.prob_g4 = g0;
    // column-major lower bands (a_ij, b_ij), 0 <= i - j <= bw, of every problem
    // whose half bandwidth is at most kBandMaxBw
    {
        std::vector<int32_t> pbw(H.prob_row0.size(), 0);
        std::vector<int64_t> poff(H.prob_row0.size(), -1);
        int64_t total = 0;
        for (size_t pi = 0; pi < H.prob_row0.size(); ++pi) {
            const int64_t r0 = H.prob_row0[pi], r1 = r0 + H.prob_n[pi];
            int64_t bw = 0;
            for (int64_t i = r0; i < r1; ++i)
                for (int32_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e)
                    bw = std::max<int64_t>(bw, std::llabs((int64_t)H.colind[e] - i));
            pbw[pi] = (int32_t)std::min<int64_t>(bw, INT32_MAX);
            if (bw <= kBandWideBw) {   // wider bands are formed from the CSR rows
                poff[pi] = total;
                total += H.prob_n[pi] * (bw + 1);
            }
        }
        if (total > 0) {
            std::vector<double2> band((size_t)total, make_double2(0.0, 0.0));
            for (size_t pi = 0; pi < H.prob_row0.size(); ++pi) {
                if (poff[pi] < 0) continue;
                const int64_t r0 = H.prob_row0[pi], r1 = r0 + H.prob_n[pi];
                const int64_t ld = pbw[pi] + 1;
                for (int64_t i = r0; i < r1; ++i)
                    for (int32_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) {
                        const int64_t j = H.colind[e];
                        if (j > i) continue;
                        band[poff[pi] + (j - r0) * ld + (i - j)] = make_double2(H.a[e], H.b[e]);
                    }
            }
            D.band = (double2*)dalloc(sizeof(double2) * band.size());
            HIPCHK(hipMemcpy(D.band, band.data(), sizeof(double2) * band.size(), hipMemcpyHostToDevice));
        }
        P->h.prob_bw = pbw;
        P->h.prob_boff = poff;
    }
    D.g4nnz = (int64_t)gcol.size();
    D.auto_grp = (double)D.g4nnz <= 0.8 * (double)H.nnz ? G : 1;
    D.g4ptr = (int32_t*)dalloc(sizeof(int32_t) * gptr.size());
    D.g4col = (int32_t*)dalloc(sizeof(int32_t) * gcol.size());
    D.g4ab = (double2*)dalloc(sizeof(double2) * gab.size());
    D.g4ab32 = (float2*)dalloc(sizeof(float2) * gab.size());
    std::vector<float2> gab32(gab.size());
    for (size_t e = 0; e < gab.size(); ++e) gab32[e] = make_float2((float)gab[e].x, (float)gab[e].y);
    HIPCHK(hipMemcpy(D.g4ptr, gptr.data(), sizeof(int32_t) * gptr.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.g4col, gcol.data(), sizeof(int32_t) * gcol.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.g4ab, gab.data(), sizeof(double2) * gab.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(D.g4ab32, gab32.data(), sizeof(float2) * gab.size(), hipMemcpyHostToDevice));
}

// The row-group view a solve uses: rg = 0 picks the pencil's automatic choice.
static DevPencil group_view(const DevPencil& D, int rg) {
    DevPencil v = D;
    v.grp = rg == 0 ? D.auto_grp : rg;
    if (v.grp == 4) {
        v.gptr = D.g4ptr;
        v.gcol = D.g4col;
        v.gab = D.g4ab;
        v.gab32 = D.g4ab32;
    } else {
        v.grp = 1;
        v.gptr = D.rowptr;
        v.gcol = D.colind;
        v.gab = D.ab;
        v.gab32 = D.ab32;
    }
    return v;
}

// ---- solve ----------------------------------------------------------------
struct SolveCfg {
    int N = 0, NH = 0, M = 0, L = 0;
    double tol = 1e-8;
    gep_opts o;
};

// One contour of one pencil of the batch.
struct Job {
    gep_contour c{};
    int prob = 0;        // problem index in the batch
    int id = 0;          // contour index within its problem
    int64_t row0 = 0;    // first row of the problem in the concatenated pencil
    int64_t n = 0;       // rows of the problem
    int64_t bsrc0 = 0;   // offset in B V of this job's right-hand side 0 at row 0
    int L = 0;           // right-hand sides (block size) of this job
};

struct ContourOut {
    int id = 0;
    int prob = 0;
    int passes = 0;
    std::vector<int> rank;
    bool saturated = false;
    double smin_ratio = 0.0;
    std::vector<double> theta, rho;      // all Ritz pairs of the last pass
    std::shared_ptr<DBuf<double>> Xbuf;  // owner of the Ritz vectors of the last pass
    double* X = nullptr;                 // n x r row-major Ritz vectors (inside Xbuf)
    int r = 0;
    long iters_max = 0;
    double iters_mean = 0.0;
};

struct Stats {
    long cocg_iters = 0;          // iterations of the COCG loop (all passes)
    long ms_iters = 0;            // iterations of the multi-shift COCG seed recurrences (all passes)
    long ms_unconverged = 0;      // shifted columns above solve_tol when the multi-shift loop stopped
    long tile_iters = 0;          // sum over tiles of iterations run
    long spmm_launches = 0;
    long replacements = 0;
    long graph_captures = 0;
    double spmm_alg_bytes = 0.0;  // algorithmic bytes of all shifted SpMM launches
    double update_alg_bytes = 0.0;
    double replace_alg_bytes = 0.0;
    long columns = 0;
    int waves = 0;
    long fp32_passes = 0;         // passes whose shifted solves ran in FP32 (mixed precision)
    long fp64_columns = 0;        // mixed: columns finished by the FP64 recurrence
    long fp64_iters = 0;          // mixed: iterations of that FP64 completion
    long band_factorisations = 0; // banded L D L^T of shifted systems
    long band_panel_steps = 0;
    long band_solves = 0;         // columns solved with the band factors
    long band_refinements = 0;    // iterative-refinement sweeps
    long band_pivot_flags = 0;    // systems with a zero or non-finite pivot
    long band_unconverged = 0;    // passes whose band residual stayed above solve_tol
    double band_relres_max = 0.0; // largest ||b - K x|| / ||b|| after refinement
    double band_panel_flops = 0.0, band_next_flops = 0.0, band_update_flops = 0.0, band_solve_flops = 0.0;
    double band_wide_flops = 0.0;   // whole wide-band factorisations (panels, strips and windows)
};

static void choose_nrb(int64_t n, int n_active, int nrb_max, int& nrb) {
    (void)n;
    int v = (4096 + n_active - 1) / std::max(1, n_active);
    v = std::max(1, std::min(v, nrb_max));
    nrb = v;
}

class Solver {
   public:
    Solver(gep_pencil* P, const SolveCfg& c) : P_(P), c_(c), dv_(group_view(P->d, c.o.row_group)) {
        s_ = (hipStream_t)c.o.stream;
        if (!s_) {
            // the legacy default stream cannot be captured into a graph: work on
            // a private blocking stream, which orders itself with the default one
            HIPCHK(hipStreamCreate(&own_));
            s_ = own_;
        }
        tm_.on = c.o.timing != 0;
        tm_.s = s_;
        // thousands of short factorisation launches: time one in 16 (the
        // event pairs would otherwise add to the gaps between launches)
        tm_.stride[T_BAND_PANEL] = tm_.stride[T_BAND_NEXT] = tm_.stride[T_BAND_UPDATE] = 16;
        if (!P_->counts_h) HIPCHK(hipHostMalloc((void**)&P_->counts_h, sizeof(int32_t) * 4, 0));
        counts_h_ = P_->counts_h;
    }
    ~Solver() {
        if (s2_) (void)hipStreamSynchronize(s2_);
        if (own_) {
            (void)hipStreamSynchronize(own_);
            (void)hipStreamDestroy(own_);
        }
    }

    // Shifted solves of a pass by banded L D L^T (band.hip, band_wide.hip)?
    // solver: 0 = automatic (every pencil of the pass has half bandwidth
    // <= kBandMaxBw), 1 = COCG, 2 = band (error if a pencil's band is wider).
    bool use_band(const std::vector<Job>& jobs) const {
        const int mode = c_.o.solver;
        if (mode == 1 || mode == 3) return false;
        for (const Job& j : jobs) {
            const int p = j.prob;
            if (P_->h.prob_bw[p] > kBandMaxBw) {
                if (mode == 2)
                    fail(GEP_EINVAL, "band solver: half bandwidth " + std::to_string(P_->h.prob_bw[p]) +
                                         " of problem " + std::to_string(p) + " exceeds " +
                                         std::to_string(kBandMaxBw));
                return false;
            }
        }
        return true;
    }

    // The wide-band kernels factor the pass's systems when the factors are
    // FP32 (mixed precision), when the caller asks for them (band_kernels =
    // 2), when a band is not kept packed (wider than kBandWideBw), and, by
    // default, when a panel no longer fits one thread per row of one
    // work-group (kPanel + bw > 512): beyond that the one-work-group panels
    // keep the panel in global memory and take over ten times as long per
    // step as the wide-band kernels' multi-work-group panels.  band_kernels
    // = 1 keeps the one-work-group kernels for every kept band.
    bool use_wide(const std::vector<Job>& jobs) const {
        if (c_.o.precision == GEP_MIXED || c_.o.band_kernels == 2) return true;
        for (const Job& j : jobs) {
            if (P_->h.prob_boff[j.prob] < 0) return true;
            if (c_.o.band_kernels == 0 && kPanel + P_->h.prob_bw[j.prob] > 512) return true;
        }
        return false;
    }

    // Solutions of every (job, node, rhs) column by banded L D L^T: X (tiled)
    // = (z B - A)^-1 b.  The factors of a pass are kept for the next pass of
    // the same solve when its contours and nodes are the same (the
    // refinement pass).
    void band_pass(const std::vector<Job>& jobs, CocgState& S, const double* BV, int64_t ldbv,
                   int L, const std::vector<int64_t>& coff, const std::vector<double2>& shifts,
                   int64_t nmax, int64_t elems, double2* X) {
        if (use_wide(jobs)) {
            band_pass_wide(jobs, S, BV, ldbv, L, coff, shifts, nmax, elems, X);
            return;
        }
        const int K = (int)jobs.size();
        const int NH = c_.NH;
        const int nsys = K * NH;
        const int ntiles = S.ntiles;
        const int64_t Wp = (int64_t)ntiles * kTile;
        std::vector<BandSys> sys(nsys);
        std::vector<double> keys;
        int64_t total = 0;
        int bwmax = 0;
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < NH; ++j) {
                BandSys& b = sys[(size_t)k * NH + j];
                const int p = jobs[k].prob;
                b.off = total;
                b.aoff = P_->h.prob_boff[p];
                b.n = (int32_t)jobs[k].n;
                b.bw = P_->h.prob_bw[p];
                b.z = shifts[coff[k] + (int64_t)j * L];
                total += (int64_t)b.n * (b.bw + 1);
                bwmax = std::max(bwmax, b.bw);
                keys.insert(keys.end(), {(double)p, b.z.x, b.z.y});
            }
        std::vector<int32_t> colsys(Wp, -1);
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < NH; ++j)
                for (int l = 0; l < L; ++l) colsys[coff[k] + (int64_t)j * L + l] = k * NH + j;
        DBuf<BandSys> dsys(nsys);
        DBuf<int32_t> dcol(Wp);
        HIPCHK(hipMemcpyAsync(dsys.get(), sys.data(), sizeof(BandSys) * nsys, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(dcol.get(), colsys.data(), sizeof(int32_t) * Wp, hipMemcpyHostToDevice, s_));
        if (!band_F_ || keys != band_keys_) {
            band_F_.reset();
            try {
                band_F_ = std::make_unique<DBuf<double2>>(total);
            } catch (const Fail& f) {
                // the wave's factors do not fit beside the rest of the pass:
                // the wide-band path factors the systems in groups that do
                if (f.code != GEP_ENOMEM) throw;
                band_keys_.clear();
                band_pass_wide(jobs, S, BV, ldbv, L, coff, shifts, nmax, elems, X);
                return;
            }
            DBuf<int32_t> flags(nsys);
            HIPCHK(hipMemsetAsync(flags.get(), 0, sizeof(int32_t) * nsys, s_));
            HIPCHK(band_form(dsys.get(), nsys, dv_.band, band_F_->get(), s_));
            // Lookahead over two panel steps.  Step k updates, on s_, the next
            // panel's columns with panels k - 1 and k (they gate panel k + 1),
            // then, on s2, the window from panel k + 3 on with panel k, beside
            // the next two panel steps.  The rest of step k writes the columns
            // of panel k + 3, so the strip update of step k + 2 waits for it;
            // concurrent launches touch disjoint columns.
            if (!P_->aux) HIPCHK(hipStreamCreateWithFlags(&P_->aux, hipStreamNonBlocking));
            if (!P_->ev_panel) HIPCHK(hipEventCreateWithFlags(&P_->ev_panel, hipEventDisableTiming));
            for (hipEvent_t& e : P_->ev_rest)
                if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            s2_ = P_->aux;
            hipEvent_t ev_panel_ = P_->ev_panel;
            hipEvent_t* ev_rest_ = P_->ev_rest;
            // direct: the cross-stream events ride on the dispatches (no marker
            // packet of their own unless the timer holds that launch); graph
            // capture: plain launches and event records, which the capture
            // turns into the graph's dependencies
            auto enqueue = [&](bool direct) -> int {
                int steps = 0;
                for (int64_t k0 = 0; k0 < nmax; k0 += kPanel, ++steps) {
                    hipEvent_t ea = nullptr, eb = nullptr;
                    if (direct) tm_.kernel_pair(T_BAND_PANEL, ea, eb);
                    HIPCHK(band_panel(dsys.get(), nsys, bwmax, band_F_->get(), (int)k0, flags.get(), s_, ea, eb));
                    if (k0 + kPanel >= nmax) continue;
                    if (steps >= 2) HIPCHK(hipStreamWaitEvent(s_, ev_rest_[steps & 1], 0));
                    if (direct) tm_.kernel_pair(T_BAND_NEXT, ea, eb);
                    HIPCHK(band_update(dsys.get(), nsys, bwmax, band_F_->get(), (int)k0, 1, s_, ea,
                                       direct && !eb ? ev_panel_ : eb));
                    if (!direct || eb) HIPCHK(hipEventRecord(ev_panel_, s_));
                    HIPCHK(hipStreamWaitEvent(s2_, ev_panel_, 0));
                    if (direct) tm_.kernel_pair(T_BAND_UPDATE, ea, eb);
                    HIPCHK(band_update(dsys.get(), nsys, bwmax, band_F_->get(), (int)k0, 2, s2_, ea,
                                       direct && !eb ? ev_rest_[steps & 1] : eb));
                    if (!direct || eb) HIPCHK(hipEventRecord(ev_rest_[steps & 1], s2_));
                }
                if (steps >= 2) {   // s_ joins s2 (the last window update)
                    HIPCHK(hipEventRecord(ev_panel_, s2_));
                    HIPCHK(hipStreamWaitEvent(s_, ev_panel_, 0));
                }
                return steps;
            };
            int steps = 0;
            if (c_.o.use_graph >= 2 && !tm_.on) {
                // The factorisation's launches replayed as one HIP graph,
                // captured once per pencil and layout (the buffers and sizes its
                // launches name) and kept with the pencil.  Opt-in: on MI355X
                // the graph's cross-queue edges cost more than the direct
                // launches' events (85.8 against 62.0 us per panel step on the
                // 2D Q1 pencil of half bandwidth 301, 64 systems).
                const std::vector<int64_t> gkey = {(int64_t)(intptr_t)band_F_->get(), (int64_t)(intptr_t)dsys.get(),
                                                   (int64_t)(intptr_t)flags.get(), nsys, bwmax, nmax};
                if (!P_->band_graph || gkey != P_->band_graph_key) {
                    if (P_->band_graph) {
                        HIPCHK(hipGraphExecDestroy(P_->band_graph));
                        P_->band_graph = nullptr;
                    }
                    hipGraph_t graph = nullptr;
                    HIPCHK(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
                    try {
                        steps = enqueue(false);
                    } catch (...) {   // leave capture mode before the error propagates
                        if (hipStreamEndCapture(s_, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
                        (void)hipGetLastError();
                        throw;
                    }
                    HIPCHK(hipStreamEndCapture(s_, &graph));
                    hipError_t e = hipGraphInstantiate(&P_->band_graph, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    if (e != hipSuccess) P_->band_graph = nullptr;
                    HIPCHK(e);
                    P_->band_graph_key = gkey;
                    P_->band_graph_steps = steps;
                    stats_.graph_captures += 1;
                }
                steps = P_->band_graph_steps;
                HIPCHK(hipGraphLaunch(P_->band_graph, s_));
            } else {
                steps = enqueue(true);
            }
            for (int k = 0; k < K; ++k) {
                double fp, fn, fr;
                band_factor_flops(jobs[k].n, P_->h.prob_bw[jobs[k].prob], fp, fn, fr);
                stats_.band_panel_flops += NH * fp;
                stats_.band_next_flops += NH * fn;
                stats_.band_update_flops += NH * fr;
            }
            std::vector<int32_t> fh(nsys);
            HIPCHK(hipMemcpyAsync(fh.data(), flags.get(), sizeof(int32_t) * nsys, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            tm_.flush();
            for (int32_t v : fh) stats_.band_pivot_flags += v != 0;
            stats_.band_factorisations += nsys;
            stats_.band_panel_steps += steps;
            band_keys_ = keys;
        }
        for (int k = 0; k < K; ++k)
            stats_.band_solve_flops +=
                (double)NH * L * band_solve_flops(jobs[k].n, P_->h.prob_bw[jobs[k].prob]);
        tm_.begin(T_BAND_SOLVE);
        HIPCHK(band_rhs(S.geom, S.bsrc, BV, ldbv, ntiles, X, s_));
        // chunks of 16 (or 8) columns belong to one system when L is a multiple
        const int chunk = L % 16 == 0 ? 16 : (L % 8 == 0 ? 8 : 0);
        HIPCHK(band_solve(dsys.get(), dcol.get(), band_F_->get(), S.geom, ntiles, bwmax, X, s_, chunk));
        tm_.end();
        // FP64 residual of every column, iterative refinement with the factors.
        // The first check forms only the norms; the residual itself is
        // written (and its buffer allocated) once a column needs refinement.
        constexpr int kCap = 1024;   // row blocks of the residual norms per tile
        DBuf<double2> R;
        DBuf<double2> part((size_t)ntiles * kCap * kTile);
        DBuf<double> rel(Wp);
        std::vector<double> relh(Wp);
        for (int ref = 0;; ++ref) {
            HIPCHK(band_residual(dv_, S.geom, S.shifts, S.bsrc, BV, ldbv, X, R.get(), ntiles, nmax,
                                 part.get(), kCap, rel.get(), s_));
            HIPCHK(hipMemcpyAsync(relh.data(), rel.get(), sizeof(double) * Wp, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            tm_.flush();
            double mx = 0.0;
            for (int64_t c = 0; c < Wp; ++c)
                if (colsys[c] >= 0) mx = std::max(mx, std::isfinite(relh[c]) ? relh[c] : INFINITY);
            if (mx <= c_.o.solve_tol || ref == kBandRefineMax) {
                // the largest relative residual after refinement
                stats_.band_relres_max = std::max(stats_.band_relres_max, mx);
                if (mx > c_.o.solve_tol) stats_.band_unconverged += 1;
                break;
            }
            if (!R.get()) {   // norms only so far: form the residual to solve against
                R.alloc((size_t)std::max<int64_t>(elems, 1));
                HIPCHK(band_residual(dv_, S.geom, S.shifts, S.bsrc, BV, ldbv, X, R.get(), ntiles, nmax,
                                     part.get(), kCap, rel.get(), s_));
            }
            tm_.begin(T_BAND_SOLVE);
            HIPCHK(band_solve(dsys.get(), dcol.get(), band_F_->get(), S.geom, ntiles, bwmax, R.get(), s_,
                              chunk));
            HIPCHK(band_axpy(S.geom, R.get(), ntiles, X, s_));
            for (int k = 0; k < K; ++k)
                stats_.band_solve_flops +=
                    (double)NH * L * band_solve_flops(jobs[k].n, P_->h.prob_bw[jobs[k].prob]);
            tm_.end();
            stats_.band_refinements += 1;
        }
        stats_.band_solves += Wp;
    }

    // Wide-band / FP32 pass (band_wide.hip).  The systems are factored in
    // groups that fit the device memory left after the pass's multivectors
    // (all at once when they fit, and then the factors are kept for a
    // refinement pass of the same systems); each group's columns are solved
    // and refined against the FP64 residual while its factors are held.
    // FP32 factors (mixed precision): the right-hand sides and each residual
    // are rounded to FP32 for the sweeps, the corrections accumulate in the
    // FP64 solution.
    void band_pass_wide(const std::vector<Job>& jobs, CocgState& S, const double* BV, int64_t ldbv,
                        int L, const std::vector<int64_t>& coff, const std::vector<double2>& shifts,
                        int64_t nmax, int64_t elems, double2* X) {
        const bool fp32 = c_.o.precision == GEP_MIXED;
        const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
        const int K = (int)jobs.size();
        const int NH = c_.NH;
        const int nsys = K * NH;
        const int ntiles = S.ntiles;
        const int64_t Wp = (int64_t)ntiles * kTile;
        if (fp32) stats_.fp32_passes += 1;
        std::vector<BandSys> sys(nsys);
        std::vector<std::vector<WbChunk>> chunks(nsys);
        std::vector<std::vector<int64_t>> cols(nsys);
        std::vector<double> keys;
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < NH; ++j) {
                const int q = k * NH + j;
                BandSys& b = sys[q];
                const int p = jobs[k].prob;
                b.aoff = -1;
                b.n = (int32_t)jobs[k].n;
                b.bw = P_->h.prob_bw[p];
                b.z = shifts[coff[k] + (int64_t)j * L];
                b.row0 = (int32_t)jobs[k].row0;
                keys.insert(keys.end(), {(double)p, b.z.x, b.z.y, fp32 ? 1.0 : 0.0});
                for (int l = 0; l < L;) {
                    const int64_t c = coff[k] + (int64_t)j * L + l;
                    const int cnt = std::min<int>(16, std::min<int64_t>(L - l, kTile - c % kTile));
                    chunks[q].push_back({q, (int32_t)(c / kTile), (int32_t)(c % kTile), cnt});
                    for (int u = 0; u < cnt; ++u) cols[q].push_back(c + u);
                    l += cnt;
                }
            }
        HIPCHK(band_rhs(S.geom, S.bsrc, BV, ldbv, ntiles, X, s_));
        const int refine_max = fp32 ? kBandRefineMax32 : kBandRefineMax;
        constexpr int kCap = 1024;   // row blocks of the residual norms per tile
        DBuf<double2> R((size_t)std::max<int64_t>(elems, 1));
        DBuf<double2> part((size_t)ntiles * kCap * kTile);
        DBuf<double> rel(Wp);
        DBuf<float2> X32;
        if (fp32) X32.alloc((size_t)std::max<int64_t>(elems, 1));
        std::vector<double> relh(Wp);
        // systems per group: what the device can hold now
        size_t per = 0;
        for (const BandSys& b : sys) per = std::max(per, (size_t)b.n * (size_t)(b.bw + 1) * esz);
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        const bool keep = band_wF_ && keys == band_keys_;
        // the factors of a group are one buffer: the largest free range of
        // the workspace, or a new chunk from the device's free memory
        double avail = std::max(0.98 * (double)P_->pool.largest_free(), 0.92 * (double)freeb) +
                       (keep ? (double)band_wF_->n * sizeof(double2) : 0.0);
        // a caller's memory budget caps the factors held at once
        if (c_.o.mem_limit_bytes > 0) avail = std::min(avail, c_.o.mem_limit_bytes);
        int G = (int)std::min<double>(nsys, std::floor(avail / (double)std::max<size_t>(per, 1)));
        if (c_.o.band_group > 0) G = std::min(G, c_.o.band_group);
        if (G < 1) fail(GEP_ENOMEM, "one banded factor needs " + std::to_string(per) + " bytes of device memory");
        if (G < nsys) {
            band_wF_.reset();
            band_keys_.clear();
        }
        DBuf<int32_t> flags(nsys);
        HIPCHK(hipMemsetAsync(flags.get(), 0, sizeof(int32_t) * nsys, s_));
        for (int g0 = 0; g0 < nsys; g0 += G) {
            const int g1 = std::min(nsys, g0 + G), ng = g1 - g0;
            std::vector<BandSys> gs(sys.begin() + g0, sys.begin() + g1);
            std::vector<WbChunk> gc;
            int64_t total = 0, gmax = 0;
            int bwmax = 0;
            for (int q = 0; q < ng; ++q) {
                gs[q].off = total;
                total += (int64_t)gs[q].n * (gs[q].bw + 1);
                gmax = std::max<int64_t>(gmax, gs[q].n);
                bwmax = std::max(bwmax, gs[q].bw);
                for (WbChunk c : chunks[g0 + q]) {
                    c.sys = q;
                    gc.push_back(c);
                }
            }
            const size_t fbytes = (size_t)total * esz;
            DBuf<BandSys> dsys(ng);
            DBuf<WbChunk> dch(gc.size());
            HIPCHK(hipMemcpyAsync(dsys.get(), gs.data(), sizeof(BandSys) * ng, hipMemcpyHostToDevice, s_));
            HIPCHK(hipMemcpyAsync(dch.get(), gc.data(), sizeof(WbChunk) * gc.size(), hipMemcpyHostToDevice, s_));
            const int nch = (int)gc.size();
            DBuf<double2> Dfar((wb_scratch_bytes(nch) + sizeof(double2) - 1) / sizeof(double2));
            std::unique_ptr<DBuf<double2>> Fown;
            DBuf<double2>* F = nullptr;
            if (ng == nsys && keep) {
                F = band_wF_.get();
            } else {
                Fown = std::make_unique<DBuf<double2>>((fbytes + sizeof(double2) - 1) / sizeof(double2));
                F = Fown.get();
                HIPCHK(hipMemsetAsync(F->get(), 0, fbytes, s_));
                HIPCHK(wb_form(P_->d, dsys.get(), ng, F->get(), fp32, s_));
                int steps = 0;
                tm_.begin(T_BAND_WIDE);
                for (int64_t k0 = 0; k0 < gmax; k0 += 2 * kPanel, steps += 2)
                    HIPCHK(wb_step(dsys.get(), ng, bwmax, F->get(), fp32, (int)k0, (int)gmax, flags.get() + g0, s_));
                tm_.end();
                for (int q = g0; q < g1; ++q) {
                    double fp, fn, fr;
                    band_factor_flops(sys[q].n, sys[q].bw, fp, fn, fr);
                    stats_.band_wide_flops += fp + fn + fr;
                }
                stats_.band_factorisations += ng;
                stats_.band_panel_steps += steps;
            }
            auto sweep_flops = [&]() {
                for (int q = g0; q < g1; ++q)
                    stats_.band_solve_flops += (double)cols[q].size() * band_solve_flops(sys[q].n, sys[q].bw);
            };
            tm_.begin(T_BAND_SOLVE);
            if (fp32) {
                HIPCHK(wb_narrow(dsys.get(), dch.get(), nch, S.geom, X, X32.get(), s_));
                HIPCHK(wb_solve(dsys.get(), dch.get(), nch, F->get(), true, S.geom, X32.get(), (int)gmax, Dfar.get(), s_));
                HIPCHK(wb_accumulate(dsys.get(), dch.get(), nch, S.geom, X32.get(), true, X, 1, s_));
            } else {
                HIPCHK(wb_solve(dsys.get(), dch.get(), nch, F->get(), false, S.geom, X, (int)gmax, Dfar.get(), s_));
            }
            tm_.end();
            sweep_flops();
            for (int ref = 0;; ++ref) {
                HIPCHK(band_residual(dv_, S.geom, S.shifts, S.bsrc, BV, ldbv, X, R.get(), ntiles, nmax,
                                     part.get(), kCap, rel.get(), s_));
                HIPCHK(hipMemcpyAsync(relh.data(), rel.get(), sizeof(double) * Wp, hipMemcpyDeviceToHost, s_));
                HIPCHK(hipStreamSynchronize(s_));
                tm_.flush();
                double mx = 0.0;
                for (int q = g0; q < g1; ++q)
                    for (int64_t c : cols[q]) mx = std::max(mx, std::isfinite(relh[c]) ? relh[c] : INFINITY);
                if (mx <= c_.o.solve_tol || ref == refine_max) {
                    // the largest relative residual after refinement
                    stats_.band_relres_max = std::max(stats_.band_relres_max, mx);
                    if (mx > c_.o.solve_tol) stats_.band_unconverged += 1;
                    break;
                }
                tm_.begin(T_BAND_SOLVE);
                if (fp32) {
                    HIPCHK(wb_narrow(dsys.get(), dch.get(), nch, S.geom, R.get(), X32.get(), s_));
                    HIPCHK(wb_solve(dsys.get(), dch.get(), nch, F->get(), true, S.geom, X32.get(), (int)gmax, Dfar.get(), s_));
                    HIPCHK(wb_accumulate(dsys.get(), dch.get(), nch, S.geom, X32.get(), true, X, 0, s_));
                } else {
                    HIPCHK(wb_solve(dsys.get(), dch.get(), nch, F->get(), false, S.geom, R.get(), (int)gmax, Dfar.get(), s_));
                    HIPCHK(wb_accumulate(dsys.get(), dch.get(), nch, S.geom, R.get(), false, X, 0, s_));
                }
                tm_.end();
                sweep_flops();
                stats_.band_refinements += 1;
            }
            if (ng == nsys && !keep) {
                band_wF_ = std::move(Fown);
                band_keys_ = keys;
            }
        }
        std::vector<int32_t> fh(nsys);
        HIPCHK(hipMemcpyAsync(fh.data(), flags.get(), sizeof(int32_t) * nsys, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        for (int32_t v : fh) stats_.band_pivot_flags += v != 0;
        stats_.band_solves += Wp;
    }

    // One pass of the pipeline for a set of jobs sharing (L, M).  Job k's
    // right-hand side l is the column of B V starting at offset
    // jobs[k].bsrc0 + l, rows of its pencil at stride ldbv.
    // Shifted solves by multi-shift COCG (solver = 3, multishift.hip): one
    // pencil whose B is beta I.  The nodes of one contour are shifts of one
    // another and share a Krylov space per right-hand side: each contour's
    // block column l is a seed column, iterated on the system of the
    // contour's node nearest the real axis (the slowest to converge); every
    // (node, l) column keeps scalar recurrences (on the host, from two small
    // reads per iteration) and its own solution and search vector (updated
    // on the device).  A column stops once ||r|| / |pi_c| <= solve_tol ||b||.
    void ms_pass(const std::vector<Job>& jobs, CocgState& S, const double* BV, int64_t ldbv, int L,
                 const std::vector<int64_t>& coff, const std::vector<double2>& shifts, int64_t Wp, size_t mv,
                 double2* X) {
        const int K = (int)jobs.size();
        const int NH = c_.NH;
        const HostPencil& H = P_->h;
        if (H.prob_n.size() != 1) fail(GEP_EINVAL, "multi-shift COCG: single pencils only (no batches)");
        const int64_t n = H.n;
        double bB = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int32_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) {
                const double v = H.b[e];
                if (H.colind[e] != i) {
                    if (v != 0.0) fail(GEP_EINVAL, "multi-shift COCG needs B = beta I (B has off-diagonal entries)");
                } else if (i == 0) {
                    bB = v;
                } else if (std::abs(v - bB) > 1e-14 * std::abs(bB)) {
                    fail(GEP_EINVAL, "multi-shift COCG needs B = beta I (B's diagonal is not constant)");
                }
            }
        if (!(bB != 0.0)) fail(GEP_EINVAL, "multi-shift COCG needs B = beta I with beta != 0");
        // seed columns s = k L + l with the shift of contour k's node nearest
        // the real axis; shifted column c -> seed column col_l[c], delta_c
        const int ntiles = S.ntiles;
        const int nseed = K * L, st = (nseed + kTile - 1) / kTile, ws = st * kTile;
        std::vector<int32_t> col_l(Wp, -1);
        std::vector<std::complex<double>> delta(Wp, 0.0);
        std::vector<double2> zseed(ws, make_double2(0.0, 0.0));
        std::vector<int64_t> bs(ws, -1);
        for (int k = 0; k < K; ++k) {
            int js = 0;
            for (int j = 1; j < NH; ++j)
                if (std::abs(shifts[coff[k] + (int64_t)j * L].y) < std::abs(shifts[coff[k] + (int64_t)js * L].y)) js = j;
            const double2 z0 = shifts[coff[k] + (int64_t)js * L];
            for (int l = 0; l < L; ++l) {
                zseed[k * L + l] = z0;
                bs[k * L + l] = jobs[k].bsrc0 + l;
            }
            for (int j = 0; j < NH; ++j)
                for (int l = 0; l < L; ++l) {
                    const int64_t c = coff[k] + (int64_t)j * L + l;
                    col_l[c] = k * L + l;
                    delta[c] = bB * std::complex<double>(shifts[c].x - z0.x, shifts[c].y - z0.y);
                }
        }
        std::vector<std::complex<double>> pi(Wp, 1.0), pip(Wp, 1.0);
        std::vector<int32_t> act(Wp, 0);
        int64_t n_act = 0;
        for (int64_t c = 0; c < Wp; ++c) n_act += (act[c] = col_l[c] >= 0);
        // seed geometry: tile t at t n 64
        std::vector<int64_t> sbase(st);
        std::vector<int32_t> sn(st, (int32_t)n), stile(st);
        for (int t = 0; t < st; ++t) {
            sbase[t] = (int64_t)t * n * kTile;
            stile[t] = t;
        }
        const size_t sv = (size_t)n * ws;
        DBuf<double2> r(sv), ps(sv), q(sv), P(mv);
        DBuf<double2> d_zs(ws), d_alpha(ws), d_beta(ws), d_coef((size_t)3 * Wp);
        DBuf<int32_t> d_col(Wp), d_act(Wp), d_stile(st), d_cnt(1), d_sn(st);
        DBuf<int64_t> d_sbase(st), d_bs(ws);
        int nrb = 0;
        choose_nrb(n, st, (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 31) / 32)), nrb);
        DBuf<double2> part_mu((size_t)st * nrb * kTile), part_rho((size_t)st * nrb * kTile);
        DBuf<double> part_nrm((size_t)st * nrb * kTile);
        const int32_t st32 = st;
        HIPCHK(hipMemcpyAsync(d_zs.get(), zseed.data(), sizeof(double2) * ws, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_col.get(), col_l.data(), sizeof(int32_t) * Wp, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_sbase.get(), sbase.data(), sizeof(int64_t) * st, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_sn.get(), sn.data(), sizeof(int32_t) * st, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_stile.get(), stile.data(), sizeof(int32_t) * st, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_cnt.get(), &st32, sizeof(int32_t), hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_bs.get(), bs.data(), sizeof(int64_t) * ws, hipMemcpyHostToDevice, s_));
        TileGeom gs;
        gs.base = d_sbase.get();
        gs.n = d_sn.get();
        // x = 0, every shifted p = b, seed r = p_s = b, q = 0
        HIPCHK(hipMemsetAsync(X, 0, sizeof(double2) * mv, s_));
        HIPCHK(band_rhs(S.geom, S.bsrc, BV, ldbv, ntiles, P.get(), s_));
        HIPCHK(band_rhs(gs, d_bs.get(), BV, ldbv, st, r.get(), s_));
        HIPCHK(hipMemcpyAsync(ps.get(), r.get(), sizeof(double2) * sv, hipMemcpyDeviceToDevice, s_));
        HIPCHK(hipMemsetAsync(q.get(), 0, sizeof(double2) * sv, s_));
        HIPCHK(hipMemsetAsync(d_alpha.get(), 0, sizeof(double2) * ws, s_));
        const size_t np = (size_t)st * nrb * kTile;
        std::vector<double2> hpart(np);
        std::vector<double> hnrm(np);
        // column sums over the row blocks of [tile][nrb][64] partials
        auto col_sum = [&](const std::vector<double2>& pp, int s_col) {
            const int t = s_col / kTile, l = s_col % kTile;
            std::complex<double> a = 0.0;
            for (int rb = 0; rb < nrb; ++rb) {
                const double2 v = pp[((size_t)t * nrb + rb) * kTile + l];
                a += std::complex<double>(v.x, v.y);
            }
            return a;
        };
        std::vector<std::complex<double>> rho(ws), rho_n(ws), alpha(ws, 0.0), beta(ws, 0.0), alpha_prev(ws, 1.0),
            beta_prev(ws, 0.0);
        std::vector<double> nrm(ws), bnorm(ws);
        auto seed_sums = [&]() {
            HIPCHK(hipMemcpyAsync(hpart.data(), part_rho.get(), sizeof(double2) * np, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipMemcpyAsync(hnrm.data(), part_nrm.get(), sizeof(double) * np, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            for (int sc = 0; sc < ws; ++sc) {
                rho_n[sc] = col_sum(hpart, sc);
                double b = 0.0;
                for (int rb = 0; rb < nrb; ++rb) b += hnrm[((size_t)(sc / kTile) * nrb + rb) * kTile + sc % kTile];
                nrm[sc] = b;
            }
        };
        HIPCHK(ms_seed_update((int)n, st, nrb, d_alpha.get(), q.get(), r.get(), part_rho.get(), part_nrm.get(), s_));
        seed_sums();
        for (int sc = 0; sc < ws; ++sc) {
            rho[sc] = rho_n[sc];
            bnorm[sc] = std::sqrt(nrm[sc]);
        }
        const double tol = c_.o.solve_tol;
        std::vector<double2> coef((size_t)3 * Wp, make_double2(0.0, 0.0)), h_ab(ws);
        long it = 0;
        while (n_act > 0 && it < c_.o.max_iter) {
            // q = K_s p_s with the column partials of p_s^T q
            tm_.begin(T_SPMM);
            HIPCHK(launch_spmm_c64(P_->d, d_zs.get(), ps.get(), q.get(), d_stile.get(), d_cnt.get(), st, nrb,
                                   part_mu.get(), s_));
            tm_.end();
            HIPCHK(hipMemcpyAsync(hpart.data(), part_mu.get(), sizeof(double2) * np, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            for (int sc = 0; sc < ws; ++sc) {
                const std::complex<double> mu = col_sum(hpart, sc);
                alpha[sc] = (sc < nseed && std::abs(mu) > 0.0) ? rho[sc] / mu : 0.0;
                h_ab[sc] = make_double2(alpha[sc].real(), alpha[sc].imag());
            }
            HIPCHK(hipMemcpyAsync(d_alpha.get(), h_ab.data(), sizeof(double2) * ws, hipMemcpyHostToDevice, s_));
            HIPCHK(ms_seed_update((int)n, st, nrb, d_alpha.get(), q.get(), r.get(), part_rho.get(), part_nrm.get(),
                                  s_));
            seed_sums();
            for (int sc = 0; sc < ws; ++sc)
                beta[sc] = (sc < nseed && std::abs(rho[sc]) > 0.0) ? rho_n[sc] / rho[sc] : 0.0;
            // shifted scalars: pi_{k+1} = (1 + a b'/a' + a delta) pi_k - (a b'/a') pi_{k-1},
            // alpha_c = a pi_k / pi_{k+1}, beta_c = (pi_k / pi_{k+1})^2 b
            std::vector<int32_t> done;
            for (int64_t c = 0; c < Wp; ++c) {
                if (!act[c]) continue;
                const int sc = col_l[c];
                const std::complex<double> a = alpha[sc];
                const std::complex<double> g =
                    (it > 0 && std::abs(alpha_prev[sc]) > 0.0) ? a * beta_prev[sc] / alpha_prev[sc] : 0.0;
                const std::complex<double> pn = (1.0 + g + a * delta[c]) * pi[c] - g * pip[c];
                const std::complex<double> rat = pi[c] / pn;
                const std::complex<double> ac = a * rat, bc = rat * rat * beta[sc], ip = 1.0 / pn;
                coef[3 * c] = make_double2(ac.real(), ac.imag());
                coef[3 * c + 1] = make_double2(bc.real(), bc.imag());
                coef[3 * c + 2] = make_double2(ip.real(), ip.imag());
                pip[c] = pi[c];
                pi[c] = pn;
                if (std::sqrt(nrm[sc]) <= tol * bnorm[sc] * std::abs(pn) || !std::isfinite(std::abs(pn)))
                    done.push_back((int32_t)c);
            }
            HIPCHK(hipMemcpyAsync(d_coef.get(), coef.data(), sizeof(double2) * coef.size(), hipMemcpyHostToDevice, s_));
            HIPCHK(hipMemcpyAsync(d_act.get(), act.data(), sizeof(int32_t) * Wp, hipMemcpyHostToDevice, s_));
            tm_.begin(T_UPDATE);
            HIPCHK(ms_shift_update(S.geom, ntiles, n, (int)n, d_col.get(), d_act.get(), d_coef.get(), r.get(), X,
                                   P.get(), s_));
            tm_.end();
            for (int sc = 0; sc < ws; ++sc) h_ab[sc] = make_double2(beta[sc].real(), beta[sc].imag());
            HIPCHK(hipMemcpyAsync(d_beta.get(), h_ab.data(), sizeof(double2) * ws, hipMemcpyHostToDevice, s_));
            HIPCHK(ms_seed_p((int)n, st, d_beta.get(), r.get(), ps.get(), s_));
            // host buffers read by the copies above must not change before they ran
            HIPCHK(hipStreamSynchronize(s_));
            tm_.flush();
            for (int32_t c : done) {
                act[c] = 0;
                --n_act;
            }
            for (int sc = 0; sc < ws; ++sc) {
                alpha_prev[sc] = alpha[sc];
                beta_prev[sc] = beta[sc];
                rho[sc] = rho_n[sc];
            }
            ++it;
            if (c_.o.verbose > 0 && it % c_.o.verbose == 0) {
                std::fprintf(stderr, "gep: multi-shift pass, iteration %ld, active columns %lld\n", it,
                             (long long)n_act);
                std::fflush(stderr);
            }
        }
        HIPCHK(hipStreamSynchronize(s_));
        stats_.ms_iters += it;
        stats_.ms_unconverged += n_act;
    }

    void run_pass(const std::vector<Job>& jobs, const double* BV, int64_t ldbv, int L, int M,
                  std::vector<ContourOut>& out) {
        const int K = (int)jobs.size();
        const int NH = c_.NH;
        const int64_t per = (int64_t)NH * L;                     // columns per job
        const int tper = (int)((per + kTile - 1) / kTile);       // tiles per job
        const int ntiles = K * tper;
        const int64_t Wp = (int64_t)ntiles * kTile;
        stats_.columns += per * K;
        // tile geometry and per-column metadata
        std::vector<int64_t> tbase(ntiles);
        std::vector<int32_t> tn(ntiles), trow0(ntiles), tg0(ntiles);
        int64_t elems = 0, nmax = 0;
        for (int k = 0; k < K; ++k) {
            nmax = std::max(nmax, jobs[k].n);
            for (int t = 0; t < tper; ++t) {
                const int tt = k * tper + t;
                tbase[tt] = elems;
                tn[tt] = (int32_t)jobs[k].n;
                trow0[tt] = (int32_t)jobs[k].row0;
                tg0[tt] = dv_.grp == 4 ? P_->h.prob_g4[jobs[k].prob] : (int32_t)jobs[k].row0;
                elems += jobs[k].n * kTile;
            }
        }
        std::vector<double2> shifts(Wp, make_double2(0.0, 1.0));
        std::vector<int64_t> bsrc(Wp, -1);
        std::vector<double2> coef((size_t)K * NH * M);
        std::vector<int64_t> coff(K), soff(K + 1, 0);
        std::vector<int32_t> cn(K);
        const int r0 = L * M;
        for (int k = 0; k < K; ++k) {
            const double c = jobs[k].c.center, R = jobs[k].c.radius;
            coff[k] = (int64_t)k * tper * kTile;
            cn[k] = (int32_t)jobs[k].n;
            soff[k + 1] = soff[k] + jobs[k].n * r0;
            for (int j = 0; j < NH; ++j) {
                const double th = M_PI * (2.0 * (j + 1) - 1.0) / c_.N;
                const std::complex<double> zeta(std::cos(th), std::sin(th));
                const std::complex<double> z = c + R * zeta;
                const std::complex<double> w = R * zeta / (double)c_.N;
                std::complex<double> zm(1.0, 0.0);
                for (int m = 0; m < M; ++m) {
                    const std::complex<double> cf = 2.0 * w * zm;
                    coef[((size_t)k * NH + j) * M + m] = make_double2(cf.real(), cf.imag());
                    zm *= zeta;
                }
                for (int l = 0; l < L; ++l) {
                    const int64_t col = coff[k] + (int64_t)j * L + l;
                    shifts[col] = make_double2(z.real(), z.imag());
                    bsrc[col] = jobs[k].bsrc0 + l;
                }
            }
        }
        // shifted solves: banded L D L^T (band.hip) or batched COCG
        const bool band = use_band(jobs);
        const bool ms = c_.o.solver == 3;
        CocgState S;
        S.ntiles = ntiles;
        const bool mixed = c_.o.precision == GEP_MIXED && !band && !ms;
        if (mixed) stats_.fp32_passes += 1;
        // small row blocks keep the gathers of concurrently running
        // work-groups inside the caches; one row group per wave by default,
        // and a whole number of groups per work-group
        const int grp = dv_.grp;
        S.rpb = c_.o.rows_per_block > 0 ? c_.o.rows_per_block : (grp == 4 ? 4 * kWaves : 2 * kWaves);
        S.rpb = (S.rpb + grp - 1) / grp * grp;
        S.nrb = (int)((nmax + S.rpb - 1) / S.rpb);
        S.n = nmax;
        const int nrb = S.nrb;
        const size_t mv = (size_t)elems;
        DBuf<double2> x(mv), u, p, pn;
        DBuf<float2> x32, u32, p32, pn32;
        if (band || ms) {
            // only x (the solutions); the COCG vectors are not needed
        } else if (mixed) {
            x32.alloc(mv);
            u32.alloc(mv);
            p32.alloc(mv);
            pn32.alloc(mv);
        } else {
            u.alloc(mv);
            p.alloc(mv);
            pn.alloc(mv);
        }
        DBuf<double2> d_shifts(Wp), rho(Wp), alpha(Wp), beta(Wp);
        DBuf<int64_t> d_bsrc(Wp), d_tbase(ntiles), d_coff(K), d_soff(K);
        DBuf<int32_t> active(Wp), iters(Wp), tile_active(ntiles), tiles(ntiles), counts(4);
        DBuf<int32_t> d_tn(ntiles), d_trow0(ntiles), d_tg0(ntiles), d_cn(K);
        DBuf<double> bb(Wp), rr(Wp), rmax(Wp);
        DBuf<int32_t> flag(Wp), stall(Wp), stalled(Wp);
        DBuf<double> rbest(Wp);
        DBuf<double2> part_c((size_t)ntiles * nrb * kTile);
        DBuf<double> part_r((size_t)ntiles * nrb * kTile);
        S.G = nrb > 64 ? 32 : 0;
        DBuf<double2> part2_c((size_t)ntiles * std::max(S.G, 1) * kTile);
        DBuf<double> part2_r((size_t)ntiles * std::max(S.G, 1) * kTile);
        S.part2_c = part2_c.get();
        S.part2_r = part2_r.get();
        DBuf<double2> d_coef(coef.size());
        S.x = x.get();
        S.u = u.get();
        S.p = p.get();
        S.pn = pn.get();
        S.x32 = x32.get();
        S.u32 = u32.get();
        S.p32 = p32.get();
        S.pn32 = pn32.get();
        S.shifts = d_shifts.get();
        S.bsrc = d_bsrc.get();
        S.rho = rho.get();
        S.alpha = alpha.get();
        S.beta = beta.get();
        S.bb = bb.get();
        S.rr = rr.get();
        S.rmax = rmax.get();
        S.flag = flag.get();
        S.rbest = rbest.get();
        S.stall = stall.get();
        S.stalled = stalled.get();
        S.active = active.get();
        S.iters = iters.get();
        S.tile_active = tile_active.get();
        S.tiles = tiles.get();
        S.counts = counts.get();
        S.part_c = part_c.get();
        S.part_r = part_r.get();
        S.geom.base = d_tbase.get();
        S.geom.n = d_tn.get();
        S.geom.row0 = d_trow0.get();
        S.geom.g0 = d_tg0.get();
        std::vector<int32_t> tl(ntiles);
        for (int t = 0; t < ntiles; ++t) tl[t] = t;
        int32_t cnt0[4] = {ntiles, (int32_t)(per * K), 0, 0};
        HIPCHK(hipMemcpyAsync(S.shifts, shifts.data(), sizeof(double2) * Wp, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(S.bsrc, bsrc.data(), sizeof(int64_t) * Wp, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_tbase.get(), tbase.data(), sizeof(int64_t) * ntiles, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_tn.get(), tn.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_trow0.get(), trow0.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_tg0.get(), tg0.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_coff.get(), coff.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_soff.get(), soff.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_cn.get(), cn.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(S.tiles, tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(S.counts, cnt0, sizeof(cnt0), hipMemcpyHostToDevice, s_));
        HIPCHK(hipMemcpyAsync(d_coef.get(), coef.data(), sizeof(double2) * coef.size(), hipMemcpyHostToDevice, s_));
        std::vector<int32_t> its(Wp, 0), its0(Wp, 0);
        if (band) {
            band_pass(jobs, S, BV, ldbv, L, coff, shifts, nmax, elems, x.get());
        } else if (ms) {
            ms_pass(jobs, S, BV, ldbv, L, coff, shifts, Wp, mv, x.get());
        } else {
        if (mixed) {
            HIPCHK(hipMemsetAsync(S.x, 0, sizeof(double2) * mv, s_));
            HIPCHK(cocg32_init(dv_, S, BV, ldbv, nrb, s_));
        } else {
            HIPCHK(cocg_init(dv_, S, BV, ldbv, nrb, s_));
        }
        const double tol2 = c_.o.solve_tol * c_.o.solve_tol;
        const int max_iter = c_.o.max_iter;
        int every = std::max(2, c_.o.check_every);
        every += every & 1;   // even: the p / p' buffers are back in place after a chunk
        const double cb = mixed ? 8.0 : 16.0;   // bytes per complex element of the recurrence
        int n_act = ntiles;
        long it = 0;
        // the mixed path runs the FP32 recurrence first, then finishes the
        // columns it gave up on with the FP64 recurrence
        bool fp32 = mixed;
        auto mat_bytes = [&]() { return (double)dv_.nnz * ((fp32 ? 8.0 : 16.0) + 4.0) + 4.0 * (dv_.n + 1); };
        // One chunk = `every` COCG iterations (+ the mixed path's residual
        // replacement), enqueued eagerly or replayed from a captured HIP graph.
        // The chunk's launch grids depend on the active-tile count known to the
        // host, so a graph is captured again whenever that count changes.
        auto enqueue_chunk = [&](bool timed) {
            for (int c = 0; c < every; ++c) {
                if (timed) tm_.begin(T_SPMM);
                if (fp32)
                    HIPCHK(cocg32_spmm_dir(dv_, S, n_act, nrb, s_));
                else
                    HIPCHK(cocg_spmm_dir(dv_, S, n_act, nrb, s_));
                if (timed) tm_.end();
                HIPCHK(cocg_reduce_alpha(S, n_act, nrb, s_));
                if (timed) tm_.begin(T_UPDATE);
                if (fp32)
                    HIPCHK(cocg32_update(dv_, S, n_act, nrb, s_));
                else
                    HIPCHK(cocg_update(dv_, S, n_act, nrb, s_));
                if (timed) tm_.end();
                // the FP64 completion continues the columns' iteration counts:
                // its cap is the sum of both phases' budgets
                const int cap = (mixed && !fp32) ? (int)std::min<long>(2L * max_iter, INT32_MAX) : max_iter;
                HIPCHK(cocg_reduce_beta(S, n_act, nrb, tol2, cap, fp32 ? 1 : 0, s_));
                HIPCHK(cocg_compact(S, s_));
                if (fp32)
                    std::swap(S.p32, S.pn32);
                else
                    std::swap(S.p, S.pn);
            }
            if (fp32) {
                if (timed) tm_.begin(T_REPLACE);
                HIPCHK(cocg32_replace(dv_, S, BV, ldbv, n_act, nrb, tol2, s_));
                if (timed) tm_.end();
            }
        };
        const bool use_graph = c_.o.use_graph != 0 && !tm_.on;
        hipGraphExec_t gexec = nullptr;
        int graph_nact = -1;
        struct GraphGuard {
            hipGraphExec_t* e;
            ~GraphGuard() {
                if (*e) (void)hipGraphExecDestroy(*e);
            }
        } gguard{&gexec};
        auto run_phase = [&]() {
        long it_phase = 0;
        while (n_act > 0 && it_phase < max_iter) {
            if (use_graph) {
                if (graph_nact != n_act) {
                    if (gexec) {
                        HIPCHK(hipGraphExecDestroy(gexec));
                        gexec = nullptr;
                    }
                    hipGraph_t graph = nullptr;
                    HIPCHK(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
                    enqueue_chunk(false);
                    HIPCHK(hipStreamEndCapture(s_, &graph));
                    hipError_t e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    HIPCHK(e);
                    graph_nact = n_act;
                    stats_.graph_captures += 1;
                }
                HIPCHK(hipGraphLaunch(gexec, s_));
            } else {
                enqueue_chunk(true);
            }
            stats_.spmm_launches += every;
            stats_.spmm_alg_bytes += every * mat_bytes();
            stats_.update_alg_bytes += every * mat_bytes();
            it += every;
            it_phase += every;
            if (fp32) {
                stats_.replacements += 1;
                // fold: read/write x64 and x32; residual: read x64, write u32
                stats_.replace_alg_bytes += (double)n_act * nmax * kTile * (32.0 + 16.0 + 16.0 + 8.0) +
                                            (double)dv_.nnz * 20.0;
            }
            HIPCHK(hipMemcpyAsync(counts_h_, S.counts, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            tm_.flush();
            n_act = counts_h_[0];
            if (c_.o.verbose > 0 && (it % c_.o.verbose) < every) {
                std::fprintf(stderr, "gep: pass columns %lld, iteration %ld, active tiles %d/%d, active columns %d\n",
                             (long long)(per * K), it, n_act, ntiles, counts_h_[1]);
                std::fflush(stderr);
            }
        }
        };
        // per-column iteration counts -> exact tile work for the byte count
        auto account = [&](double bytes_per_elem) {
            HIPCHK(hipMemcpyAsync(its.data(), S.iters, sizeof(int32_t) * Wp, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            for (int t = 0; t < ntiles; ++t) {
                int mx = 0;
                for (int l = 0; l < kTile; ++l) {
                    const size_t c = (size_t)t * kTile + l;
                    mx = std::max(mx, its[c] - its0[c]);
                }
                stats_.tile_iters += mx;
                const double tile_bytes = (double)tn[t] * kTile * bytes_per_elem;
                // kernel A: read u, p, write p' (3 passes); kernel B: read x, u, p', write x, u (5)
                stats_.spmm_alg_bytes += mx * 3.0 * tile_bytes;
                stats_.update_alg_bytes += mx * 5.0 * tile_bytes;
            }
            its0 = its;
        };
        run_phase();
        account(cb);
        if (mixed) {
            // fold the remaining FP32 corrections of every tile
            int32_t cntall[4] = {ntiles, (int32_t)(per * K), 0, 0};
            HIPCHK(hipMemcpyAsync(S.tiles, tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
            HIPCHK(hipMemcpyAsync(S.counts, cntall, sizeof(cntall), hipMemcpyHostToDevice, s_));
            HIPCHK(cocg32_fold(dv_, S, ntiles, nrb, s_));
            // FP64 completion of the columns the FP32 recurrence gave up on
            std::vector<int32_t> st(Wp);
            HIPCHK(hipMemcpyAsync(st.data(), S.stalled, sizeof(int32_t) * Wp, hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
            long n_stalled = 0;
            for (int32_t v : st) n_stalled += v != 0;
            if (n_stalled > 0) {
                stats_.fp64_columns += n_stalled;
                HIPCHK(hipStreamSynchronize(s_));
                x32.release();
                u32.release();
                p32.release();
                pn32.release();
                S.x32 = S.u32 = S.p32 = S.pn32 = nullptr;
                u.alloc(mv);
                p.alloc(mv);
                pn.alloc(mv);
                S.u = u.get();
                S.p = p.get();
                S.pn = pn.get();
                HIPCHK(hipMemsetAsync(S.u, 0, sizeof(double2) * mv, s_));
                HIPCHK(hipMemsetAsync(S.p, 0, sizeof(double2) * mv, s_));
                HIPCHK(hipMemsetAsync(S.pn, 0, sizeof(double2) * mv, s_));
                HIPCHK(hipMemcpyAsync(S.tiles, tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s_));
                HIPCHK(hipMemcpyAsync(S.counts, cntall, sizeof(cntall), hipMemcpyHostToDevice, s_));
                HIPCHK(cocg64_restart(dv_, S, BV, ldbv, nrb, tol2, s_));
                HIPCHK(hipMemcpyAsync(counts_h_, S.counts, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s_));
                HIPCHK(hipStreamSynchronize(s_));
                n_act = counts_h_[0];
                fp32 = false;
                if (gexec) {
                    HIPCHK(hipGraphExecDestroy(gexec));
                    gexec = nullptr;
                }
                graph_nact = -1;
                const long it0 = it;
                run_phase();
                stats_.fp64_iters += it - it0;
                account(16.0);
            }
        }
        stats_.cocg_iters += it;
        }
        // moments
        auto Sall = std::make_shared<DBuf<double>>(std::max<int64_t>(soff[K], 1));
        tm_.begin(T_MOMENTS);
        HIPCHK(launch_moments(S.x, S.geom, nmax, K, NH, L, M, d_coff.get(), d_cn.get(), d_soff.get(),
                              d_coef.get(), Sall->get(), s_));
        tm_.end();
        HIPCHK(hipStreamSynchronize(s_));
        // release the multivectors before the dense phase
        x.release();
        u.release();
        p.release();
        pn.release();
        x32.release();
        u32.release();
        p32.release();
        pn32.release();
        out.resize(K);
        for (int k = 0; k < K; ++k) {
            ContourOut& co = out[k];
            co.id = jobs[k].id;
            co.prob = jobs[k].prob;
            long mx = 0;
            double sum = 0.0;
            long cnt = 0;
            for (int j = 0; j < NH; ++j)
                for (int l = 0; l < L; ++l) {
                    const int v = its[coff[k] + (size_t)j * L + l];
                    mx = std::max<long>(mx, v);
                    sum += v;
                    ++cnt;
                }
            co.iters_max = mx;
            co.iters_mean = cnt ? sum / cnt : 0.0;
        }
        rayleigh_ritz_batch(Sall->get(), soff, jobs, r0, out);
    }

    // B-orthonormalise span(S_k) for every job k of the pass and extract all
    // Ritz pairs.  S_k is n_k x r0 row-major at Sall + soff[k].  Products run
    // one job at a time on the job's rows of the pencil; the small dense
    // solves (eigen-decompositions, Cholesky) run batched, one work-group per
    // job.
    void rayleigh_ritz_batch(const double* Sall, const std::vector<int64_t>& soff,
                             const std::vector<Job>& jobs, int r0, std::vector<ContourOut>& outs) {
        const DevPencil& D = dv_;
        const int K = (int)jobs.size();
        const size_t tot = (size_t)soff[K], rr2 = (size_t)r0 * r0;
        int64_t nmax = 0;
        for (const Job& j : jobs) nmax = std::max(nmax, j.n);
        DBuf<double> T(tot), Q1(tot), G(rr2 * K), U(rr2 * K), w((size_t)r0 * K), jw(std::max(rr2 * K, sym_eig_work_elems(r0, K)));
        DBuf<double> gw(gram_work_elems(nmax, r0, r0));
        DBuf<int32_t> ks(K), st(K);
        // pass 1: SVQB on the B-Gram G = S^T B S
        for (int k = 0; k < K; ++k) {
            const double* Sk = Sall + soff[k];
            const int64_t nk = jobs[k].n;
            HIPCHK(launch_spmm_real(D, Sk, r0, r0, nullptr, T.get() + soff[k], s_, jobs[k].row0, nk));
            gram(Sk, r0, T.get() + soff[k], r0, nk, r0, r0, G.get() + k * rr2, gw);
            HIPCHK(launch_symmetrise(G.get() + k * rr2, r0, s_));
        }
        tm_.begin(T_DENSE);
        HIPCHK(launch_sym_eig(G.get(), w.get(), U.get(), r0, K, nullptr, jw.get(), s_));
        tm_.end();
        std::vector<double> wh((size_t)r0 * K);
        HIPCHK(hipMemcpyAsync(wh.data(), w.get(), sizeof(double) * r0 * K, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        tm_.flush();
        std::vector<int32_t> keep(K, 0);
        int kmax = 0;
        for (int k = 0; k < K; ++k) {
            ContourOut& co = outs[k];
            const double* wk = wh.data() + (size_t)k * r0;
            const double wmax = wk[r0 - 1];
            if (wmax > 0.0) {
                const double cut = std::max(1, r0) * 2.220446049250313e-16 * wmax;
                for (int i = 0; i < r0; ++i)
                    if (wk[i] > cut) ++keep[k];
            }
            co.rank.push_back(keep[k]);
            if (co.rank.size() == 1) {
                co.smin_ratio = wmax > 0 ? std::sqrt(std::max(0.0, wk[0]) / wmax) : 0.0;
                co.saturated = co.smin_ratio > 1e-3;
            }
            co.r = keep[k];
            co.theta.assign(keep[k], 0.0);
            co.rho.assign(keep[k], 0.0);
            kmax = std::max(kmax, keep[k]);
        }
        std::shared_ptr<DBuf<double>> Xbuf;
        {
            LongLived ll;   // the Ritz vectors are kept until the solve's merge
            Xbuf = std::make_shared<DBuf<double>>(std::max<size_t>(tot, 1));
        }
        for (int k = 0; k < K; ++k) {
            outs[k].Xbuf = Xbuf;
            outs[k].X = Xbuf->get() + soff[k];
        }
        if (kmax == 0) return;
        HIPCHK(hipMemcpyAsync(ks.get(), keep.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s_));
        // Q1_k = S_k U_k,keep Sigma^-1/2; pass 2: Cholesky of Q1^T B Q1
        DBuf<double> Tsc(rr2 * K), LT(rr2 * K);
        for (int k = 0; k < K; ++k) {
            const int kk = keep[k];
            if (!kk) continue;
            const int64_t nk = jobs[k].n;
            HIPCHK(launch_svqb_scale(U.get() + k * rr2, w.get() + (size_t)k * r0, r0, kk, Tsc.get() + k * rr2, s_));
            gemm(Sall + soff[k], r0, Tsc.get() + k * rr2, kk, nk, r0, kk, Q1.get() + soff[k], kk);
            HIPCHK(launch_spmm_real(D, Q1.get() + soff[k], kk, kk, nullptr, T.get() + soff[k], s_, jobs[k].row0, nk));
            gram(Q1.get() + soff[k], kk, T.get() + soff[k], kk, nk, kk, kk, G.get() + k * rr2, gw);
            HIPCHK(launch_symmetrise(G.get() + k * rr2, kk, s_));
        }
        tm_.begin(T_DENSE);
        HIPCHK(launch_chol_inv(G.get(), LT.get(), r0, K, ks.get(), jw.get(), st.get(), s_));
        tm_.end();
        check_status(st, K, "B-Gram of the SVQB basis");
        // Q = Q1 L^-T (B-orthonormal); Rayleigh-Ritz matrices
        DBuf<double> Q(tot), AQ(tot), TA(rr2 * K), TB(rr2 * K);
        for (int k = 0; k < K; ++k) {
            const int kk = keep[k];
            if (!kk) continue;
            const int64_t nk = jobs[k].n;
            double* Qk = Q.get() + soff[k];
            gemm(Q1.get() + soff[k], kk, LT.get() + k * rr2, kk, nk, kk, kk, Qk, kk);
            HIPCHK(launch_spmm_real(D, Qk, kk, kk, AQ.get() + soff[k], T.get() + soff[k], s_, jobs[k].row0, nk));
            gram(Qk, kk, AQ.get() + soff[k], kk, nk, kk, kk, TA.get() + k * rr2, gw);
            gram(Qk, kk, T.get() + soff[k], kk, nk, kk, kk, TB.get() + k * rr2, gw);
            HIPCHK(launch_symmetrise(TA.get() + k * rr2, kk, s_));
            HIPCHK(launch_symmetrise(TB.get() + k * rr2, kk, s_));
        }
        Q1.release();
        tm_.begin(T_DENSE);
        HIPCHK(launch_chol_inv(TB.get(), LT.get(), r0, K, ks.get(), jw.get(), st.get(), s_));
        // C = L^-1 TA L^-T = LT^T TA LT
        DBuf<double> C1(rr2 * K), C2(rr2 * K), Z(rr2 * K), th((size_t)r0 * K);
        for (int k = 0; k < K; ++k) {
            const int kk = keep[k];
            if (!kk) continue;
            HIPCHK(launch_small_gemm(LT.get() + k * rr2, 1, TA.get() + k * rr2, 0, C1.get() + k * rr2, kk, kk, kk, kk, kk, kk, s_));
            HIPCHK(launch_small_gemm(C1.get() + k * rr2, 0, LT.get() + k * rr2, 0, C2.get() + k * rr2, kk, kk, kk, kk, kk, kk, s_));
            HIPCHK(launch_symmetrise(C2.get() + k * rr2, kk, s_));
        }
        HIPCHK(launch_sym_eig(C2.get(), th.get(), Z.get(), r0, K, ks.get(), jw.get(), s_));
        for (int k = 0; k < K; ++k) {
            const int kk = keep[k];
            if (!kk) continue;
            // U = L^-T Z
            HIPCHK(launch_small_gemm(LT.get() + k * rr2, 0, Z.get() + k * rr2, 0, C1.get() + k * rr2, kk, kk, kk, kk, kk, kk, s_));
        }
        tm_.end();
        check_status(st, K, "projected B matrix");
        DBuf<double> num((size_t)r0 * K), den((size_t)r0 * K), rw((size_t)2 * r0 * 1024);
        for (int k = 0; k < K; ++k) {
            const int kk = keep[k];
            if (!kk) continue;
            const int64_t nk = jobs[k].n;
            double* Xk = outs[k].X;
            gemm(Q.get() + soff[k], kk, C1.get() + k * rr2, kk, nk, kk, kk, Xk, kk);
            // residuals with the pencil itself
            HIPCHK(launch_spmm_real(D, Xk, kk, kk, AQ.get() + soff[k], T.get() + soff[k], s_, jobs[k].row0, nk));
            HIPCHK(launch_resid_norms(AQ.get() + soff[k], T.get() + soff[k], Xk, th.get() + (size_t)k * r0, nk, kk,
                                      num.get() + (size_t)k * r0, den.get() + (size_t)k * r0, rw.get(), s_));
        }
        std::vector<double> thh((size_t)r0 * K), nh((size_t)r0 * K), dh((size_t)r0 * K);
        HIPCHK(hipMemcpyAsync(thh.data(), th.get(), sizeof(double) * r0 * K, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(nh.data(), num.get(), sizeof(double) * r0 * K, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(dh.data(), den.get(), sizeof(double) * r0 * K, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        tm_.flush();
        for (int k = 0; k < K; ++k) {
            const double ainf = P_->h.prob_ainf[jobs[k].prob];
            for (int i = 0; i < keep[k]; ++i) {
                outs[k].theta[i] = thh[(size_t)k * r0 + i];
                outs[k].rho[i] = nh[(size_t)k * r0 + i] / (ainf * std::max(dh[(size_t)k * r0 + i], 1e-300));
            }
        }
    }

    void gram(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n, int64_t k1,
              int64_t k2, double* G, DBuf<double>& work) {
        // the split plan depends on (n, k1, k2): grow the partial buffer when a
        // call needs more than the pass planned
        const size_t need = gram_work_elems(n, k1, k2);
        if (need > work.n) work.alloc(need);
        tm_.begin(T_GRAM);
        HIPCHK(launch_gram(X, ld1, Y, ld2, n, k1, k2, G, work.get(), work.n, s_));
        tm_.end();
        gram_flops_ += 2.0 * n * k1 * k2;
    }
    void gemm(const double* X, int64_t ldx, const double* T, int64_t ldt, int64_t n, int64_t k,
              int64_t m, double* C, int64_t ldc) {
        tm_.begin(T_GEMM);
        HIPCHK(launch_gemm_tall(X, ldx, T, ldt, n, k, m, C, ldc, s_));
        tm_.end();
        gemm_flops_ += 2.0 * n * k * m;
    }
    void check_status(DBuf<int32_t>& st, int K, const char* what) {
        std::vector<int32_t> h(K, 0);
        HIPCHK(hipMemcpyAsync(h.data(), st.get(), sizeof(int32_t) * K, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        tm_.flush();
        for (int k = 0; k < K; ++k)
            if (h[k] != 0)
                fail(GEP_ENOTSPD, std::string("Cholesky failed on the ") + what + " of contour slot " +
                                      std::to_string(k) + " at pivot " + std::to_string(h[k]));
    }

    gep_pencil* P_;
    SolveCfg c_;
    DevPencil dv_;   // the pencil with the row-group view of this solve
    // banded factors of the last pass and the (problem, z) list they belong to
    std::unique_ptr<DBuf<double2>> band_F_;
    hipStream_t s2_ = nullptr;           // second stream of the factorisation (the pencil's)
    std::vector<double> band_keys_;
    std::unique_ptr<DBuf<double2>> band_wF_;   // kept wide / FP32 factors (any precision, bytes / 16)
    hipStream_t s_ = nullptr;
    hipStream_t own_ = nullptr;
    Timer tm_;
    Stats stats_;
    int32_t* counts_h_ = nullptr;
    double gram_flops_ = 0.0, gemm_flops_ = 0.0;
};

// Device bytes of one job in a wave.  bw >= 0: the job may take the band
// path (factors of its NH systems, x and the residual; with min_factor only
// one system's factor: the band path then factors its systems in groups);
// the larger of the two paths is planned.
static size_t bytes_per_job(int64_t n, int NH, int L, int M, bool mixed, int64_t bw, bool min_factor = false) {
    const size_t W = (size_t)((NH * L + kTile - 1) / kTile) * kTile;
    const size_t r = (size_t)L * M;
    // FP64: x, u, p, pn.  Mixed: x and four FP32 vectors, then (FP64
    // completion) x, u, p, pn again, so both are planned for the FP64 size.
    const size_t mv = (size_t)n * W * 16 * 4;
    // per-row-block partials: row blocks of at least 8 rows
    const size_t parts = W * (size_t)((n + 7) / 8) * 24;
    size_t solve = mv + parts;
    if (bw >= 0) {
        const size_t esz = mixed ? 8 : 16;
        const size_t fac = (size_t)(min_factor ? 1 : NH) * n * (size_t)(bw + 1) * esz;
        const size_t bandb = fac + (size_t)n * W * 16 * 2 + (mixed ? (size_t)n * W * 8 : 0) + W * 4096 * 16;
        solve = bw > kBandWideBw || mixed ? bandb : std::max(solve, bandb);
    }
    return solve + (size_t)n * r * 8 * 9 + (size_t)W * 160;
}

static std::string json_stats(const Solver& s, double wall_ms, const std::vector<ContourOut>& cos,
                              int precision) {
    std::ostringstream o;
    o.precision(10);
    // precision: what the shifted solves actually ran in ("mixed" when some
    // pass solved in FP32); precision_requested: the caller's option
    o << "{\"wall_ms\":" << wall_ms << ",\"precision\":\"" << (s.stats_.fp32_passes > 0 ? "mixed" : "fp64")
      << "\",\"precision_requested\":\"" << (precision == GEP_MIXED ? "mixed" : "fp64")
      << "\",\"method\":\"" << (s.c_.o.method == GEP_FEAST ? "feast" : "cirr")
      << "\",\"fp32_passes\":" << s.stats_.fp32_passes << ",\"solver_run\":\""
      << (s.stats_.ms_iters > 0 ? "multishift"
                                : s.stats_.band_factorisations > 0 ? (s.stats_.cocg_iters > 0 ? "band+cocg" : "band")
                                                                   : "cocg")
      << "\",\"cocg_iters\":" << s.stats_.cocg_iters << ",\"tile_iters\":" << s.stats_.tile_iters
      << ",\"multishift_iters\":" << s.stats_.ms_iters << ",\"multishift_unconverged\":" << s.stats_.ms_unconverged
      << ",\"columns\":" << s.stats_.columns << ",\"waves\":" << s.stats_.waves
      << ",\"spmm_launches\":" << s.stats_.spmm_launches
      << ",\"replacements\":" << s.stats_.replacements
      << ",\"fp64_columns\":" << s.stats_.fp64_columns << ",\"fp64_iters\":" << s.stats_.fp64_iters
      << ",\"band_factorisations\":" << s.stats_.band_factorisations
      << ",\"band_panel_steps\":" << s.stats_.band_panel_steps
      << ",\"band_solves\":" << s.stats_.band_solves
      << ",\"band_refinements\":" << s.stats_.band_refinements
      << ",\"band_pivot_flags\":" << s.stats_.band_pivot_flags
      << ",\"band_unconverged\":" << s.stats_.band_unconverged
      << ",\"band_relres_max\":" << s.stats_.band_relres_max
      << ",\"band_panel_flops\":" << s.stats_.band_panel_flops
      << ",\"band_update_flops\":" << s.stats_.band_update_flops
      << ",\"band_update_next_flops\":" << s.stats_.band_next_flops
      << ",\"band_solve_flops\":" << s.stats_.band_solve_flops
      << ",\"band_wide_flops\":" << s.stats_.band_wide_flops
      << ",\"graph_captures\":" << s.stats_.graph_captures
      << ",\"spmm_alg_bytes\":" << s.stats_.spmm_alg_bytes
      << ",\"update_alg_bytes\":" << s.stats_.update_alg_bytes
      << ",\"replace_alg_bytes\":" << s.stats_.replace_alg_bytes
      << ",\"gram_flops\":" << s.gram_flops_ << ",\"gemm_flops\":" << s.gemm_flops_
      << ",\"kernel_ms\":{";
    for (int c = 0; c < Timer::kClasses; ++c)
        o << (c ? "," : "") << "\"" << kTimerNames[c] << "\":" << s.tm_.total_ms(c);
    o << "},\"kernel_launches\":{";
    for (int c = 0; c < Timer::kClasses; ++c)
        o << (c ? "," : "") << "\"" << kTimerNames[c] << "\":" << s.tm_.seen[c];
    o << "},\"kernel_timed_launches\":{";
    for (int c = 0; c < Timer::kClasses; ++c)
        o << (c ? "," : "") << "\"" << kTimerNames[c] << "\":" << s.tm_.count[c];
    o << "},\"contours\":[";
    for (size_t i = 0; i < cos.size(); ++i) {
        const auto& c = cos[i];
        o << (i ? "," : "") << "{\"id\":" << c.id << ",\"problem\":" << c.prob << ",\"passes\":" << c.passes
          << ",\"rank\":[";
        for (size_t j = 0; j < c.rank.size(); ++j) o << (j ? "," : "") << c.rank[j];
        o << "],\"saturated\":" << (c.saturated ? "true" : "false") << ",\"smin_ratio\":" << c.smin_ratio
          << ",\"iters_max\":" << c.iters_max << ",\"iters_mean\":" << c.iters_mean << "}";
    }
    o << "]}";
    return o.str();
}

// Solve every problem of a (possibly single-element) batch.  contours[p] and
// n_contours[p] describe problem p's circles.  out[p] receives its result.
// Boundary-proximity check (robustness safeguards of the paper's appendix on
// mild distribution shifts): the value at lam of the rational filter that the
// N-node trapezoid rule applies to the spectrum (quadrature equation of the
// appendix on numerical quadrature), f(lam) = Re sum_j w_j / (z_j - lam),
// z_j = c + r zeta_j, w_j = r zeta_j / N, zeta_j = e^{i pi (2j - 1) / N}:
// 1 at the centre, 1/2 on the circle, about 0 outside.  Pairs with f below
// kNearBoundary sit in the filter's transition band, where the subspace
// holds them only weakly and eigenvalues just outside the circle leak in.
constexpr double kNearBoundary = 0.9;
static double quad_filter(const gep_contour& c, int N, double lam) {
    double f = 0.0;
    for (int j = 1; j <= N; ++j) {
        const double th = M_PI * (2.0 * j - 1.0) / N;
        const double zr = std::cos(th), zi = std::sin(th);
        const double dr = c.radius * zr + (c.center - lam), di = c.radius * zi;   // z_j - lam
        f += (c.radius * zr * dr + c.radius * zi * di) / (N * (dr * dr + di * di));
    }
    return f;
}

// "near_boundary_pairs" and "filter_min" of a result's pairs, for its JSON statistics.
static std::string boundary_stats(const std::vector<double>& filt) {
    int64_t near = 0;
    double fmin = 1.0;
    for (double f : filt) {
        near += f < kNearBoundary;
        fmin = std::min(fmin, f);
    }
    return "\"near_boundary_pairs\":" + std::to_string(near) + ",\"filter_min\":" +
           (std::isfinite(fmin) ? std::to_string(fmin) : std::string("null")) + ",";
}

static int solve_batch_impl(gep_pencil* P, int n_problems, const gep_contour* const* contours,
                            const int* n_contours, const SolveCfg& cfg, gep_result** out) {
    auto t0 = std::chrono::steady_clock::now();
    PoolScope pool_scope(&P->pool);
    P->pool.verbose = cfg.o.verbose;
    const HostPencil& H = P->h;
    const int64_t ntot = P->d.n;
    auto svp = std::make_unique<Solver>(P, cfg);
    Solver& sv = *svp;
    hipStream_t s = sv.s_;
    const int L = cfg.L;
    // V (problem p: counter-based stream of seed + p on its own rows) and B V
    DBuf<double> V((size_t)ntot * L), BV((size_t)ntot * L);
    if (cfg.o.rhs) {
        if (n_problems != 1) fail(GEP_EINVAL, "an explicit right-hand-side block needs a single problem");
        const int64_t n = ntot;
        std::vector<double> vc((size_t)n * L), vr((size_t)n * L);
        if (cfg.o.inputs_on_device)
            HIPCHK(hipMemcpy(vc.data(), cfg.o.rhs, sizeof(double) * n * L, hipMemcpyDeviceToHost));
        else
            std::memcpy(vc.data(), cfg.o.rhs, sizeof(double) * n * L);
        for (int64_t i = 0; i < n; ++i)
            for (int l = 0; l < L; ++l) vr[(size_t)i * L + l] = vc[(size_t)l * n + i];
        HIPCHK(hipMemcpyAsync(V.get(), vr.data(), sizeof(double) * n * L, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        for (int p = 0; p < n_problems; ++p)
            HIPCHK(launch_gaussian(cfg.o.seed + (uint64_t)p, H.prob_n[p], L, V.get() + H.prob_row0[p] * L, s));
    }
    HIPCHK(launch_spmm_real(P->d, V.get(), L, L, nullptr, BV.get(), s));
    V.release();
    // jobs and memory plan: waves of jobs in order
    std::vector<Job> all;
    int64_t boff = 0;   // problem p's first entry of cfg.o.blocks (problems in order)
    for (int p = 0; p < n_problems; boff += n_contours[p], ++p)
        for (int k = 0; k < n_contours[p]; ++k) {
            Job j;
            j.c = contours[p][k];
            j.prob = p;
            j.id = k;
            j.row0 = H.prob_row0[p];
            j.n = H.prob_n[p];
            j.bsrc0 = H.prob_row0[p] * L;
            j.L = cfg.o.blocks ? cfg.o.blocks[boff + k] : L;
            all.push_back(j);
        }
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    // memory the pencil's idle workspace holds is available to this solve
    const double budget = cfg.o.mem_limit_bytes > 0 ? cfg.o.mem_limit_bytes
                                                    : 0.85 * (double)(freeb + P->pool.idle_bytes);
    const bool mixed = cfg.o.precision == GEP_MIXED;
    std::vector<ContourOut> finals(all.size());
    // jobs ordered by block size so that equal sizes share waves
    std::vector<size_t> ord(all.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    // (larger problems first among equal block sizes, so that a wave holds
    // problems of similar size and its banded factorisation no more steps
    // than its largest problem needs)
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        return all[a].L != all[b].L ? all[a].L < all[b].L : all[a].n > all[b].n;
    });
    std::vector<Job> sorted_jobs;
    for (size_t i : ord) sorted_jobs.push_back(all[i]);
    // waves: consecutive jobs with the same block size within the budget
    struct Wave {
        size_t k0, k1;
        double used;
    };
    std::vector<Wave> plan;
    double long_lived = 0.0, max_used = 0.0;
    for (size_t k0 = 0; k0 < sorted_jobs.size();) {
        size_t k1 = k0;
        double used = 0.0;
        const int Lw = sorted_jobs[k0].L;
        while (k1 < sorted_jobs.size() && sorted_jobs[k1].L == Lw) {
            const int pj = sorted_jobs[k1].prob;
            const int64_t bwj = (cfg.o.solver != 1 && P->h.prob_bw[pj] <= kBandMaxBw) ? P->h.prob_bw[pj] : -1;
            double need = (double)bytes_per_job(sorted_jobs[k1].n, cfg.NH, Lw, cfg.M, mixed, bwj);
            // a job whose factors alone exceed the budget factors its systems in groups
            if (bwj >= 0 && need > budget)
                need = (double)bytes_per_job(sorted_jobs[k1].n, cfg.NH, Lw, cfg.M, mixed, bwj, true);
            if (k1 > k0 && used + need > budget) break;
            used += need;
            long_lived += (double)sorted_jobs[k1].n * Lw * cfg.M * 8.0;   // Ritz vectors kept to the merge
            ++k1;
        }
        if (used > budget)
            fail(GEP_ENOMEM, "one contour needs " + std::to_string((long long)used) + " bytes of device memory");
        plan.push_back({k0, k1, used});
        max_used = std::max(max_used, used);
        k0 = k1;
    }
    // one region for every wave (memory given back with hipFree does not
    // become allocatable again right away, so waves of different shapes
    // must share what the first one obtained)
    P->pool.reserve((size_t)std::min(1.06 * max_used + long_lived + (double)(1 << 30),
                                     0.95 * (double)(freeb + P->pool.largest_free())));
    for (const Wave& wv : plan) {
        const size_t k0 = wv.k0, k1 = wv.k1;
        const double used = wv.used;
        const int Lw = sorted_jobs[k0].L;
        std::vector<Job> jobs(sorted_jobs.begin() + k0, sorted_jobs.begin() + k1);
        std::vector<ContourOut> res;
        sv.stats_.waves += 1;
        if (cfg.o.verbose > 0) {
            size_t fb = 0, tb = 0;
            (void)hipMemGetInfo(&fb, &tb);
            std::fprintf(stderr,
                         "[gep] wave %d: jobs %zu..%zu, planned %.2f GB of budget %.2f GB; free %.2f GB, "
                         "pool live %.2f GB idle %.2f GB\n",
                         sv.stats_.waves, k0, k1 - 1, used / 1e9, budget / 1e9, fb / 1e9,
                         P->pool.live_bytes / 1e9, P->pool.idle_bytes / 1e9);
        }
        sv.run_pass(jobs, BV.get(), L, Lw, cfg.M, res);
        for (auto& r : res) r.passes = 1;
        // refinement: jobs whose kept pairs miss tol (FEAST-type pass, V <- all Ritz vectors)
        for (int pass = 1; pass <= cfg.o.max_refine; ++pass) {
            std::vector<int> redo;
            for (size_t i = 0; i < res.size(); ++i) {
                const gep_contour& c = jobs[i].c;
                bool bad = false;
                for (int j = 0; j < res[i].r; ++j)
                    if (res[i].theta[j] >= c.keep_lo && res[i].theta[j] < c.keep_hi && !(res[i].rho[j] <= cfg.tol))
                        bad = true;
                if (bad) redo.push_back((int)i);
            }
            if (redo.empty()) break;
            int L2 = 0;
            for (int i : redo) L2 = std::max(L2, res[i].r);
            // per-job row-major blocks n_k x L2 (columns beyond the job's rank stay zero)
            std::vector<Job> jobs2;
            int64_t off = 0;
            for (int i : redo) {
                Job j = jobs[i];
                j.bsrc0 = off;
                j.L = L2;
                off += j.n * L2;
                jobs2.push_back(j);
            }
            DBuf<double> V2((size_t)off), BV2((size_t)off);
            HIPCHK(hipMemsetAsync(V2.get(), 0, sizeof(double) * off, s));
            for (size_t a = 0; a < redo.size(); ++a) {
                const ContourOut& co = res[redo[a]];
                const Job& j = jobs2[a];
                if (co.r > 0)
                    HIPCHK(hipMemcpy2DAsync(V2.get() + j.bsrc0, sizeof(double) * L2, co.X, sizeof(double) * co.r,
                                            sizeof(double) * co.r, j.n, hipMemcpyDeviceToDevice, s));
                HIPCHK(launch_spmm_real(P->d, V2.get() + j.bsrc0, L2, L2, nullptr, BV2.get() + j.bsrc0, s, j.row0, j.n));
            }
            std::vector<ContourOut> res2;
            sv.run_pass(jobs2, BV2.get(), L2, L2, 1, res2);
            for (size_t a = 0; a < redo.size(); ++a) {
                ContourOut& dst = res[redo[a]];
                ContourOut& src = res2[a];
                src.passes = dst.passes + 1;
                std::vector<int> rk = dst.rank;
                rk.insert(rk.end(), src.rank.begin(), src.rank.end());
                src.rank = rk;
                src.saturated = dst.saturated;
                src.smin_ratio = dst.smin_ratio;
                src.iters_max = std::max(src.iters_max, dst.iters_max);
                dst = src;
            }
        }
        for (size_t i = 0; i < res.size(); ++i) finals[ord[k0 + i]] = res[i];
        // this wave's factors are no longer needed: free them for the next wave
        sv.band_F_.reset();
        sv.band_wF_.reset();
        sv.band_keys_.clear();
    }
    // per problem: selection, gather, merge
    const double wall_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = GEP_OK;
    size_t base = 0;
    for (int p = 0; p < n_problems; ++p) {
        const int K = n_contours[p];
        const int64_t n = H.prob_n[p];
        const int64_t row0 = H.prob_row0[p];
        struct Pair {
            double lam, rho;
            int cid;
            int col;
        };
        std::vector<Pair> pairs;
        // selected Ritz vectors of contour k stay on the device: n x sel, column-major
        std::vector<std::unique_ptr<DBuf<double>>> cms(K);
        bool saturated = false;
        std::vector<ContourOut> mine(finals.begin() + base, finals.begin() + base + K);
        for (int k = 0; k < K; ++k) {
            ContourOut& co = mine[k];
            const gep_contour& cc = contours[p][k];
            saturated |= co.saturated;
            std::vector<int32_t> sel;
            for (int j = 0; j < co.r; ++j)
                if (co.theta[j] >= cc.keep_lo && co.theta[j] < cc.keep_hi) sel.push_back(j);
            if (sel.empty()) continue;
            DBuf<int32_t> dsel(sel.size());
            cms[k] = std::make_unique<DBuf<double>>((size_t)n * sel.size());
            HIPCHK(hipMemcpyAsync(dsel.get(), sel.data(), sizeof(int32_t) * sel.size(), hipMemcpyHostToDevice, s));
            DBuf<double> gwork(gather_cols_work(n, (int)sel.size()));
            HIPCHK(launch_gather_cols(co.X, n, co.r, dsel.get(), (int)sel.size(), cms[k]->get(), gwork.get(), s));
            HIPCHK(hipStreamSynchronize(s));   // dsel and gwork are released at the end of this iteration
            for (size_t a = 0; a < sel.size(); ++a) pairs.push_back({co.theta[sel[a]], co.rho[sel[a]], k, (int)a});
        }
        std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) { return a.lam < b.lam; });
        // Merge pairs that several contours found for one eigenvalue.  Values
        // form clusters (consecutive values within 1e-8 relative).  In a
        // cluster holding pairs of more than one contour, the contour whose
        // cluster pairs have the smallest worst residual (lowest id on ties)
        // keeps them all; the other contours' pairs follow in ascending
        // residual and are dropped when their B-orthogonal projection onto the
        // span of the pairs kept so far has B-norm >= 0.9 of their own.  Pairs
        // of one contour are never merged (exact multiple eigenvalues keep all
        // their vectors).  Only the vectors of such clusters come to the host.
        auto fetch = [&](const Pair& q, std::vector<double>& h) {
            h.resize((size_t)n);
            HIPCHK(hipMemcpyAsync(h.data(), cms[q.cid]->get() + (size_t)q.col * n, sizeof(double) * n,
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        };
        auto bmul = [&](const std::vector<double>& x, std::vector<double>& y) {
            y.assign((size_t)n, 0.0);
            for (int64_t i = 0; i < n; ++i) {
                double t = 0.0;
                for (int32_t e = H.rowptr[row0 + i]; e < H.rowptr[row0 + i + 1]; ++e)
                    t += H.b[e] * x[H.colind[e] - row0];
                y[i] = t;
            }
        };
        auto dot = [&](const std::vector<double>& x, const std::vector<double>& y) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc += x[i] * y[i];
            return acc;
        };
        std::vector<char> drop(pairs.size(), 0);
        for (size_t c0 = 0; c0 < pairs.size();) {
            size_t c1 = c0 + 1;
            while (c1 < pairs.size() &&
                   pairs[c1].lam - pairs[c1 - 1].lam <=
                       1e-8 * std::max(std::fabs(pairs[c1].lam), std::fabs(pairs[c1 - 1].lam)))
                ++c1;
            std::vector<std::pair<double, int>> owners;   // (worst residual, contour)
            for (size_t a = c0; a < c1; ++a) {
                auto it = std::find_if(owners.begin(), owners.end(),
                                       [&](const std::pair<double, int>& o) { return o.second == pairs[a].cid; });
                if (it == owners.end())
                    owners.push_back({pairs[a].rho, pairs[a].cid});
                else
                    it->first = std::max(it->first, pairs[a].rho);
            }
            if (owners.size() > 1) {
                std::sort(owners.begin(), owners.end());
                const size_t m = c1 - c0;
                std::vector<std::vector<double>> xv(m), bx(m);
                for (size_t a = 0; a < m; ++a) {
                    fetch(pairs[c0 + a], xv[a]);
                    bmul(xv[a], bx[a]);
                }
                std::vector<size_t> kept;
                for (size_t a = 0; a < m; ++a)
                    if (pairs[c0 + a].cid == owners[0].second) kept.push_back(a);
                for (size_t o = 1; o < owners.size(); ++o) {
                    std::vector<size_t> mine;
                    for (size_t a = 0; a < m; ++a)
                        if (pairs[c0 + a].cid == owners[o].second) mine.push_back(a);
                    std::stable_sort(mine.begin(), mine.end(), [&](size_t u, size_t v) {
                        return pairs[c0 + u].rho < pairs[c0 + v].rho;
                    });
                    for (size_t a : mine) {
                        // proj2 = b^T G^{-1} b, G = K^T B K, b = K^T B x (Cholesky of G)
                        const size_t q = kept.size();
                        std::vector<double> G(q * q), rhs(q);
                        for (size_t u = 0; u < q; ++u) {
                            rhs[u] = dot(xv[kept[u]], bx[a]);
                            for (size_t v = 0; v <= u; ++v) G[u * q + v] = dot(xv[kept[u]], bx[kept[v]]);
                        }
                        bool spd = true;
                        for (size_t j = 0; j < q && spd; ++j) {
                            double d = G[j * q + j];
                            for (size_t t = 0; t < j; ++t) d -= G[j * q + t] * G[j * q + t];
                            if (!(d > 0.0)) {
                                spd = false;
                                break;
                            }
                            d = std::sqrt(d);
                            G[j * q + j] = d;
                            for (size_t i = j + 1; i < q; ++i) {
                                double v = G[i * q + j];
                                for (size_t t = 0; t < j; ++t) v -= G[i * q + t] * G[j * q + t];
                                G[i * q + j] = v / d;
                            }
                        }
                        double proj2 = 0.0;
                        if (spd) {
                            for (size_t i = 0; i < q; ++i) {   // forward solve L y = b
                                double v = rhs[i];
                                for (size_t t = 0; t < i; ++t) v -= G[i * q + t] * rhs[t];
                                rhs[i] = v / G[i * q + i];
                                proj2 += rhs[i] * rhs[i];
                            }
                        }
                        if (proj2 >= 0.81 * dot(xv[a], bx[a]))
                            drop[c0 + a] = 1;
                        else
                            kept.push_back(a);
                    }
                }
            }
            c0 = c1;
        }
        auto* R = new gep_result();
        R->n = n;
        bool noconv = false;
        size_t kept = 0;
        for (size_t a = 0; a < pairs.size(); ++a) kept += !drop[a];
        if (kept) {
            PoolScope own(nullptr);   // the result outlives the pencil's workspace
            R->dvecs = std::make_unique<DBuf<double>>((size_t)n * kept);
        }
        size_t idx = 0;
        for (size_t a = 0; a < pairs.size(); ++a) {
            if (drop[a]) continue;
            const Pair& pr = pairs[a];
            R->evals.push_back(pr.lam);
            R->resid.push_back(pr.rho);
            R->cid.push_back(pr.cid);
            R->filt.push_back(quad_filter(contours[p][pr.cid], cfg.N, pr.lam));
            const bool ok = pr.rho <= cfg.tol;
            noconv |= !ok;
            R->conv.push_back(ok ? 1 : 0);
            HIPCHK(hipMemcpyAsync(R->dvecs->get() + idx * n, cms[pr.cid]->get() + (size_t)pr.col * n,
                                  sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            ++idx;
        }
        HIPCHK(hipStreamSynchronize(s));
        R->m = (int64_t)R->evals.size();
        for (const ContourOut& co : mine) R->csat.push_back(co.saturated ? 1 : 0);
        R->stats = json_stats(sv, wall_solve, mine, cfg.o.precision);
        R->stats.insert(1, boundary_stats(R->filt));
        R->stats.insert(1, "\"wall_select_ms\":" +
                               std::to_string(std::chrono::duration<double, std::milli>(
                                                  std::chrono::steady_clock::now() - t0).count() - wall_solve) + ",");
        out[p] = R;
        const int st = noconv ? GEP_WNOCONV : (saturated ? GEP_WSATURATED : GEP_OK);
        if (st == GEP_WNOCONV || (st == GEP_WSATURATED && worst == GEP_OK)) worst = st;
        base += K;
    }
    // release the solver's device buffers; the time it takes is reported
    const auto tf = std::chrono::steady_clock::now();
    svp.reset();
    const double free_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
    for (int p = 0; p < n_problems; ++p)
        if (out[p]) out[p]->stats.insert(1, "\"wall_free_ms\":" + std::to_string(free_ms) + ",");
    return worst;
}

static int solve_impl(gep_pencil* P, const gep_contour* contours, int K, const SolveCfg& cfg,
                      gep_result** out) {
    const gep_contour* cs[1] = {contours};
    int nk[1] = {K};
    return solve_batch_impl(P, 1, cs, nk, cfg, out);
}

}  // namespace gep

// ---- C ABI ------------------------------------------------------------------
extern "C" {

void gep_opts_default(gep_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->seed = 1;
    o->precision = GEP_FP64;
    o->max_refine = 1;
    o->solve_tol = 1e-9;
    o->max_iter = 100000;
    o->check_every = 16;
    o->stream = nullptr;
    o->inputs_on_device = 0;
    o->rhs = nullptr;
    o->mem_limit_bytes = 0.0;
    o->timing = 0;
    o->band_kernels = 0;
    o->rows_per_block = 0;
    o->verbose = 0;
    o->use_graph = 1;
    o->blocks = nullptr;
    o->row_group = 0;
    o->solver = 0;
}

const char* gep_strerror(int st) {
    switch (st) {
        case GEP_OK: return "ok";
        case GEP_EINVAL: return "invalid argument";
        case GEP_ENOTSYM: return "matrix not symmetric";
        case GEP_ENOTSPD: return "B not positive definite";
        case GEP_ENOMEM: return "out of device memory";
        case GEP_EDEVICE: return "HIP runtime error";
        case GEP_WNOCONV: return "warning: some pairs did not reach the residual tolerance";
        case GEP_WSATURATED: return "warning: saturated subspace, eigenvalues may be missed";
        default: return "unknown status";
    }
}

const char* gep_last_error(void) { return gep::g_err.c_str(); }

int gep_pencil_create(const gep_csr* A, const gep_csr* B, int on_dev, void* stream, gep_pencil** out) {
    (void)stream;
    if (!out) {
        gep::set_error("out is NULL");
        return GEP_EINVAL;
    }
    *out = nullptr;
    auto* P = new gep_pencil();
    try {
        gep::pack(A, B, on_dev != 0, P->h);
        gep::upload(P->h, P);
    } catch (const gep::Fail& f) {
        delete P;
        return f.code;
    }
    *out = P;
    return GEP_OK;
}

void gep_pencil_free(gep_pencil* p) { delete p; }

int gep_pencil_info(const gep_pencil* p, int64_t* n, int64_t* nnz, double* a_inf) {
    if (!p) return GEP_EINVAL;
    if (n) *n = p->d.n;
    if (nnz) *nnz = p->d.nnz;
    if (a_inf) *a_inf = p->d.a_inf;
    return GEP_OK;
}

static int validate_problem(const gep_contour* contours, int K, int N, int M, int L, double tol,
                            const gep_opts* o) {
    if (!contours || K <= 0) { gep::set_error("no contours"); return GEP_EINVAL; }
    if (N < 2 || (N & 1)) { gep::set_error("n_nodes must be even and >= 2"); return GEP_EINVAL; }
    if (M < 1 || M > 16) { gep::set_error("moments must be in [1, 16]"); return GEP_EINVAL; }
    if (L < 1) { gep::set_error("block must be >= 1"); return GEP_EINVAL; }
    if ((int64_t)L * M > 1024) { gep::set_error("block*moments must be <= 1024"); return GEP_EINVAL; }
    if (!(tol > 0.0)) { gep::set_error("tol must be > 0"); return GEP_EINVAL; }
    if (o->precision != GEP_FP64 && o->precision != GEP_MIXED) { gep::set_error("bad precision"); return GEP_EINVAL; }
    if (!(o->solve_tol > 0.0) || o->max_iter < 1) { gep::set_error("bad solve_tol/max_iter"); return GEP_EINVAL; }
    if (o->rows_per_block < 0) { gep::set_error("rows_per_block must be >= 0"); return GEP_EINVAL; }
    if (o->row_group != 0 && o->row_group != 1 && o->row_group != 4) {
        gep::set_error("row_group must be 0, 1 or 4");
        return GEP_EINVAL;
    }
    if (o->solver < 0 || o->solver > 3) {
        gep::set_error("solver must be 0 (automatic), 1 (COCG), 2 (band) or 3 (multi-shift COCG)");
        return GEP_EINVAL;
    }
    if (o->method != GEP_CIRR && o->method != GEP_FEAST) {
        gep::set_error("method must be GEP_CIRR (0) or GEP_FEAST (1)");
        return GEP_EINVAL;
    }
    if (o->band_group < 0) {
        gep::set_error("band_group must be >= 0");
        return GEP_EINVAL;
    }
    if (o->band_kernels < 0 || o->band_kernels > 2) {
        gep::set_error("band_kernels must be 0 (automatic), 1 or 2");
        return GEP_EINVAL;
    }
    for (int k = 0; k < K; ++k) {
        const gep_contour& c = contours[k];
        if (!std::isfinite(c.center) || !std::isfinite(c.radius) || !(c.radius > 0.0) ||
            !std::isfinite(c.keep_lo) || !std::isfinite(c.keep_hi) || !(c.keep_lo < c.keep_hi) ||
            c.keep_lo < c.center - c.radius * (1 + 1e-12) || c.keep_hi > c.center + c.radius * (1 + 1e-12)) {
            gep::set_error("contour " + std::to_string(k) + " is invalid (radius, or keep window outside the circle)");
            return GEP_EINVAL;
        }
    }
    return GEP_OK;
}

int gep_ci_solve_pencil(gep_pencil* P, const gep_contour* contours, int K, int N, int M, int L,
                        double tol, const gep_opts* opts, gep_result** out) {
    if (!out || !P) { gep::set_error("NULL pencil or out"); return GEP_EINVAL; }
    *out = nullptr;
    if (P->h.prob_n.size() != 1) {
        gep::set_error("a batch pencil is solved with gep_ci_solve_pencil_batch");
        return GEP_EINVAL;
    }
    gep_opts o;
    if (opts) o = *opts; else gep_opts_default(&o);
    int st = validate_problem(contours, K, N, M, L, tol, &o);
    if (st) return st;
    if (o.blocks)
        for (int k = 0; k < K; ++k)
            if (o.blocks[k] < 1 || o.blocks[k] > L) {
                gep::set_error("blocks[" + std::to_string(k) + "] must be in [1, block]");
                return GEP_EINVAL;
            }
    gep::SolveCfg cfg;
    cfg.N = N;
    cfg.NH = N / 2;
    cfg.M = o.method == GEP_FEAST ? 1 : M;
    cfg.L = L;
    cfg.tol = tol;
    cfg.o = o;
    try {
        return gep::solve_impl(P, contours, K, cfg, out);
    } catch (const gep::Fail& f) {
        return f.code;
    }
}

int gep_ci_solve(const gep_csr* A, const gep_csr* B, const gep_contour* contours, int n_contours,
                 int n_nodes, int moments, int block, double tol, const gep_opts* opts,
                 gep_result** out) {
    if (!out) { gep::set_error("out is NULL"); return GEP_EINVAL; }
    *out = nullptr;
    gep_opts o;
    if (opts) o = *opts; else gep_opts_default(&o);
    int st = validate_problem(contours, n_contours, n_nodes, moments, block, tol, &o);
    if (st) return st;
    gep_pencil* P = nullptr;
    st = gep_pencil_create(A, B, o.inputs_on_device, o.stream, &P);
    if (st) return st;
    st = gep_ci_solve_pencil(P, contours, n_contours, n_nodes, moments, block, tol, &o, out);
    gep_pencil_free(P);
    return st;
}

int gep_pencil_create_batch(int n_problems, const gep_csr* A, const gep_csr* B, int on_dev, void* stream,
                            gep_pencil** out) {
    (void)stream;
    if (!out || n_problems <= 0 || !A || !B) {
        gep::set_error("bad batch pencil arguments");
        return GEP_EINVAL;
    }
    *out = nullptr;
    auto* P = new gep_pencil();
    try {
        for (int p = 0; p < n_problems; ++p) {
            gep::HostPencil h;
            try {
                gep::pack(&A[p], &B[p], on_dev != 0, h);
            } catch (const gep::Fail& f) {
                gep::set_error("problem " + std::to_string(p) + ": " + gep::g_err);
                throw;
            }
            gep::append_pencil(P->h, h);
        }
        if (P->h.nnz >= (1ll << 31) - 1) gep::fail(GEP_EINVAL, "batch nnz >= 2^31");
        gep::upload(P->h, P);
    } catch (const gep::Fail& f) {
        delete P;
        return f.code;
    }
    *out = P;
    return GEP_OK;
}

int gep_pencil_problems(const gep_pencil* p, int* n_problems) {
    if (!p || !n_problems) return GEP_EINVAL;
    *n_problems = (int)p->h.prob_n.size();
    return GEP_OK;
}

int gep_ci_solve_pencil_batch(gep_pencil* P, const gep_contour* const* contours, const int* n_contours,
                              int n_nodes, int moments, int block, double tol, const gep_opts* opts,
                              gep_result** out) {
    if (!out || !P || !contours || !n_contours) {
        gep::set_error("bad batch arguments");
        return GEP_EINVAL;
    }
    const int n_problems = (int)P->h.prob_n.size();
    for (int p = 0; p < n_problems; ++p) out[p] = nullptr;
    gep_opts o;
    if (opts) o = *opts; else gep_opts_default(&o);
    int64_t nk = 0;
    for (int p = 0; p < n_problems; ++p) {
        int st = validate_problem(contours[p], n_contours[p], n_nodes, moments, block, tol, &o);
        if (st) {
            gep::set_error("problem " + std::to_string(p) + ": " + gep::g_err);
            return st;
        }
        nk += n_contours[p];
    }
    if (o.blocks)
        for (int64_t k = 0; k < nk; ++k)
            if (o.blocks[k] < 1 || o.blocks[k] > block) {
                gep::set_error("blocks[" + std::to_string(k) + "] must be in [1, block]");
                return GEP_EINVAL;
            }
    gep::SolveCfg cfg;
    cfg.N = n_nodes;
    cfg.NH = n_nodes / 2;
    cfg.M = o.method == GEP_FEAST ? 1 : moments;
    cfg.L = block;
    cfg.tol = tol;
    cfg.o = o;
    try {
        return gep::solve_batch_impl(P, n_problems, contours, n_contours, cfg, out);
    } catch (const gep::Fail& f) {
        for (int p = 0; p < n_problems; ++p) {
            delete out[p];
            out[p] = nullptr;
        }
        return f.code;
    }
}

int gep_ci_solve_batch(int n_problems, const gep_csr* A, const gep_csr* B,
                       const gep_contour* const* contours, const int* n_contours, int n_nodes,
                       int moments, int block, double tol, const gep_opts* opts, gep_result** out) {
    if (!out || n_problems <= 0 || !A || !B || !contours || !n_contours) {
        gep::set_error("bad batch arguments");
        return GEP_EINVAL;
    }
    for (int p = 0; p < n_problems; ++p) out[p] = nullptr;
    gep_opts o;
    if (opts) o = *opts; else gep_opts_default(&o);
    for (int p = 0; p < n_problems; ++p) {
        int st = validate_problem(contours[p], n_contours[p], n_nodes, moments, block, tol, &o);
        if (st) {
            gep::set_error("problem " + std::to_string(p) + ": " + gep::g_err);
            return st;
        }
    }
    gep_pencil* P = nullptr;
    int st = gep_pencil_create_batch(n_problems, A, B, o.inputs_on_device, o.stream, &P);
    if (st) return st;
    st = gep_ci_solve_pencil_batch(P, contours, n_contours, n_nodes, moments, block, tol, &o, out);
    gep_pencil_free(P);
    return st;
}

int gep_ci_solve_smallest(gep_pencil* P, int64_t m, double lower, int per_contour, int n_nodes, int moments,
                          int block, double tol, const gep_opts* opts, gep_result** out) {
    if (!out || !P) { gep::set_error("NULL pencil or out"); return GEP_EINVAL; }
    *out = nullptr;
    if (P->h.prob_n.size() != 1) { gep::set_error("one pencil per call"); return GEP_EINVAL; }
    const int64_t n = P->h.n;
    if (m < 1 || m > n) { gep::set_error("m must be in [1, n]"); return GEP_EINVAL; }
    if (per_contour < 1) { gep::set_error("per_contour must be >= 1"); return GEP_EINVAL; }
    if (!std::isfinite(lower)) { gep::set_error("lower must be finite"); return GEP_EINVAL; }
    gep_opts o;
    if (opts) o = *opts; else gep_opts_default(&o);
    o.blocks = nullptr;
    const gep::HostPencil& H = P->h;
    try {
        // largest eigenvalue estimate: power iteration on diag(B)^-1 A, its
        // Rayleigh quotient x^T A x / x^T B x (only the first window uses it)
        std::vector<double> x((size_t)n), y((size_t)n);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        for (int64_t i = 0; i < n; ++i) {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            x[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
        }
        double lmax = 0.0;
        for (int it = 0; it < 60; ++it) {
            double xax = 0.0, xbx = 0.0, nrm = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double ax = 0.0, bx = 0.0;
                for (int32_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) {
                    ax += H.a[e] * x[H.colind[e]];
                    bx += H.b[e] * x[H.colind[e]];
                }
                xax += x[i] * ax;
                xbx += x[i] * bx;
                y[i] = ax / H.dB[i];
                nrm += y[i] * y[i];
            }
            if (xbx > 0) lmax = std::max(lmax, xax / xbx);
            nrm = std::sqrt(nrm);
            if (!(nrm > 0)) break;
            for (int64_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
        }
        if (!(lmax > lower)) gep::fail(GEP_EINVAL, "no spectrum above the lower bound");
        struct Found {
            double lam, rho;
            int cid;
            const gep_result* res;
            int col;
        };
        struct Span {
            double a, b;
            int depth;
        };
        std::vector<std::unique_ptr<gep_result, void (*)(gep_result*)>> rounds;
        std::vector<Found> found;
        // The first window assumes the fastest growth of the count with the
        // eigenvalue among 1D-3D Weyl laws (N ~ n (lambda / lmax)^(1/2)), so it
        // holds at most about m; later windows are sized by the density found
        // so far.  A circle whose subspace is saturated or that leaves a kept
        // pair above tol is solved again as three circles.
        double covered = lower;
        double first = lower + (lmax - lower) * std::min(1.0, std::pow((double)m / (double)n, 2.0));
        std::vector<Span> pending{{lower, first, 0}};
        covered = first;
        int circle0 = 0, worst = GEP_OK, windows = 1;
        for (int round = 0; round < 40 && !pending.empty(); ++round) {
            const int K = (int)pending.size();
            std::vector<gep_contour> cs(K);
            for (int k = 0; k < K; ++k) {
                const double a = pending[k].a, b = pending[k].b;
                cs[k] = {0.5 * (a + b), 0.55 * (b - a), a, b};
            }
            gep::SolveCfg cfg;
            cfg.N = n_nodes;
            cfg.NH = n_nodes / 2;
            cfg.M = o.method == GEP_FEAST ? 1 : moments;
            cfg.L = block;
            cfg.tol = tol;
            cfg.o = o;
            int stv = validate_problem(cs.data(), K, n_nodes, moments, block, tol, &o);
            if (stv) return stv;
            gep_result* r = nullptr;
            stv = gep::solve_impl(P, cs.data(), K, cfg, &r);
            if (stv < 0) return stv;
            rounds.emplace_back(r, gep_result_free);
            std::vector<char> bad(K, 0);
            for (int k = 0; k < K; ++k) bad[k] = k < (int)r->csat.size() && r->csat[k];
            for (int64_t q = 0; q < r->m; ++q)
                if (!r->conv[q]) bad[r->cid[q]] = 1;
            std::vector<Span> next;
            for (int k = 0; k < K; ++k) {
                if (bad[k] && pending[k].depth < 4) {
                    const double a = pending[k].a, w3 = (pending[k].b - a) / 3.0;
                    for (int t = 0; t < 3; ++t) next.push_back({a + t * w3, a + (t + 1) * w3, pending[k].depth + 1});
                    continue;
                }
                if (bad[k]) worst = GEP_WNOCONV;
                for (int64_t q = 0; q < r->m; ++q)
                    if (r->cid[q] == k) found.push_back({r->evals[q], r->resid[q], circle0 + k, r, (int)q});
            }
            circle0 += K;
            if (next.empty() && (int64_t)found.size() < m && covered < lmax * 1.5) {
                // extend the covered range by the density found so far
                const double width = covered - lower;
                double ext = found.empty() ? 2.0 * width
                                           : 1.25 * (double)(m - (int64_t)found.size()) * width / (double)found.size();
                ext = std::max(ext, 0.05 * width);
                const double b = std::min(covered + ext, lmax * 1.5);
                const double expect = found.empty() ? (double)m : (double)found.size() / width * (b - covered);
                const int Kn = std::max(1, (int)std::ceil(expect / per_contour));
                for (int k = 0; k < Kn; ++k)
                    next.push_back({covered + (b - covered) * k / Kn, covered + (b - covered) * (k + 1) / Kn, 0});
                covered = b;
                ++windows;
            }
            pending = next;
        }
        double lo = covered;
        std::stable_sort(found.begin(), found.end(), [](const Found& a, const Found& b) { return a.lam < b.lam; });
        const int64_t keep = std::min<int64_t>(m, (int64_t)found.size());
        auto* R = new gep_result();
        R->n = n;
        if (keep) {
            gep::PoolScope own(nullptr);
            R->dvecs = std::make_unique<gep::DBuf<double>>((size_t)n * keep);
        }
        bool noconv = false;
        for (int64_t a = 0; a < keep; ++a) {
            const Found& f = found[a];
            R->evals.push_back(f.lam);
            R->resid.push_back(f.rho);
            R->cid.push_back(f.cid);
            R->filt.push_back(f.col < (int)f.res->filt.size() ? f.res->filt[f.col] : 1.0);
            R->conv.push_back(f.rho <= tol ? 1 : 0);
            noconv |= !(f.rho <= tol);
            HIPCHK(hipMemcpy(R->dvecs->get() + a * n, f.res->dvecs->get() + (size_t)f.col * n, sizeof(double) * n,
                             hipMemcpyDeviceToDevice));
        }
        R->m = keep;
        std::ostringstream js;
        js << "{" << gep::boundary_stats(R->filt) << "\"rounds\":" << rounds.size() << ",\"windows\":" << windows
           << ",\"circles\":" << circle0
           << ",\"found\":" << found.size() << ",\"lmax_estimate\":" << lmax << ",\"window_hi\":" << lo
           << ",\"round_stats\":[";
        for (size_t i = 0; i < rounds.size(); ++i) js << (i ? "," : "") << rounds[i]->stats;
        js << "]}";
        R->stats = js.str();
        *out = R;
        if ((int64_t)found.size() < m) {
            gep::set_error("found only " + std::to_string(found.size()) + " of " + std::to_string(m) +
                           " eigenpairs below " + std::to_string(lo));
            return GEP_WNOCONV;
        }
        return noconv ? GEP_WNOCONV : worst;
    } catch (const gep::Fail& f) {
        return f.code;
    }
}

int gep_result_count(const gep_result* r, int64_t* m, int64_t* n) {
    if (!r) return GEP_EINVAL;
    if (m) *m = r->m;
    if (n) *n = r->n;
    return GEP_OK;
}

int gep_result_copy(const gep_result* r, double* evals, double* evecs, double* resid, int32_t* cid,
                    uint8_t* conv) {
    if (!r) return GEP_EINVAL;
    if (evals) std::copy(r->evals.begin(), r->evals.end(), evals);
    if (evecs && r->dvecs && r->dvecs->n) {
        hipError_t e = hipMemcpy(evecs, r->dvecs->get(), sizeof(double) * r->dvecs->n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            gep::set_error(std::string("eigenvector copy failed: ") + hipGetErrorString(e));
            return GEP_EDEVICE;
        }
    }
    if (resid) std::copy(r->resid.begin(), r->resid.end(), resid);
    if (cid) std::copy(r->cid.begin(), r->cid.end(), cid);
    if (conv) std::copy(r->conv.begin(), r->conv.end(), conv);
    return GEP_OK;
}

int gep_result_copy_evecs_device(const gep_result* r, double* evecs_dev, void* stream) {
    if (!r || (!evecs_dev && r->m > 0)) return GEP_EINVAL;
    if (!r->dvecs || !r->dvecs->n) return GEP_OK;
    hipError_t e = hipMemcpyAsync(evecs_dev, r->dvecs->get(), sizeof(double) * r->dvecs->n,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    r->copy_enqueued = true;
    if (e != hipSuccess) {
        gep::set_error(std::string("eigenvector copy failed: ") + hipGetErrorString(e));
        return GEP_EDEVICE;
    }
    return GEP_OK;
}

int gep_result_filter(const gep_result* r, double* filter) {
    if (!r || (!filter && r->m > 0)) return GEP_EINVAL;
    std::copy(r->filt.begin(), r->filt.end(), filter);
    return GEP_OK;
}

int gep_result_stats(const gep_result* r, char* json, size_t cap, size_t* needed) {
    if (!r) return GEP_EINVAL;
    if (needed) *needed = r->stats.size() + 1;
    if (json && cap > 0) {
        const size_t k = std::min(cap - 1, r->stats.size());
        std::memcpy(json, r->stats.data(), k);
        json[k] = 0;
    }
    return GEP_OK;
}

void gep_result_free(gep_result* r) {
    if (r && r->copy_enqueued) (void)hipDeviceSynchronize();   // the copy still reads dvecs
    delete r;
}

// ---- component entry points -------------------------------------------------
int gep_spmm_shifted(const gep_pencil* p, const double* shifts, const double* X, double* Y,
                     int64_t W, double* pq, void* stream) {
    if (!p || !shifts || !X || !Y || W <= 0 || W % gep::kTile) { gep::set_error("bad spmm arguments"); return GEP_EINVAL; }
    try {
        const int ntiles = (int)(W / gep::kTile);
        hipStream_t s = (hipStream_t)stream;
        gep::DBuf<int32_t> tiles(ntiles), cnt(1);
        std::vector<int32_t> tl(ntiles);
        for (int t = 0; t < ntiles; ++t) tl[t] = t;
        HIPCHK(hipMemcpyAsync(tiles.get(), tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(cnt.get(), &ntiles, sizeof(int32_t), hipMemcpyHostToDevice, s));
        int nrb = 0;
        gep::choose_nrb(p->d.n, ntiles, (int)std::max<int64_t>(1, std::min<int64_t>(1024, (p->d.n + 31) / 32)), nrb);
        gep::DBuf<double2> part;
        if (pq) part.alloc((size_t)ntiles * nrb * gep::kTile);
        HIPCHK(gep::launch_spmm_c64(p->d, (const double2*)shifts, (const double2*)X, (double2*)Y, tiles.get(),
                                    cnt.get(), ntiles, nrb, pq ? part.get() : nullptr, s));
        if (pq) {
            std::vector<double2> ph((size_t)ntiles * nrb * gep::kTile), out(W);
            HIPCHK(hipMemcpyAsync(ph.data(), part.get(), sizeof(double2) * ph.size(), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int t = 0; t < ntiles; ++t)
                for (int l = 0; l < gep::kTile; ++l) {
                    double2 a = make_double2(0, 0);
                    for (int rb = 0; rb < nrb; ++rb) {
                        const double2 v = ph[((size_t)t * nrb + rb) * gep::kTile + l];
                        a.x += v.x;
                        a.y += v.y;
                    }
                    out[(size_t)t * gep::kTile + l] = a;
                }
            HIPCHK(hipMemcpy(pq, out.data(), sizeof(double2) * W, hipMemcpyHostToDevice));
        }
        HIPCHK(hipStreamSynchronize(s));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_cocg_direction(const gep_pencil* p, const double* shifts, const double* beta,
                       const double* U, const double* P, double* Pn, int64_t W, double* pq,
                       int row_group, void* stream) {
    if (!p || !shifts || !beta || !U || !P || !Pn || !pq || W <= 0 || W % gep::kTile ||
        (row_group != 1 && row_group != 4)) {
        gep::set_error("bad cocg_direction arguments");
        return GEP_EINVAL;
    }
    try {
        const int ntiles = (int)(W / gep::kTile);
        const int64_t n = p->d.n;
        hipStream_t s = (hipStream_t)stream;
        const gep::DevPencil dv = gep::group_view(p->d, row_group);
        gep::CocgState S;
        S.n = n;
        S.ntiles = ntiles;
        S.u = (double2*)U;
        S.p = (double2*)P;
        S.pn = (double2*)Pn;
        S.shifts = (double2*)shifts;
        S.beta = (double2*)beta;
        S.rpb = dv.grp == 4 ? 4 * gep::kWaves : 2 * gep::kWaves;
        const int nrb = (int)((n + S.rpb - 1) / S.rpb);
        S.nrb = nrb;
        std::vector<int64_t> tb(ntiles);
        std::vector<int32_t> tn(ntiles, (int32_t)n), tr(ntiles, 0), tg(ntiles, dv.grp == 4 ? p->h.prob_g4[0] : 0),
            tl(ntiles);
        for (int t = 0; t < ntiles; ++t) {
            tb[t] = (int64_t)t * n * gep::kTile;
            tl[t] = t;
        }
        gep::DBuf<int64_t> dtb(ntiles);
        gep::DBuf<int32_t> dtn(ntiles), dtr(ntiles), dtg(ntiles), tiles(ntiles), cnt(2);
        gep::DBuf<double2> part((size_t)ntiles * nrb * gep::kTile);
        const int32_t counts[2] = {ntiles, (int32_t)W};
        HIPCHK(hipMemcpyAsync(dtb.get(), tb.data(), sizeof(int64_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dtn.get(), tn.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dtr.get(), tr.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dtg.get(), tg.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(tiles.get(), tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(cnt.get(), counts, sizeof(counts), hipMemcpyHostToDevice, s));
        S.geom.base = dtb.get();
        S.geom.n = dtn.get();
        S.geom.row0 = dtr.get();
        S.geom.g0 = dtg.get();
        S.tiles = tiles.get();
        S.counts = cnt.get();
        S.part_c = part.get();
        HIPCHK(gep::cocg_spmm_dir(dv, S, ntiles, nrb, s));
        std::vector<double2> ph((size_t)ntiles * nrb * gep::kTile), out(W);
        HIPCHK(hipMemcpyAsync(ph.data(), part.get(), sizeof(double2) * ph.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int t = 0; t < ntiles; ++t)
            for (int l = 0; l < gep::kTile; ++l) {
                double2 a = make_double2(0, 0);
                for (int rb = 0; rb < nrb; ++rb) {
                    const double2 v = ph[((size_t)t * nrb + rb) * gep::kTile + l];
                    a.x += v.x;
                    a.y += v.y;
                }
                out[(size_t)t * gep::kTile + l] = a;
            }
        HIPCHK(hipMemcpy(pq, out.data(), sizeof(double2) * W, hipMemcpyHostToDevice));
        HIPCHK(hipStreamSynchronize(s));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_spmm_shifted_f32(const gep_pencil* p, const double* shifts, const float* X, float* Y,
                         int64_t W, void* stream) {
    if (!p || !shifts || !X || !Y || W <= 0 || W % gep::kTile) { gep::set_error("bad spmm arguments"); return GEP_EINVAL; }
    try {
        const int ntiles = (int)(W / gep::kTile);
        hipStream_t s = (hipStream_t)stream;
        gep::DBuf<int32_t> tiles(ntiles), cnt(1);
        std::vector<int32_t> tl(ntiles);
        for (int t = 0; t < ntiles; ++t) tl[t] = t;
        HIPCHK(hipMemcpyAsync(tiles.get(), tl.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(cnt.get(), &ntiles, sizeof(int32_t), hipMemcpyHostToDevice, s));
        int nrb = 0;
        gep::choose_nrb(p->d.n, ntiles, (int)std::max<int64_t>(1, std::min<int64_t>(1024, (p->d.n + 31) / 32)), nrb);
        HIPCHK(gep::launch_spmm_c32(p->d, (const double2*)shifts, (const float2*)X, (float2*)Y, tiles.get(),
                                    cnt.get(), ntiles, nrb, nullptr, s));
        HIPCHK(hipStreamSynchronize(s));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_spmm_real(const gep_pencil* p, const double* X, int64_t k, int64_t ld, double* YA, double* YB,
                  void* stream) {
    if (!p || !X || k <= 0 || ld < k) { gep::set_error("bad spmm_real arguments"); return GEP_EINVAL; }
    try {
        HIPCHK(gep::launch_spmm_real(p->d, X, k, ld, YA, YB, (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_gram(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n, int64_t k1,
             int64_t k2, double* G, void* stream) {
    if (!X || !Y || !G || n < 0 || k1 <= 0 || k2 <= 0 || ld1 < k1 || ld2 < k2) { gep::set_error("bad gram arguments"); return GEP_EINVAL; }
    try {
        const size_t we = gep::gram_work_elems(n, k1, k2);
        gep::DBuf<double> w(std::max<size_t>(we, 1));
        HIPCHK(gep::launch_gram(X, ld1, Y, ld2, n, k1, k2, G, w.get(), w.n, (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_gram_noalloc(const double* X, int64_t ld1, const double* Y, int64_t ld2, int64_t n,
                     int64_t k1, int64_t k2, double* G, void* stream) {
    if (!X || !Y || !G || n < 0 || k1 <= 0 || k2 <= 0 || ld1 < k1 || ld2 < k2) { gep::set_error("bad gram arguments"); return GEP_EINVAL; }
    const size_t we = gep::gram_work_elems(n, k1, k2);
    if (we > gep::gram_scratch_elems()) {
        gep::set_error("gep_gram_noalloc: the split-K partials need " + std::to_string(we) +
                       " doubles, more than the " + std::to_string(gep::gram_scratch_elems()) +
                       " of the library's static scratch (use gep_gram)");
        return GEP_EINVAL;
    }
    try {
        double* work = nullptr;
        HIPCHK(gep::gram_scratch(&work));
        HIPCHK(gep::launch_gram(X, ld1, Y, ld2, n, k1, k2, G, work, gep::gram_scratch_elems(),
                                (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_gemm_tall(const double* X, int64_t ldx, const double* T, int64_t ldt, int64_t n, int64_t k,
                  int64_t m, double* C, int64_t ldc, void* stream) {
    if (!X || !T || !C || n < 0 || k <= 0 || m <= 0 || ldx < k || ldt < m || ldc < m) { gep::set_error("bad gemm arguments"); return GEP_EINVAL; }
    try {
        HIPCHK(gep::launch_gemm_tall(X, ldx, T, ldt, n, k, m, C, ldc, (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_sym_eig(double* A, double* w, double* V, int64_t k, int batch, void* stream) {
    if (!A || !w || !V || k <= 0 || k > 1024 || batch <= 0) { gep::set_error("bad sym_eig arguments"); return GEP_EINVAL; }
    try {
        gep::DBuf<double> work(gep::sym_eig_work_elems(k, batch));
        HIPCHK(gep::launch_sym_eig(A, w, V, k, batch, nullptr, work.get(), (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

int gep_gaussian_block(uint64_t seed, int64_t n, int64_t L, double* V, void* stream) {
    if (!V || n <= 0 || L <= 0) { gep::set_error("bad gaussian arguments"); return GEP_EINVAL; }
    try {
        HIPCHK(gep::launch_gaussian(seed, n, L, V, (hipStream_t)stream));
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    } catch (const gep::Fail& f) {
        return f.code;
    }
    return GEP_OK;
}

}  // extern "C"
