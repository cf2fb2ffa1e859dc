// bsde_host.cpp -- C ABI of libbsde.so: problem set-up (index set, grid,
// derivative channel matrices on the host; the Chebyshev basis matrix and
// its rank-checked pseudo-inverse R^{-1} Q' by CholeskyQR2 on the device),
// device buffers, the Picard loop that launches the HIP kernels, and the
// price/delta read-out.
//
// The method is Algorithm "algodetail" of Labart & Lelong (arXiv:1102.4666,
// Section 4.1); the least-squares extrapolating operator is that of
// Section 4.2 (eq. lspb) with polynomials centred and normalised to
// [-1, 1]^{d+1}; the model is Section 5 (eq. 4) with the correlation of
// Section 6.2.
#include "bsde_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <tuple>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace bsde {
bool kernel_exists(int d, int eta, int q10);
int index_table(int d, int eta, int q10, int8_t *nu, int cap);
// ev0/ev1 (may be null): start and end times of the path-kernel dispatch
hipError_t launch_path(int d, int eta, int q10, bool fp32, int blocks, hipStream_t s,
                       const PathParams &prm, const double *pts,
                       const void *gamma, double *partial,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_update(int n, int groups, int M, int ppg, int p, int nnz,
                         hipStream_t s, const double *partial, double *c,
                         double *var, const double *W, double *beta,
                         const double *alpha_in, double *alpha_out,
                         const int *rowptr, const int *cols, const double *vals,
                         double *g64, float *g32, hipEvent_t *ev);
hipError_t launch_channels(int p, int nnz, hipStream_t s, const double *alpha,
                           const int *rowptr, const int *cols, const double *vals,
                           double *g64, float *g32);
hipError_t launch_batch(int d, int eta, int q10, bool fp32, int vol, int blocks,
                        hipStream_t s, const BatchTileDesc *probs, int nprob,
                        const long long *tile_begin, unsigned int *counter);
int batch_occupancy(int d, int eta, int q10, bool fp32, int vol);
bool variant_exists(int d, int eta, int q10, bool fp32, int vol);
hipError_t launch_batch_update(int nprob, int max_n, int max_p, int max_cb,
                               hipStream_t s, const BatchUpdateDesc *d);
hipError_t launch_batch_channels(int nprob, int max_cb, hipStream_t s,
                                 const BatchUpdateDesc *d);
hipError_t launch_reset_counters(unsigned int *c, int n, hipStream_t s);
hipError_t launch_basis_matrix(const double *pts, int n, int ld, int dp,
                               const int8_t *nu, int pa, int pap,
                               const double *mid, const double *scale,
                               double T, double *B, hipStream_t s);
hipError_t launch_gram(const double *A, int ld, int pap, int rows_per_chunk,
                       int chunks, const int2 *pairs, int npairs,
                       double *partial, int pa, double *G, hipStream_t s);
hipError_t launch_gemm_ax(const double *A, int ld, const double *X, int pap,
                          double *Y, int ldy, int nrows, const int *colmap,
                          int ncols, hipStream_t s, const int *skip = nullptr);
hipError_t launch_small_factor(const double *G, int pa, int pap, double rel_tol,
                               int stage, double *X1, double *Xp, int *status,
                               hipStream_t s);
bool kernel_op_exists(int d, int vol);
hipError_t launch_kernel_path(int d, bool fp32, int blocks, hipStream_t s,
                              const PathParams &prm, const double *pts,
                              const void *table, double *partial,
                              hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_kernel_update(const PathParams &prm, int d, const double *pts,
                                const double *yprev, const double *c, double *ynew,
                                void *table, int fp32, hipStream_t s);
hipError_t launch_finalize(const double *partial, int n, int groups, int M,
                           int ppg, double *c, double *var, hipStream_t s);
} // namespace bsde

using namespace bsde;

static thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// Caching device allocator: buffers of released problems are kept per
// (device, size class) and handed to later problems, so that creating and
// destroying problems does not go through hipMalloc / hipFree each time.
// Size classes are powers of two from 256 bytes.  Thread-safe.
// ---------------------------------------------------------------------------
namespace {
struct DevicePool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_lists;
    std::map<void *, std::pair<int, size_t>> live;
    size_t cached_bytes = 0;
};
DevicePool &pool()
{
    static DevicePool *p = new DevicePool(); // never destroyed: buffers live
    return *p;                               // until the process ends
}
size_t size_class(size_t bytes)
{
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
}
hipError_t pool_alloc(void **ptr, size_t bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t cls = size_class(bytes);
    DevicePool &P = pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto &fl = P.free_lists[{dev, cls}];
        if (!fl.empty()) {
            *ptr = fl.back();
            fl.pop_back();
            P.cached_bytes -= cls;
            P.live[*ptr] = {dev, cls};
            return hipSuccess;
        }
    }
    e = hipMalloc(ptr, cls);
    if (e == hipErrorOutOfMemory) {
        // release the cache of this device and retry once
        std::lock_guard<std::mutex> g(P.mu);
        for (auto &kv : P.free_lists)
            if (kv.first.first == dev) {
                for (void *q : kv.second) (void)hipFree(q);
                P.cached_bytes -= kv.first.second * kv.second.size();
                kv.second.clear();
            }
        e = hipMalloc(ptr, cls);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(P.mu);
    P.live[*ptr] = {dev, cls};
    return hipSuccess;
}
void pool_free(void *ptr)
{
    if (!ptr) return;
    DevicePool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(ptr);
    if (it == P.live.end()) return;
    P.free_lists[it->second].push_back(ptr);
    P.cached_bytes += it->second.second;
    P.live.erase(it);
}

// HIP events are reused across solves for the kernel timings.
std::mutex g_ev_mu;
std::vector<hipEvent_t> g_events;
hipError_t event_get(hipEvent_t *e)
{
    {
        std::lock_guard<std::mutex> g(g_ev_mu);
        if (!g_events.empty()) {
            *e = g_events.back();
            g_events.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreate(e);
}
void event_put(hipEvent_t e)
{
    std::lock_guard<std::mutex> g(g_ev_mu);
    g_events.push_back(e);
}

// Side streams of a device for the parallel branches of a batched solve
// (default priority, non-blocking), with the events that fork them from and
// join them back to the caller's stream.  Created once per device; the
// batched solves of one device take turns on them.
struct SideStreams {
    static constexpr int kCount = 3; // with the caller's stream, four queues
    hipStream_t s[kCount] = {};
    hipEvent_t fork = nullptr, join[kCount] = {};
    std::mutex mu;
};
std::mutex g_side_mu;
std::map<int, SideStreams *> g_side;
hipError_t side_streams(SideStreams **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(g_side_mu);
    auto it = g_side.find(dev);
    if (it != g_side.end()) {
        *out = it->second;
        return hipSuccess;
    }
    auto *ss = new SideStreams(); // kept until the process ends
    for (int k = 0; k < SideStreams::kCount && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&ss->s[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ss->join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss->fork, hipEventDisableTiming);
    if (e != hipSuccess) return e; // (the partial set is not reused)
    g_side[dev] = ss;
    *out = ss;
    return hipSuccess;
}

// The instantiated graph of the last captured batched solve of a device,
// with the descriptor tables it reads and the launch plan it was captured
// from (a later batch with the same tables and plan replays it).
struct GraphCache {
    std::vector<char> blob;
    std::vector<long long> launches;
    char *dblob = nullptr;
    hipGraphExec_t exec = nullptr;
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        pool_free(dblob);
        dblob = nullptr;
        blob.clear();
        launches.clear();
    }
};
std::mutex g_graph_mu;
std::map<int, GraphCache> g_graph_cache;
} // namespace

bsde_status bsde::fail(bsde_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

// ---------------------------------------------------------------------------
// Set-up helpers
// ---------------------------------------------------------------------------
static bool cholesky(int d, double rho, double *L)
{
    for (int j = 0; j < kMaxD * kMaxD; ++j) L[j] = 0.0;
    for (int j = 0; j < d; ++j)
        for (int k = 0; k <= j; ++k) {
            double s = (j == k) ? 1.0 : rho;
            for (int l = 0; l < k; ++l) s -= L[j * kMaxD + l] * L[k * kMaxD + l];
            if (j == k) {
                if (!(s > 0.0)) return false;
                L[j * kMaxD + j] = std::sqrt(s);
            } else {
                L[j * kMaxD + k] = s / L[k * kMaxD + k];
            }
        }
    return true;
}

static double cheb_value(int a, double z)
{
    double t0 = 1.0, t1 = z;
    if (a == 0) return t0;
    for (int k = 1; k < a; ++k) {
        double t2 = 2.0 * z * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return t1;
}

// coefficient of T_b in the derivative of T_a
static double cheb_deriv_coef(int a, int b)
{
    if (b >= a || ((a - b) & 1) == 0) return 0.0;
    return b == 0 ? (double)a : 2.0 * a;
}

// Runs fn(begin, end) over [0, count) split across up to 16 host threads;
// work is the number of multiply-adds of the whole loop, and loops below
// 2^20 of them run in the calling thread.
template <typename F>
static void parallel_for(long count, long min_chunk, double work, F fn)
{
    const long hw = std::max(1u, std::thread::hardware_concurrency());
    long nt = std::max(1L, std::min({16L, hw, count / std::max(1L, min_chunk)}));
    if (work < (double)(1 << 20)) nt = 1;
    if (nt <= 1) {
        fn(0L, count);
        return;
    }
    std::vector<std::thread> th;
    const long per = (count + nt - 1) / nt;
    for (long t = 0; t < nt; ++t) {
        const long b = t * per, e = std::min(count, b + per);
        if (b < e) th.emplace_back(fn, b, e);
    }
    for (auto &x : th) x.join();
}

// q in tenths when a kernel of that hyperbolic set is built for (d, eta),
// else 10 (the total-degree kernel, used with a mask for q < 1)
static int kernel_q10(int d, int eta, double q)
{
    const double q10 = q * 10.0;
    const int r = (int)std::lround(q10);
    if (r >= 1 && r < 10 && std::fabs(q10 - r) < 1e-9 && kernel_exists(d, eta, r)) return r;
    return 10;
}

// Upper Cholesky factor R of a symmetric positive definite G (p x p,
// row-major): G = R'R.  Right-looking; false when a pivot is not positive
// or falls below rel_tol times the largest diagonal entry of R.
static bool chol_upper(const std::vector<double> &G, int p, double rel_tol,
                       std::vector<double> &R)
{
    R = G;
    double dmax = 0.0;
    for (int j = 0; j < p; ++j) dmax = std::max(dmax, G[(size_t)j * p + j]);
    dmax = std::sqrt(std::max(dmax, 0.0));
    for (int j = 0; j < p; ++j) {
        double *rj = &R[(size_t)j * p];
        const double piv = rj[j];
        if (!(piv > 0.0) || !(std::sqrt(piv) > rel_tol * dmax)) return false;
        const double r = std::sqrt(piv);
        for (int c = j; c < p; ++c) rj[c] /= r;
        // trailing update of the upper triangle, rows independent
        parallel_for(p - j - 1, 8, 0.5 * (double)(p - j) * (p - j),
                     [&, j, rj](long b, long e) {
            for (long rr = j + 1 + b; rr < j + 1 + e; ++rr) {
                double *row = &R[(size_t)rr * p];
                const double f = rj[rr];
                for (int c = (int)rr; c < p; ++c) row[c] -= f * rj[c];
            }
        });
    }
    for (int r = 1; r < p; ++r)
        for (int c = 0; c < r; ++c) R[(size_t)r * p + c] = 0.0;
    return true;
}

// Inverse of an upper triangular R (p x p, row-major), column by column
static std::vector<double> tri_inv_upper(const std::vector<double> &R, int p)
{
    std::vector<double> X((size_t)p * p, 0.0);
    parallel_for(p, 8, (double)p * p * p / 6, [&](long b, long e) {
        for (long c = b; c < e; ++c) {
            X[(size_t)c * p + c] = 1.0 / R[(size_t)c * p + c];
            for (long r = c - 1; r >= 0; --r) {
                double s = 0.0;
                for (long k = r + 1; k <= c; ++k) s += R[(size_t)r * p + k] * X[(size_t)k * p + c];
                X[(size_t)r * p + c] = -s / R[(size_t)r * p + r];
            }
        }
    });
    return X;
}

// Set-up streams (non-blocking, one per concurrent set-up, reused)
namespace {
std::mutex g_stream_mu;
std::map<int, std::vector<hipStream_t>> g_setup_streams;
hipError_t setup_stream_get(hipStream_t *s)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> g(g_stream_mu);
        auto &v = g_setup_streams[dev];
        if (!v.empty()) {
            *s = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}
void setup_stream_put(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_stream_mu);
    g_setup_streams[dev].push_back(s);
}
} // namespace

// The points of Picard iteration k.  Uniform kind: n points uniform over
// [0, T] x D.  Otherwise time-major (point i = a n_spatial + b):
// time nodes a T / (n_t - 1); tensor grid digits equispaced in [-1, 1]; or
// Philox-uniform spatial points from the counter (b, 0, k', 2 << 24 |
// block) with k' = k when the points are redrawn every iteration, else 0.
static void make_points(const bsde_problem_s *h, int k, std::vector<double> &pts)
{
    const int d = h->d, dp = d + 1;
    const long ns = h->n_spatial;
    const uint64_t seed = h->base.seed;
    const uint32_t kdraw = (h->redraw && h->grid_kind != BSDE_GRID_TENSOR) ? (uint32_t)k : 0u;
    pts.resize((size_t)h->n * dp);
    if (h->grid_kind == BSDE_GRID_UNIFORM) {
        // point i: word q of the counter (i, 0, k', 3 << 24 | q / 4) gives
        // t (q = 0) and x_j (q = 1 + j), uniform on [0, T] and [lo_j, hi_j]
        for (int i = 0; i < h->n; ++i) {
            double *row = &pts[(size_t)i * dp];
            for (int q = 0; q <= d; ++q) {
                u32x4 w = philox10((uint32_t)i, 0, kdraw, (3u << 24) | (uint32_t)(q / 4),
                                   (uint32_t)seed, (uint32_t)(seed >> 32));
                uint32_t word = q % 4 == 0 ? w.x : q % 4 == 1 ? w.y : q % 4 == 2 ? w.z : w.w;
                const double u = ((double)word + 0.5) * 0x1p-32;
                row[q] = q == 0 ? h->base.T * u : h->lo[q - 1] + u * (h->hi[q - 1] - h->lo[q - 1]);
            }
        }
        return;
    }
    for (int a = 0; a < h->n_t; ++a) {
        double t = a * h->base.T / (h->n_t - 1);
        for (long s = 0; s < ns; ++s) {
            double *row = &pts[(size_t)(a * ns + s) * dp];
            row[0] = t;
            long rest = s;
            for (int j = 0; j < d; ++j) {
                double z;
                if (h->grid_kind == BSDE_GRID_TENSOR) {
                    long digit = rest % h->n_x;
                    rest /= h->n_x;
                    z = h->n_x > 1 ? -1.0 + 2.0 * digit / (h->n_x - 1) : 0.0;
                } else {
                    u32x4 w = philox10((uint32_t)s, 0, kdraw, (2u << 24) | (uint32_t)(j / 4),
                                       (uint32_t)seed, (uint32_t)(seed >> 32));
                    uint32_t word = j % 4 == 0 ? w.x : j % 4 == 1 ? w.y : j % 4 == 2 ? w.z : w.w;
                    z = 2.0 * (((double)word + 0.5) * 0x1p-32) - 1.0;
                }
                row[1 + j] = h->lo[j] + 0.5 * (z + 1.0) * (h->hi[j] - h->lo[j]);
            }
        }
    }
}

// Shapes of the set-up: the leading dimension of the n x pap point matrices
// and the row chunks of the Gram kernel (about 2048 waves over the
// 64 x 64 block pairs, at least 256 rows each)
static void setup_shape(int n, int pap, int &ld, int &rpc, int &chunks)
{
    ld = (n + 63) & ~63;
    const int nb = (pap + 63) / 64;
    // about 2048 single-wave workgroups over the block pairs and chunks,
    // at least 64 rows a chunk (a chunk's loads are a dependent chain, so
    // small problems want many short chunks)
    const int want = std::max(1, 2048 / (nb * (nb + 1) / 2));
    rpc = std::max(64, ((ld + want - 1) / want + 15) & ~15);
    chunks = (ld + rpc - 1) / rpc;
}

// Pinned host staging buffers for uploads: size classes of powers of two,
// reused, held until the process ends (like the device pool).
namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void *> g_pin_free;
constexpr size_t kPinnedMax = size_t(16) << 20; // larger uploads stage in HIP
} // namespace
static void *pinned_get(size_t bytes, size_t *cap)
{
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    *cap = c;
    {
        std::lock_guard<std::mutex> g(g_pin_mu);
        auto it = g_pin_free.find(c);
        if (it != g_pin_free.end()) {
            void *p = it->second;
            g_pin_free.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}
static void pinned_put(void *p, size_t cap)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_free.emplace(cap, p);
}

// Pseudo-inverse W = B^+ (p x n, row-major; rows of inactive multi-indices
// zero) of the basis matrix of the grid by CholeskyQR2 on the device:
// B (n x pa) is formed from the device copy of the points, the Gram
// matrices and the tall-skinny products run on the device; the two pa x pa
// Cholesky factorisations and triangular inverses run on the device too
// when pa <= kSmallFactorP (one wave, LDS), else on the host.  Returns
// BSDE_ERANK when B is numerically rank deficient (a Cholesky pivot of B'B
// below 1e-7 of the largest, i.e. a condition number beyond ~1e7).
// Stream-ordered on s (the points must be uploaded on s or before); the
// call synchronizes s.
static bsde_status device_pseudo_inverse(bsde_problem_s *h, const std::vector<int> &act,
                                         hipStream_t s)
{
    const int n = h->n, pa = (int)act.size(), pap = pad16(pa), dp = h->d + 1;
    std::vector<int2> pairs;
    const int nb = (pap + 63) / 64;
    for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj) pairs.push_back(make_int2(bi, bj));
    int ld, rpc, chunks;
    setup_shape(n, pap, ld, rpc, chunks);
    std::vector<int8_t> nu_act((size_t)pa * dp);
    for (int c = 0; c < pa; ++c)
        std::memcpy(&nu_act[(size_t)c * dp], &h->nu[(size_t)act[c] * dp], dp);
    std::vector<double> ms(2 * kMaxD, 0.0);
    for (int j = 0; j < h->d; ++j) {
        ms[j] = h->base.mid[j];
        ms[kMaxD + j] = h->base.scale[j];
    }

    // the small inputs of the set-up kernels travel in one upload:
    // index set | domain map | Gram block pairs | active columns | status
    auto al8 = [](size_t b) { return (b + 7) & ~(size_t)7; };
    const size_t o_ms = al8(nu_act.size()), o_pairs = o_ms + sizeof(double) * ms.size(),
                 o_map = o_pairs + sizeof(int2) * pairs.size(),
                 o_status = al8(o_map + sizeof(int) * pa), n_small = o_status + 8;
    size_t pin_cap = 0;
    unsigned char *stage = (unsigned char *)pinned_get(n_small, &pin_cap);
    std::vector<unsigned char> stage_pageable;
    if (!stage) {
        stage_pageable.resize(n_small);
        stage = stage_pageable.data();
    }
    std::memset(stage, 0, n_small);
    std::memcpy(stage, nu_act.data(), nu_act.size());
    std::memcpy(stage + o_ms, ms.data(), sizeof(double) * ms.size());
    std::memcpy(stage + o_pairs, pairs.data(), sizeof(int2) * pairs.size());
    std::memcpy(stage + o_map, act.data(), sizeof(int) * pa);
    const bool small = pa <= kSmallFactorP;

    double *dB = nullptr, *dQ = nullptr, *dPart = nullptr, *dG = nullptr,
           *dX = nullptr, *dX1 = nullptr;
    unsigned char *dSmall = nullptr;
    bsde_status st = BSDE_OK;
    std::string why;
    auto chk = [&](hipError_t e, const char *what) {
        if (e == hipSuccess || st != BSDE_OK) return st == BSDE_OK;
        st = e == hipErrorOutOfMemory ? BSDE_ENOMEM : BSDE_EDEVICE;
        why = std::string(what) + ": " + hipGetErrorString(e);
        return false;
    };
    std::vector<double> G((size_t)pa * pa), R1, R2;
    do {
        if (!chk(pool_alloc((void **)&dB, sizeof(double) * ld * pap), "device allocation") ||
            !chk(pool_alloc((void **)&dQ, sizeof(double) * ld * pap), "device allocation") ||
            !chk(pool_alloc((void **)&dPart, sizeof(double) * chunks * pap * pap), "device allocation") ||
            !chk(pool_alloc((void **)&dG, sizeof(double) * pa * pa), "device allocation") ||
            !chk(pool_alloc((void **)&dX, sizeof(double) * pap * pap), "device allocation") ||
            !chk(pool_alloc((void **)&dSmall, n_small), "device allocation") ||
            (small && !chk(pool_alloc((void **)&dX1, sizeof(double) * pa * pa), "device allocation")))
            break;
        if (!chk(hipMemcpyAsync(dSmall, stage, n_small, hipMemcpyHostToDevice, s), "upload"))
            break;
        const int8_t *dNu = (const int8_t *)dSmall;
        const double *dMS = (const double *)(dSmall + o_ms);
        const int2 *dPairs = (const int2 *)(dSmall + o_pairs);
        const int *dMap = (const int *)(dSmall + o_map);
        int *dStatus = (int *)(dSmall + o_status);
        if (small) {
            // CholeskyQR2 with the p x p steps on the device: stream-ordered,
            // one synchronisation (the status) at the end; the last product
            // leaves W untouched when a rank test failed
            int status = 0;
            if (!chk(launch_basis_matrix(h->d_pts, n, ld, dp, dNu, pa, pap, dMS, dMS + kMaxD,
                                         h->base.T, dB, s), "basis kernel") ||
                !chk(launch_gram(dB, ld, pap, rpc, chunks, dPairs, (int)pairs.size(), dPart, pa,
                                 dG, s), "gram kernel") ||
                !chk(launch_small_factor(dG, pa, pap, 1e-7, 1, dX1, dX, dStatus, s),
                     "factor kernel") ||
                !chk(launch_gemm_ax(dB, ld, dX, pap, dQ, ld, ld, nullptr, pap, s, dStatus),
                     "gemm kernel") ||
                !chk(launch_gram(dQ, ld, pap, rpc, chunks, dPairs, (int)pairs.size(), dPart, pa,
                                 dG, s), "gram kernel") ||
                !chk(launch_small_factor(dG, pa, pap, 1e-3, 2, dX1, dX, dStatus, s),
                     "factor kernel"))
                break;
            if (pa < h->p &&
                !chk(hipMemsetAsync(h->d_W, 0, sizeof(double) * (size_t)h->p * n, s), "memset"))
                break;
            if (!chk(launch_gemm_ax(dQ, ld, dX, pap, h->d_W, n, n, dMap, pa, s, dStatus),
                     "gemm kernel") ||
                !chk(hipMemcpyAsync(&status, dStatus, sizeof(int), hipMemcpyDeviceToHost, s),
                     "download") ||
                !chk(hipStreamSynchronize(s), "set-up"))
                break;
            if (status != 0) {
                st = BSDE_ERANK;
                why = "basis matrix is numerically rank deficient on the grid";
            }
            break;
        }
        // B and G1 = B'B
        if (!chk(launch_basis_matrix(h->d_pts, n, ld, dp, dNu, pa, pap, dMS, dMS + kMaxD,
                                     h->base.T, dB, s), "basis kernel") ||
            !chk(launch_gram(dB, ld, pap, rpc, chunks, dPairs, (int)pairs.size(), dPart, pa, dG, s),
                 "gram kernel") ||
            !chk(hipMemcpyAsync(G.data(), dG, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s),
                 "download") ||
            !chk(hipStreamSynchronize(s), "set-up"))
            break;
        if (!chol_upper(G, pa, 1e-7, R1)) {
            st = BSDE_ERANK;
            why = "basis matrix is numerically rank deficient on the grid";
            break;
        }
        // Q1 = B R1^{-1} (all pap columns: the padding comes out zero)
        const std::vector<double> X1 = tri_inv_upper(R1, pa);
        std::vector<double> Xp((size_t)pap * pap, 0.0);
        for (int r = 0; r < pa; ++r)
            std::memcpy(&Xp[(size_t)r * pap], &X1[(size_t)r * pa], sizeof(double) * pa);
        if (!chk(hipMemcpyAsync(dX, Xp.data(), sizeof(double) * Xp.size(), hipMemcpyHostToDevice, s),
                 "upload") ||
            !chk(launch_gemm_ax(dB, ld, dX, pap, dQ, ld, ld, nullptr, pap, s), "gemm kernel") ||
            !chk(launch_gram(dQ, ld, pap, rpc, chunks, dPairs, (int)pairs.size(), dPart, pa, dG, s),
                 "gram kernel") ||
            !chk(hipMemcpyAsync(G.data(), dG, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s),
                 "download") ||
            !chk(hipStreamSynchronize(s), "set-up"))
            break;
        if (!chol_upper(G, pa, 1e-3, R2)) {
            st = BSDE_ERANK;
            why = "basis matrix is numerically rank deficient on the grid";
            break;
        }
        // B^+' = Q1 P with P = R2^{-1} R2^{-T} R1^{-T}
        const std::vector<double> Y2 = tri_inv_upper(R2, pa);
        std::vector<double> T2((size_t)pa * pa, 0.0); // R2^{-1} R2^{-T}
        parallel_for(pa, 8, (double)pa * pa * pa / 3, [&](long b, long e) {
            for (long r = b; r < e; ++r)
                for (int c = 0; c < pa; ++c) {
                    double v = 0.0;
                    for (int k = (int)std::max<long>(r, c); k < pa; ++k)
                        v += Y2[(size_t)r * pa + k] * Y2[(size_t)c * pa + k];
                    T2[(size_t)r * pa + c] = v;
                }
        });
        std::fill(Xp.begin(), Xp.end(), 0.0);
        parallel_for(pa, 8, (double)pa * pa * pa / 2, [&](long b, long e) {
            for (long r = b; r < e; ++r)
                for (int c = 0; c < pa; ++c) {
                    double v = 0.0; // sum_k T2[r][k] X1[c][k], X1 upper
                    for (int k = c; k < pa; ++k) v += T2[(size_t)r * pa + k] * X1[(size_t)c * pa + k];
                    Xp[(size_t)r * pap + c] = v;
                }
        });
        if (pa < h->p &&
            !chk(hipMemsetAsync(h->d_W, 0, sizeof(double) * (size_t)h->p * n, s), "memset"))
            break;
        if (!chk(hipMemcpyAsync(dX, Xp.data(), sizeof(double) * Xp.size(), hipMemcpyHostToDevice, s),
                 "upload") ||
            !chk(launch_gemm_ax(dQ, ld, dX, pap, h->d_W, n, n, dMap, pa, s), "gemm kernel") ||
            !chk(hipStreamSynchronize(s), "set-up"))
            break;
    } while (false);
    if (st != BSDE_OK) (void)hipStreamSynchronize(s);
    if (stage_pageable.empty()) pinned_put(stage, pin_cap);
    for (void *q : {(void *)dB, (void *)dQ, (void *)dPart, (void *)dG, (void *)dX,
                    (void *)dX1, (void *)dSmall})
        pool_free(q);
    if (st != BSDE_OK) return fail(st, why);
    return BSDE_OK;
}

// the channel tables: dense, then the live rows packed (bsde_common.h)
static size_t table_floats(const bsde_problem_s *h)
{
    if (h->kop) return 0; // the kernel operator reads its point table instead
    return (size_t)h->n_live;
}

static void free_device(bsde_problem_s *h)
{
    pool_free(h->d_block);
    pool_free(h->d_W);
    pool_free(h->d_beta);
    pool_free(h->d_partial);
    pool_free(h->d_c);
    pool_free(h->d_var);
    h->d_pts = h->d_W = h->d_vals = h->d_alpha = h->d_beta = h->d_g64 = nullptr;
    h->d_partial = h->d_c = h->d_var = nullptr;
    h->d_g32 = nullptr;
    h->d_rowptr = h->d_cols = nullptr;
    h->d_block = nullptr;
}



#define HIP_TRY(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(BSDE_EDEVICE, std::string(#expr) + ": " +              \
                                          hipGetErrorString(e_));              \
    } while (0)

// Tilings chosen by bsde_autotune, keyed by kernel signature and size
// class; consulted when a problem is created.
namespace {
struct TuneKey {
    int d, eta, q10, prec, vol, M, N, nclass;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(d, eta, q10, prec, vol, M, N, nclass) <
               std::tie(o.d, o.eta, o.q10, o.prec, o.vol, o.M, o.N, o.nclass);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tuned;

TuneKey tune_key(const bsde_problem_s *h)
{
    int nclass = 0;
    while ((1 << nclass) < h->n) ++nclass;
    return {h->d, h->eta, h->q10, h->precision, h->base.vol_kind, h->M, h->N, nclass};
}
} // namespace

static void auto_tiling(const bsde_problem_s *h, int &groups, int &ppl)
{
    // fill the GPU with >= ~2048 workgroups; lanes run whole paths
    int max_groups = (h->M + kBlock - 1) / kBlock;
    int want = (2048 + h->n - 1) / h->n;
    groups = std::max(1, std::min(max_groups, want));
    ppl = (h->M + groups * kBlock - 1) / (groups * kBlock);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *bsde_status_string(bsde_status s)
{
    switch (s) {
    case BSDE_OK: return "ok";
    case BSDE_EINVAL: return "invalid argument";
    case BSDE_ENOMEM: return "out of memory";
    case BSDE_ERANK: return "rank-deficient least-squares problem";
    case BSDE_EDEVICE: return "HIP device error";
    case BSDE_ESTATE: return "invalid state";
    case BSDE_EUNSUPPORTED: return "no kernel for this (d, eta)";
    case BSDE_EBUSY: return "request not finished";
    }
    return "unknown status";
}

const char *bsde_last_error(void) { return g_last_error.c_str(); }

} // extern "C"

static bsde_status prepare_tiling(bsde_problem h, int &groups, int &ppl,
                                  bool allow_alloc = true);

extern "C" {

bsde_status bsde_create_problem(int d, const bsde_sigma *sigma, double r,
                                const bsde_payoff *payoff,
                                const bsde_grid *grid, int M, int N,
                                int n_picard, double penalty,
                                unsigned long long seed, int precision,
                                bsde_problem *out)
{
    if (out) *out = nullptr;
    if (!out || !sigma || !payoff || !grid || !sigma->level || !payoff->S0)
        return fail(BSDE_EINVAL, "null argument");
    if (d < 1 || d > kMaxD) return fail(BSDE_EINVAL, "d must be in [1, 10]");
    if (M < 1 || N < 1 || n_picard < 1)
        return fail(BSDE_EINVAL, "M, N and n_picard must be >= 1");
    if (!(penalty >= 0.0) || !std::isfinite(r))
        return fail(BSDE_EINVAL, "penalty must be >= 0 and r finite");
    if (!(payoff->T > 0.0) || payoff->kind < 0 || payoff->kind > 5)
        return fail(BSDE_EINVAL, "bad payoff");
    if (sigma->kind != BSDE_VOL_CONST && sigma->kind != BSDE_VOL_BUMP &&
        sigma->kind != BSDE_VOL_DUPIRE)
        return fail(BSDE_EINVAL, "bad volatility kind");
    if (sigma->kind == BSDE_VOL_BUMP && !(sigma->bump_c > 0.0))
        return fail(BSDE_EINVAL, "bump centre must be > 0");
    if (grid->kind != BSDE_GRID_TENSOR && grid->kind != BSDE_GRID_RANDOM &&
        grid->kind != BSDE_GRID_UNIFORM)
        return fail(BSDE_EINVAL, "bad grid kind");
    if (grid->redraw != 0 && (grid->redraw != 1 || grid->kind == BSDE_GRID_TENSOR))
        return fail(BSDE_EINVAL, "redraw needs random or uniform points");
    if ((grid->kind != BSDE_GRID_UNIFORM && grid->n_t < 2) || grid->n_x < 1 ||
        !(grid->width > 0.0) ||
        grid->eta < 1 || !(grid->q > 0.0 && grid->q <= 1.0))
        return fail(BSDE_EINVAL, "bad grid (n_t >= 2, n_x >= 1, width > 0, "
                                 "eta >= 1, 0 < q <= 1)");
    if (precision != BSDE_FP64 && precision != BSDE_FP32_PATHS)
        return fail(BSDE_EINVAL, "bad precision");
    for (int j = 0; j < d; ++j)
        if (!(sigma->level[j] > 0.0) || !(payoff->S0[j] > 0.0))
            return fail(BSDE_EINVAL, "levels and spots must be > 0");
    // the kernel operator of Section 3.2 instead of least squares
    const bool kop = grid->kernel_bw != 0.0;
    if (kop) {
        if (!(grid->kernel_bw > 0.0) || !std::isfinite(grid->kernel_bw))
            return fail(BSDE_EINVAL, "kernel_bw must be 0 or a finite bandwidth > 0");
        if (grid->redraw)
            return fail(BSDE_EUNSUPPORTED, "the kernel operator takes fixed points");
        if (!kernel_op_exists(d, sigma->kind))
            return fail(BSDE_EUNSUPPORTED, "the kernel operator is built for d <= 2 "
                                           "with constant or bump volatility");
    }
    // a kernel of the hyperbolic set itself when one is built, else the
    // total-degree kernel with the entries outside the set kept at zero
    const int q10 = kernel_q10(d, grid->eta, grid->q);
    if (kop) {
        // no basis: eta and q are not used
    } else if (!kernel_exists(d, grid->eta, q10))
        return fail(BSDE_EUNSUPPORTED, "no kernel instantiated for d=" +
                                           std::to_string(d) + ", eta=" +
                                           std::to_string(grid->eta));
    if (!kop && !variant_exists(d, grid->eta, q10, precision == BSDE_FP32_PATHS, sigma->kind))
        return fail(BSDE_EUNSUPPORTED,
                    "no kernel instantiated for d=" + std::to_string(d) + ", eta=" +
                        std::to_string(grid->eta) + " with this precision and "
                        "volatility kind (d = 10: FP64 paths for total degree "
                        "only; the Dupire-type volatility: d=1 eta=4, d=2 "
                        "eta=3, d=5 eta=2,3)");
    double Lc[kMaxD * kMaxD];
    if (!cholesky(d, sigma->rho, Lc))
        return fail(BSDE_EINVAL, "correlation matrix not positive definite");

    auto *h = new (std::nothrow) bsde_problem_s();
    if (!h) return fail(BSDE_ENOMEM, "host allocation");
    h->d = d;
    h->eta = grid->eta;
    h->q = grid->q;
    h->M = M;
    h->N = N;
    h->K_it = n_picard;
    h->omega = penalty;
    h->precision = precision;
    PathParams &b = h->base;
    b.seed = seed;
    b.M = M;
    b.N = N;
    b.vol_kind = sigma->kind;
    b.payoff = payoff->kind;
    b.r = r;
    b.omega = penalty;
    b.K = payoff->K;
    b.T = payoff->T;
    b.bump_a = sigma->kind == BSDE_VOL_BUMP ? sigma->bump_a : 0.0;
    b.log_bump_c = sigma->kind == BSDE_VOL_BUMP ? std::log(sigma->bump_c) : 0.0;
    b.rho = sigma->rho;
    std::memcpy(b.L, Lc, sizeof(Lc));
    h->lo.resize(d);
    h->hi.resize(d);
    for (int j = 0; j < d; ++j) {
        b.level[j] = sigma->level[j];
        b.spot[j] = payoff->S0[j];
        b.div[j] = sigma->dividend ? sigma->dividend[j] : 0.0;
        double half = grid->width * sigma->level[j] * std::sqrt(payoff->T);
        h->lo[j] = std::log(payoff->S0[j]) - half;
        h->hi[j] = std::log(payoff->S0[j]) + half;
        b.mid[j] = 0.5 * (h->lo[j] + h->hi[j]);
        b.scale[j] = 2.0 / (h->hi[j] - h->lo[j]);
    }
    fill_asset_consts(b, d);
    h->kop = kop;
    b.kbw = kop ? grid->kernel_bw : 0.0;

    // index set in kernel order; hyperbolic subset marked active (a
    // one-function placeholder for the kernel operator)
    const int dp = d + 1;
    h->q10 = q10;
    h->p = kop ? 1 : index_table(d, grid->eta, q10, nullptr, 0);
    h->nu.assign((size_t)h->p * dp, 0);
    if (!kop) index_table(d, grid->eta, q10, h->nu.data(), h->p);
    h->active.assign(h->p, 1);
    if (!kop && grid->q < 1.0) {
        for (int l = 0; l < h->p; ++l) {
            double s = 0.0;
            for (int v = 0; v < dp; ++v)
                if (h->nu[(size_t)l * dp + v]) s += std::pow((double)h->nu[(size_t)l * dp + v], grid->q);
            h->active[l] = s <= std::pow((double)grid->eta, grid->q) * (1.0 + 1e-12);
        }
    }
    h->C = num_channels(d);

    // grid points (time-major)
    long ns = 1;
    if (grid->kind == BSDE_GRID_TENSOR) {
        for (int j = 0; j < d; ++j) {
            ns *= grid->n_x;
            if (ns > (1L << 26)) {
                delete h;
                return fail(BSDE_EINVAL, "tensor grid too large");
            }
        }
    } else {
        ns = grid->n_x;
    }
    // uniform points: n_x of them, no time nodes
    const int n_t = grid->kind == BSDE_GRID_UNIFORM ? 1 : grid->n_t;
    if ((long)ns * n_t > (1L << 26)) {
        delete h;
        return fail(BSDE_EINVAL, "too many points");
    }
    h->n_spatial = (int)ns;
    h->n = (int)(ns * n_t);
    h->grid_kind = grid->kind;
    h->n_t = n_t;
    h->n_x = grid->n_x;
    h->redraw = grid->redraw;
    h->pts_k = 0;
    make_points(h, 0, h->pts);

    // basis matrix over the active multi-indices and its pseudo-inverse
    std::vector<int> &act = h->act;
    for (int l = 0; l < h->p; ++l)
        if (h->active[l]) act.push_back(l);
    const int pa = (int)act.size();
    if (h->n < pa) {
        delete h;
        return fail(BSDE_ERANK, "fewer points than basis functions");
    }

    // The derivative channels as sparse rows over the basis: the derivative
    // of T_a in one variate is a combination of the T_b, b < a, a - b odd
    // (cheb_deriv_coef), so row mu of d/dz_v holds the functions mu + k e_v of
    // the set, k odd; rows columns ascending.  Channel 1 is d_t (2/T d/dz_0),
    // channel 2 + j d_{x_j} (scale_j d/dz_{1+j}), then the second
    // derivatives, the products of two of those.
    std::map<std::vector<int8_t>, int> pos;
    for (int l = 0; l < h->p; ++l)
        pos[std::vector<int8_t>(&h->nu[(size_t)l * dp], &h->nu[(size_t)l * dp] + dp)] = l;
    using SRow = std::vector<std::pair<int, double>>;
    std::vector<std::vector<SRow>> Dv(dp, std::vector<SRow>(h->p));
    for (int v = 0; v < dp && !kop; ++v) {
        for (int l = 0; l < h->p; ++l) {
            std::vector<int8_t> e(&h->nu[(size_t)l * dp], &h->nu[(size_t)l * dp] + dp);
            const int a = e[v];
            for (int bb = 0; bb < a; ++bb) {
                const double cf = cheb_deriv_coef(a, bb);
                if (cf == 0.0) continue;
                std::vector<int8_t> mu = e;
                mu[v] = (int8_t)bb;
                Dv[v][pos[mu]].push_back({l, cf});
            }
        }
        for (auto &r : Dv[v]) std::sort(r.begin(), r.end());
    }
    const double tfac = 2.0 / payoff->T;
    h->Dx.assign(kop ? 0 : d, std::vector<SRow>(h->p));
    for (int j = 0; j < d && !kop; ++j)
        for (int l = 0; l < h->p; ++l)
            for (const auto &x : Dv[1 + j][l]) h->Dx[j][l].push_back({x.first, b.scale[j] * x.second});
    // the packed channel table (bsde_common.h) as a sparse matrix over the
    // coefficients, in the order the path kernels read it: channel 0; each
    // second derivative over its live rows; then row by row the time
    // derivative and the gradient.  The kernel's index set is the set of
    // rows here.
    std::vector<int> csr_ptr(1, 0), csr_col;
    std::vector<double> csr_val;
    if (!kop) {
        auto in_set = [&](const int *mu) {
            std::vector<int8_t> key(dp);
            for (int v = 0; v < dp; ++v) key[v] = (int8_t)mu[v];
            return pos.count(key) > 0;
        };
        auto live = [&](int l, int c) {
            return channel_row_live<kMaxD + 1>(&h->nu[(size_t)l * dp], dp, c, in_set);
        };
        auto put = [&](const SRow &r, double f) {
            for (const auto &x : r) {
                csr_col.push_back(x.first);
                csr_val.push_back(f * x.second);
            }
            csr_ptr.push_back((int)csr_col.size());
        };
        for (int l = 0; l < h->p; ++l) put(SRow{{l, 1.0}}, 1.0);
        for (int c = 2 + d; c < h->C; ++c) {
            const int j = hess_j(d, c - 2 - d), k = hess_k(d, c - 2 - d);
            for (int l = 0; l < h->p; ++l) {
                if (!live(l, c)) continue;
                // row l of (d/dx_j)(d/dx_k): sum over the middle function mm,
                // in ascending order
                std::map<int, double> acc;
                for (const auto &x1 : h->Dx[j][l])
                    for (const auto &x2 : h->Dx[k][x1.first]) acc[x2.first] += x1.second * x2.second;
                put(SRow(acc.begin(), acc.end()), 1.0);
            }
        }
        for (int l = 0; l < h->p; ++l)
            for (int c = 1; c < 2 + d; ++c)
                if (live(l, c)) put(Dv[c - 1][l], c == 1 ? tfac : b.scale[c - 2]);
        h->n_live = (int)csr_ptr.size() - 1;
    }

    if (kop) {
        // the coefficients of a kernel-operator problem are its point values
        h->p = h->n;
    }

    // device buffers
    hipError_t alloc_err = hipSuccess;
    auto dalloc = [&](void **ptr, size_t bytes) {
        alloc_err = pool_alloc(ptr, bytes == 0 ? 8 : bytes);
        return alloc_err == hipSuccess;
    };
    // points, channel matrices, coefficients and channel tables in one
    // block (256-byte aligned parts)
    auto al256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t real_size = precision == BSDE_FP32_PATHS ? sizeof(float) : sizeof(double);
    const size_t b_pts = sizeof(double) * h->pts.size(),
                 b_val = sizeof(double) * csr_val.size(),
                 b_alpha = sizeof(double) * (size_t)(h->K_it + 1) * h->p,
                 b_g64 = sizeof(double) * table_floats(h),
                 b_g32 = sizeof(float) * table_floats(h),
                 b_ptr = kop ? 0 : sizeof(int) * csr_ptr.size(),
                 b_col = sizeof(int) * csr_col.size(),
                 b_ktab = kop ? real_size * kKernelRow * (size_t)h->n : 0;
    const size_t o_val = al256(b_pts), o_alpha = o_val + al256(b_val),
                 o_g64 = o_alpha + al256(b_alpha), o_g32 = o_g64 + al256(b_g64),
                 o_ptr = o_g32 + al256(b_g32), o_col = o_ptr + al256(b_ptr),
                 o_ktab = o_col + al256(b_col), n_block = o_ktab + al256(b_ktab);
    bool ok = dalloc(&h->d_block, n_block) &&
              (kop || dalloc((void **)&h->d_W, sizeof(double) * (size_t)h->p * h->n)) &&
              dalloc((void **)&h->d_beta, sizeof(double) * h->p) &&
              dalloc((void **)&h->d_c, sizeof(double) * (size_t)h->K_it * h->n) &&
              dalloc((void **)&h->d_var, sizeof(double) * (size_t)h->K_it * h->n);
    if (!ok) {
        free_device(h);
        delete h;
        if (alloc_err == hipErrorOutOfMemory)
            return fail(BSDE_ENOMEM, "device allocation failed");
        return fail(BSDE_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(alloc_err));
    }
    {
        char *b = (char *)h->d_block;
        h->d_pts = (double *)b;
        h->d_vals = (double *)(b + o_val);
        h->d_alpha = (double *)(b + o_alpha);
        h->d_g64 = (double *)(b + o_g64);
        h->d_g32 = (float *)(b + o_g32);
        h->d_rowptr = b_ptr ? (int *)(b + o_ptr) : nullptr;
        h->d_cols = b_ptr ? (int *)(b + o_col) : nullptr;
        h->d_ktab = kop ? (void *)(b + o_ktab) : nullptr;
    }
    // the kernel operator's table: rows {z_0, .., z_d, y = 0} in the path
    // precision, z the mapped coordinates of the points
    std::vector<unsigned char> ktab(b_ktab, 0);
    for (int i = 0; kop && i < h->n; ++i) {
        double z[kKernelRow] = {0, 0, 0, 0};
        z[0] = 2.0 * h->pts[(size_t)i * dp] / payoff->T - 1.0;
        for (int j = 0; j < d; ++j)
            z[1 + j] = (h->pts[(size_t)i * dp + 1 + j] - b.mid[j]) * b.scale[j];
        for (int v = 0; v < kKernelRow; ++v) {
            if (real_size == sizeof(float)) {
                const float f = (float)z[v];
                std::memcpy(&ktab[((size_t)i * kKernelRow + v) * real_size], &f, sizeof(f));
            } else {
                std::memcpy(&ktab[((size_t)i * kKernelRow + v) * real_size], &z[v], sizeof(double));
            }
        }
    }
    // uploads and the set-up kernels go to a set-up stream of the library
    // (non-blocking: a problem created while another one solves does not
    // wait for it).  The block goes up in one copy from pinned staging
    // memory: points, the channel update's sparse rows and zeros for the
    // starting coefficients and the channel tables.
    hipStream_t us = nullptr;
    size_t pin_cap = 0;
    void *pin = n_block <= kPinnedMax ? pinned_get(n_block, &pin_cap) : nullptr;
    hipError_t e = setup_stream_get(&us);
    if (e == hipSuccess && pin) {
        std::memset(pin, 0, n_block);
        std::memcpy(pin, h->pts.data(), b_pts);
        if (b_val) std::memcpy((char *)pin + o_val, csr_val.data(), b_val);
        if (b_ptr) std::memcpy((char *)pin + o_ptr, csr_ptr.data(), b_ptr);
        if (b_col) std::memcpy((char *)pin + o_col, csr_col.data(), b_col);
        if (b_ktab) std::memcpy((char *)pin + o_ktab, ktab.data(), b_ktab);
        e = hipMemcpyAsync(h->d_block, pin, n_block, hipMemcpyHostToDevice, us);
    } else if (e == hipSuccess) {
        e = hipMemcpyAsync(h->d_pts, h->pts.data(), b_pts, hipMemcpyHostToDevice, us);
        if (e == hipSuccess && b_val)
            e = hipMemcpyAsync(h->d_vals, csr_val.data(), b_val, hipMemcpyHostToDevice, us);
        if (e == hipSuccess)
            e = hipMemsetAsync((char *)h->d_block + o_alpha, 0, o_ptr - o_alpha, us);
        if (e == hipSuccess && b_ptr)
            e = hipMemcpyAsync(h->d_rowptr, csr_ptr.data(), b_ptr, hipMemcpyHostToDevice, us);
        if (e == hipSuccess && b_col)
            e = hipMemcpyAsync(h->d_cols, csr_col.data(), b_col, hipMemcpyHostToDevice, us);
        if (e == hipSuccess && b_ktab)
            e = hipMemcpyAsync(h->d_ktab, ktab.data(), b_ktab, hipMemcpyHostToDevice, us);
    }
    if (e != hipSuccess) {
        if (us) {
            (void)hipStreamSynchronize(us);
            setup_stream_put(us);
        }
        pinned_put(pin, pin_cap);
        free_device(h);
        delete h;
        return fail(BSDE_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    // pseudo-inverse of the basis matrix of the grid, on the device (it
    // synchronizes the set-up stream: the sparse rows and the points may go
    // out of scope)
    // (the kernel operator fits nothing: only the upload to wait for)
    bsde_status pst = BSDE_OK;
    if (!kop) {
        pst = device_pseudo_inverse(h, act, us);
    } else {
        const hipError_t se = hipStreamSynchronize(us);
        if (se != hipSuccess)
            pst = fail(BSDE_EDEVICE, std::string("upload: ") + hipGetErrorString(se));
    }
    setup_stream_put(us);
    pinned_put(pin, pin_cap);
    if (pst != BSDE_OK) {
        free_device(h);
        delete h;
        return pst; // the last error is already recorded
    }
    h->alpha_hist.assign((size_t)(h->K_it + 1) * h->p, 0.0);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(tune_key(h));
        if (it != g_tuned.end()) {
            h->groups = it->second.first;
            h->ppl = it->second.second;
        }
    }
    // the per-group sum buffer of the tiling the problem starts with, so
    // that solving it allocates nothing more
    int groups0, ppl0;
    const bsde_status tst = prepare_tiling(h, groups0, ppl0);
    if (tst != BSDE_OK) {
        free_device(h);
        delete h;
        return tst;
    }
    *out = h;
    return BSDE_OK;
}

bsde_status bsde_set_tiling(bsde_problem h, int groups_per_point,
                            int paths_per_lane)
{
    if (!h || groups_per_point < 0 || paths_per_lane < 0)
        return fail(BSDE_EINVAL, "bad tiling");
    if ((groups_per_point == 0) != (paths_per_lane == 0))
        return fail(BSDE_EINVAL, "set both tiling values or neither");
    if (groups_per_point > 0 &&
        (long)groups_per_point * paths_per_lane * kBlock < h->M)
        return fail(BSDE_EINVAL, "tiling covers fewer than M paths");
    h->groups = groups_per_point;
    h->ppl = paths_per_lane;
    return BSDE_OK;
}

// Tiling of a solve and the per-group sum buffer it needs (grown from the
// pool unless allow_alloc is false: then a buffer too small is an error).
static bsde_status prepare_tiling(bsde_problem h, int &groups, int &ppl,
                                  bool allow_alloc)
{
    groups = h->groups;
    ppl = h->ppl;
    if (groups == 0) auto_tiling(h, groups, ppl);
    const size_t need = (size_t)h->n * groups * 2;
    if (need > h->partial_cap) {
        if (!allow_alloc)
            return fail(BSDE_ESTATE, "the problem's tiling needs a larger per-group sum "
                                     "buffer than it was created with (solve it once with "
                                     "an allocating entry point first)");
        pool_free(h->d_partial);
        h->d_partial = nullptr;
        h->partial_cap = 0;
        HIP_TRY(pool_alloc((void **)&h->d_partial, sizeof(double) * need));
        h->partial_cap = need;
    }
    return BSDE_OK;
}

// the Monte Carlo path kernel of h's operator (least squares: the channel
// table; kernel operator: the point table)
static hipError_t launch_problem_path(const bsde_problem_s *h, int blocks, hipStream_t s,
                                      const PathParams &prm, hipEvent_t ev0, hipEvent_t ev1)
{
    const bool fp32 = h->precision == BSDE_FP32_PATHS;
    if (h->kop)
        return launch_kernel_path(h->d, fp32, blocks, s, prm, h->d_pts, h->d_ktab,
                                  h->d_partial, ev0, ev1);
    return launch_path(h->d, h->eta, h->q10, fp32, blocks, s, prm, h->d_pts,
                       fp32 ? (const void *)h->d_g32 : (const void *)h->d_g64,
                       h->d_partial, ev0, ev1);
}

bsde_status bsde_solve(bsde_problem h, void *hip_stream)
{
    if (!h) return fail(BSDE_EINVAL, "null handle");
    hipStream_t s = (hipStream_t)hip_stream;
    int groups, ppl;
    bsde_status st = prepare_tiling(h, groups, ppl);
    if (st != BSDE_OK) return st;
    const bool fp32 = h->precision == BSDE_FP32_PATHS;
    const int iters = h->K_it - h->k_done;
    // events: start, end, and per iteration (timing level 1) the start and
    // end of the path-kernel dispatch (taken by the dispatch itself, no
    // marker packets), (level 2) also after the reduction, the projection
    // and the channel update
    const int lvl = h->timing;
    const int per = lvl >= 2 ? 5 : (lvl == 1 ? 2 : 0);
    std::vector<hipEvent_t> ev(2 + (size_t)per * iters);
    for (auto &x : ev) HIP_TRY(event_get(&x));
    struct Release {
        std::vector<hipEvent_t> &v;
        ~Release() { for (auto &x : v) event_put(x); }
    } release_events{ev};
    double t_setup = 0.0;
    HIP_TRY(hipEventRecord(ev[0], s));
    // channel table of the starting coefficients (the kernel operator's
    // table already holds the current point values)
    if (!h->kop)
        HIP_TRY(launch_channels(h->p, h->n_live, s, h->d_alpha + (size_t)h->k_done * h->p,
                                h->d_rowptr, h->d_cols, h->d_vals, h->d_g64, h->d_g32));
    for (int it = 0; it < iters; ++it) {
        const int k = h->k_done + it;
        hipEvent_t *e = per ? &ev[2 + (size_t)per * it] : nullptr;
        if (h->redraw && h->pts_k != k) {
            // Algorithm 1: new points for this iteration, and the
            // pseudo-inverse of their basis matrix (after the previous
            // iteration is done with the old ones)
            HIP_TRY(hipStreamSynchronize(s));
            const auto t0 = std::chrono::steady_clock::now();
            make_points(h, k, h->pts);
            HIP_TRY(hipMemcpyAsync(h->d_pts, h->pts.data(), sizeof(double) * h->pts.size(),
                                   hipMemcpyHostToDevice, s));
            const bsde_status pst = device_pseudo_inverse(h, h->act, s);
            if (pst != BSDE_OK) return pst;
            h->pts_k = k;
            t_setup += std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
        }
        PathParams prm = h->base;
        prm.k = (uint32_t)k;
        prm.groups = groups;
        prm.paths_per_lane = ppl;
        prm.n = h->n;
        HIP_TRY(launch_problem_path(h, h->n * groups, s, prm, e ? e[0] : nullptr,
                                    e ? e[1] : nullptr));
        if (h->kop) {
            // c^k, then y^k = u^k(points) + c^k with u^k = h[y^{k-1}]
            // (alpha row k; row 0 = 0 is u^0 = 0) into row k + 1 and the table
            double *ck = h->d_c + (size_t)k * h->n;
            HIP_TRY(launch_finalize(h->d_partial, h->n, groups, h->M, kBlock * ppl, ck,
                                    h->d_var + (size_t)k * h->n, s));
            if (per == 5) HIP_TRY(hipEventRecord(e[2], s));
            HIP_TRY(launch_kernel_update(prm, h->d, h->d_pts,
                                         k ? h->d_alpha + (size_t)k * h->p : nullptr, ck,
                                         h->d_alpha + (size_t)(k + 1) * h->p, h->d_ktab,
                                         fp32 ? 1 : 0, s));
            if (per == 5) {
                HIP_TRY(hipEventRecord(e[3], s));
                HIP_TRY(hipEventRecord(e[4], s));
            }
            continue;
        }
        HIP_TRY(launch_update(h->n, groups, h->M, kBlock * ppl, h->p, h->n_live, s,
                              h->d_partial, h->d_c + (size_t)k * h->n,
                              h->d_var + (size_t)k * h->n, h->d_W, h->d_beta,
                              h->d_alpha + (size_t)k * h->p,
                              h->d_alpha + (size_t)(k + 1) * h->p, h->d_rowptr, h->d_cols,
                              h->d_vals, h->d_g64, h->d_g32,
                              per == 5 ? e + 2 : nullptr)); // records e[2..4] // records e[2..4]
    }
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipEventSynchronize(ev[1]));
    double t_path = 0, t_fin = 0, t_proj = 0, t_chan = 0;
    for (int it = 0; it < iters && per; ++it) {
        hipEvent_t *e = &ev[2 + (size_t)per * it];
        float ms;
        hipEventElapsedTime(&ms, e[0], e[1]); t_path += ms;
        if (per == 5) {
            hipEventElapsedTime(&ms, e[1], e[2]); t_fin += ms;
            hipEventElapsedTime(&ms, e[2], e[3]); t_proj += ms;
            hipEventElapsedTime(&ms, e[3], e[4]); t_chan += ms;
        } else {
            // the rest of the iteration: up to the next path kernel (or
            // the end of the solve)
            hipEvent_t next = it + 1 < iters ? ev[2 + (size_t)per * (it + 1)] : ev[1];
            hipEventElapsedTime(&ms, e[1], next); t_fin += ms;
        }
    }
    float tot;
    hipEventElapsedTime(&tot, ev[0], ev[1]);
    (void)t_setup; // included in the total (host-side set-up between launches)
    HIP_TRY(hipMemcpyAsync(h->alpha_hist.data(), h->d_alpha,
                           sizeof(double) * h->alpha_hist.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (iters > 0) {
        h->timings[0] = t_path / iters;
        h->timings[1] = t_fin / iters;
        h->timings[2] = t_proj / iters;
        h->timings[3] = t_chan / iters;
        h->timings[4] = tot;
    }
    h->k_done = h->K_it;
    h->have_alpha = true;
    return BSDE_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Batched solve: all remaining iterations of many problems.  Per iteration
// step and kernel signature (d, eta, precision, volatility kind) one
// persistent launch drains the tiles of every active problem of that
// signature; one launch each then reduces, projects and updates all active
// problems.  With BSDE_BATCH_GRAPH the whole schedule is captured once as a
// hipGraph and replayed.
// ---------------------------------------------------------------------------
namespace {
struct Sig {
    int d, eta, q10;
    bool fp32;
    int vol;
    bool operator<(const Sig &o) const
    {
        return std::tie(d, eta, q10, fp32, vol) < std::tie(o.d, o.eta, o.q10, o.fp32, o.vol);
    }
};

int num_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                  dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

BatchUpdateDesc update_desc(bsde_problem h, int k, int groups, int ppl, bool advance)
{
    BatchUpdateDesc u{};
    u.partial = h->d_partial;
    u.n = h->n;
    u.groups = groups;
    u.ppg = kBlock * ppl;
    u.M = h->M;
    u.p = h->p;
    u.nnz = h->n_live;
    u.c = h->d_c + (size_t)std::min(k, h->K_it - 1) * h->n;
    u.var = h->d_var + (size_t)std::min(k, h->K_it - 1) * h->n;
    u.W = h->d_W;
    u.beta = h->d_beta;
    u.alpha_in = h->d_alpha + (size_t)k * h->p;
    u.alpha_out = advance ? h->d_alpha + (size_t)(k + 1) * h->p : nullptr;
    u.rowptr = h->d_rowptr;
    u.cols = h->d_cols;
    u.vals = h->d_vals;
    u.g64 = h->d_g64;
    u.g32 = h->d_g32;
    return u;
}
} // namespace

// Runs `steps` iterations (at most the remaining ones) of every problem.
// Copies the coefficient histories back when copy_back is set.
bsde_status bsde::run_batch(bsde_problem *probs, int count, hipStream_t s,
                            int steps, bool graph, bool copy_back, double *ms,
                            const int *steps_each, void *workspace,
                            size_t workspace_bytes, bool parallel_branches,
                            int cu_reserve)
{
    std::vector<int> G(count), PPL(count), R(count);
    int S = 0;
    for (int q = 0; q < count; ++q) {
        bsde_status st = prepare_tiling(probs[q], G[q], PPL[q], workspace == nullptr);
        if (st != BSDE_OK) return st;
        // iterations problem q runs in this call
        R[q] = std::max(0, std::min(steps_each ? steps_each[q] : steps,
                                    probs[q]->K_it - probs[q]->k_done));
        S = std::max(S, R[q]);
    }
    std::map<Sig, std::vector<int>> sigs;
    for (int q = 0; q < count; ++q) {
        bsde_problem h = probs[q];
        sigs[{h->d, h->eta, h->q10, h->precision == BSDE_FP32_PATHS,
              h->base.vol_kind}].push_back(q);
    }
    // host-side descriptor tables, laid out in one byte buffer
    std::vector<char> blob;
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (blob.size() + 255) & ~(size_t)255;
        blob.resize(off + bytes);
        std::memcpy(blob.data() + off, src, bytes);
        return off;
    };
    struct PathLaunch { Sig sig; size_t desc_off, begin_off; int nprob; long long tiles; int counter; };
    struct StepPlan { std::vector<PathLaunch> paths; size_t upd_off; int nact, max_n, max_p, max_cb; };
    std::vector<StepPlan> plan(S);
    int n_counters = 0;
    int max_cb_all = 0; // workgroups of the channel update (256 entries each)
    for (int step = 0; step < S; ++step) {
        std::vector<BatchUpdateDesc> upd;
        int max_n = 0, max_p = 0, max_cb = 0;
        for (auto &kv : sigs) {
            std::vector<int> act;
            for (int q : kv.second)
                if (step < R[q]) act.push_back(q);
            if (act.empty()) continue;
            // heaviest tiles first (paths per lane x Euler steps)
            std::stable_sort(act.begin(), act.end(), [&](int a, int b) {
                return (long long)PPL[a] * probs[a]->N > (long long)PPL[b] * probs[b]->N;
            });
            std::vector<BatchTileDesc> td;
            std::vector<long long> begin(1, 0);
            for (int q : act) {
                bsde_problem h = probs[q];
                BatchTileDesc t{};
                t.prm = h->base;
                t.prm.k = (uint32_t)(h->k_done + step);
                t.prm.groups = G[q];
                t.prm.paths_per_lane = PPL[q];
                t.prm.n = h->n;
                t.pts = h->d_pts;
                t.gamma = kv.first.fp32 ? (const void *)h->d_g32 : (const void *)h->d_g64;
                t.partial = h->d_partial;
                td.push_back(t);
                begin.push_back(begin.back() + (long long)h->n * G[q]);
                upd.push_back(update_desc(h, h->k_done + step, G[q], PPL[q], true));
                max_n = std::max(max_n, h->n);
                max_p = std::max(max_p, h->p);
                max_cb = std::max(max_cb, (h->n_live + 255) / 256);
            }
            PathLaunch pl{kv.first, put(td.data(), sizeof(BatchTileDesc) * td.size()),
                          put(begin.data(), sizeof(long long) * begin.size()),
                          (int)act.size(), begin.back(), n_counters++};
            plan[step].paths.push_back(pl);
        }
        plan[step].upd_off = put(upd.data(), sizeof(BatchUpdateDesc) * upd.size());
        plan[step].nact = (int)upd.size();
        plan[step].max_n = max_n;
        plan[step].max_p = max_p;
        plan[step].max_cb = max_cb;
        max_cb_all = std::max(max_cb_all, max_cb);
    }
    std::vector<BatchUpdateDesc> init;
    for (int q = 0; q < count; ++q) {
        init.push_back(update_desc(probs[q], probs[q]->k_done, G[q], PPL[q], false));
        max_cb_all = std::max(max_cb_all, (probs[q]->n_live + 255) / 256);
    }
    const size_t init_off = put(init.data(), sizeof(BatchUpdateDesc) * init.size());
    const size_t ctr_off = (blob.size() + 255) & ~(size_t)255;
    blob.resize(ctr_off + sizeof(unsigned int) * std::max(1, n_counters), 0);

    // the descriptor tables and tile counters: from the pool, or in the
    // caller's workspace
    char *dblob = nullptr;
    if (workspace) {
        if (blob.size() > workspace_bytes)
            return fail(BSDE_EINVAL, "the batch's descriptor tables need " +
                                         std::to_string(blob.size()) +
                                         " bytes, more than the workspace of " +
                                         std::to_string(workspace_bytes));
        dblob = (char *)workspace;
    } else {
        HIP_TRY(pool_alloc((void **)&dblob, blob.size()));
    }
    struct Release {
        char *p;
        ~Release() { pool_free(p); }
    } release{workspace ? nullptr : dblob};
    HIP_TRY(hipMemcpyAsync(dblob, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
    unsigned int *counters = (unsigned int *)(dblob + ctr_off);

    // Launches of different kernel signatures in one step run as parallel
    // branches: the first on s, the others on the library's side streams of
    // this device (forked from s and joined back before the step's update),
    // so that the tiles of one signature fill the tail of another's launch.
    // The no-allocation form (and a caller that asks) keeps everything on s.
    const bool parallel = workspace == nullptr && parallel_branches;
    SideStreams *side = nullptr;
    std::unique_lock<std::mutex> side_lock; // held until the batch is done
    if (parallel) {
        bool fork_any = false;
        for (int step = 0; step < S; ++step) fork_any |= plan[step].paths.size() > 1;
        if (fork_any) {
            HIP_TRY(side_streams(&side));
            side_lock = std::unique_lock<std::mutex>(side->mu);
        }
    }
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = launch_reset_counters(counters, std::max(1, n_counters), s);
        if (e != hipSuccess) return e;
        e = launch_batch_channels(count, max_cb_all, s,
                                  (const BatchUpdateDesc *)(dblob + init_off));
        if (e != hipSuccess) return e;
        for (int step = 0; step < S; ++step) {
            const int nl = (int)plan[step].paths.size();
            const int nside = side ? std::min(nl - 1, SideStreams::kCount) : 0;
            if (nside > 0) {
                e = hipEventRecord(side->fork, s);
                for (int k = 0; k < nside && e == hipSuccess; ++k)
                    e = hipStreamWaitEvent(side->s[k], side->fork, 0);
                if (e != hipSuccess) return e;
            }
            for (int j = 0; j < nl; ++j) {
                const PathLaunch &pl = plan[step].paths[j];
                hipStream_t ls = (j == 0 || nside == 0) ? s : side->s[(j - 1) % nside];
                const int occ = std::max(1, batch_occupancy(pl.sig.d, pl.sig.eta, pl.sig.q10,
                                                            pl.sig.fp32, pl.sig.vol));
                const long long cap = (long long)occ * std::max(1, num_cus() - cu_reserve);
                const int blocks = (int)std::max(1LL, std::min(pl.tiles, cap));
                e = launch_batch(pl.sig.d, pl.sig.eta, pl.sig.q10, pl.sig.fp32, pl.sig.vol, blocks, ls,
                                 (const BatchTileDesc *)(dblob + pl.desc_off), pl.nprob,
                                 (const long long *)(dblob + pl.begin_off),
                                 counters + pl.counter);
                if (e != hipSuccess) return e;
            }
            for (int k = 0; k < nside; ++k) {
                e = hipEventRecord(side->join[k], side->s[k]);
                if (e == hipSuccess) e = hipStreamWaitEvent(s, side->join[k], 0);
                if (e != hipSuccess) return e;
            }
            e = launch_batch_update(plan[step].nact, plan[step].max_n, plan[step].max_p,
                                    plan[step].max_cb, s,
                                    (const BatchUpdateDesc *)(dblob + plan[step].upd_off));
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };

    // timing events only when the time is asked for
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        HIP_TRY(event_get(&e0));
        HIP_TRY(event_get(&e1));
        HIP_TRY(hipEventRecord(e0, s));
    }
    if (graph) {
        // The instantiated graph of the last captured batch on this device
        // is kept with its descriptor tables; a batch whose tables and
        // launch plan are byte for byte the same (the same problems, from
        // the same iteration) replays it instead of capturing again.  The
        // tables hold every address and parameter the kernels read, so
        // equal tables mean the same work.
        std::vector<long long> launches;
        for (int step = 0; step < S; ++step) {
            for (const PathLaunch &pl : plan[step].paths)
                launches.insert(launches.end(), {pl.sig.d, pl.sig.eta, pl.sig.q10, pl.sig.fp32,
                                                 pl.sig.vol, (long long)pl.desc_off,
                                                 (long long)pl.begin_off, pl.nprob, pl.tiles,
                                                 pl.counter});
            launches.insert(launches.end(), {-1, (long long)plan[step].upd_off, plan[step].nact,
                                             plan[step].max_n, plan[step].max_p,
                                             plan[step].max_cb});
        }
        launches.insert(launches.end(), {count, max_cb_all, (long long)init_off, n_counters,
                                         (long long)(side != nullptr)});
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        std::lock_guard<std::mutex> gl(g_graph_mu);
        GraphCache &gc = g_graph_cache[dev];
        const bool hit = gc.exec && gc.blob == blob && gc.launches == launches;
        if (!hit) {
            gc.release();
            // the cached graph owns its descriptor tables: move them out of
            // this call's release
            gc.dblob = dblob;
            release.p = nullptr;
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t le = enqueue();
            hipError_t ce = hipStreamEndCapture(s, &g);
            if (le != hipSuccess || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                gc.release();
                return fail(BSDE_EDEVICE, std::string("graph capture: ") +
                                              hipGetErrorString(le != hipSuccess ? le : ce));
            }
            hipError_t ie = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                gc.exec = nullptr;
                gc.release();
                return fail(BSDE_EDEVICE, std::string("graph instantiate: ") +
                                              hipGetErrorString(ie));
            }
            gc.blob = blob;
            gc.launches = launches;
        }
        hipError_t ie = hipGraphLaunch(gc.exec, s);
        if (ie == hipSuccess) ie = hipStreamSynchronize(s);
        if (ie != hipSuccess) {
            gc.release();
            return fail(BSDE_EDEVICE, std::string("graph launch: ") + hipGetErrorString(ie));
        }
    } else {
        HIP_TRY(enqueue());
    }
    if (ms) {
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        event_put(e0);
        event_put(e1);
        *ms = t;
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    for (int q = 0; q < count; ++q) {
        bsde_problem h = probs[q];
        h->k_done += R[q];
        h->have_alpha = true;
        if (copy_back) {
            HIP_TRY(hipMemcpyAsync(h->alpha_hist.data(), h->d_alpha,
                                   sizeof(double) * h->alpha_hist.size(),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    return BSDE_OK;
}

bsde_status bsde::fetch_coefficients(bsde_problem h)
{
    HIP_TRY(hipMemcpy(h->alpha_hist.data(), h->d_alpha,
                      sizeof(double) * h->alpha_hist.size(), hipMemcpyDeviceToHost));
    return BSDE_OK;
}

size_t bsde::problem_device_bytes(int d, const bsde_grid *grid, int M, int K_it)
{
    if (d < 1 || d > kMaxD || !grid) return 0;
    const int p = index_table(d, grid->eta, kernel_q10(d, grid->eta, grid->q), nullptr, 0);
    if (p == 0) return 0;
    size_t ns = 1;
    if (grid->kind == BSDE_GRID_TENSOR)
        for (int j = 0; j < d; ++j) ns *= (size_t)grid->n_x;
    else
        ns = (size_t)grid->n_x;
    const size_t n = ns * (size_t)(grid->kind == BSDE_GRID_UNIFORM ? 1 : grid->n_t);
    const size_t C = (size_t)num_channels(d);
    bsde_problem_s tmp;
    tmp.n = (int)n;
    tmp.M = M;
    int groups, ppl;
    auto_tiling(&tmp, groups, ppl);
    // the block of points, the channel update's sparse rows, coefficients
    // and tables (one allocation, 256-byte aligned parts), then the separate
    // buffers; at most p C table entries, each row of the update at most 16
    // non-zeros (a row of a mixed second derivative has one per pair of odd
    // degree steps k1 + k2 <= eta: 10 at eta = 8, the most of any set built)
    auto al256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t entries = table_entries(p, (int)C), nonzeros = 16 * entries;
    const size_t block = al256(n * (d + 1) * 8) + al256(nonzeros * 8) +
                         al256((size_t)(K_it + 1) * p * 8) + al256(entries * 8) +
                         al256(entries * 4) + al256((entries + 1) * 4) +
                         al256(nonzeros * 4);
    const size_t sizes[] = {block, (size_t)p * n * 8, (size_t)p * 8,
                            (size_t)K_it * n * 8,
                            (size_t)K_it * n * 8,
                            n * groups * 16};
    size_t total = 0;
    for (size_t b : sizes) total += size_class(b == 0 ? 8 : b);
    // transient set-up buffers: two point matrices and the Gram partials
    int ld, rpc, chunks;
    setup_shape((int)n, pad16(p), ld, rpc, chunks);
    total += 2 * size_class((size_t)ld * pad16(p) * 8) +
             size_class((size_t)chunks * pad16(p) * pad16(p) * 8);
    return total;
}

extern "C" {

bsde_status bsde_solve_batch(bsde_problem *problems, int count,
                                        void *hip_stream, int flags, double *ms)
{
    if (!problems || count < 1) return fail(BSDE_EINVAL, "no problems");
    for (int q = 0; q < count; ++q) {
        if (!problems[q]) return fail(BSDE_EINVAL, "null handle in batch");
        for (int r = 0; r < q; ++r)
            if (problems[r] == problems[q]) return fail(BSDE_EINVAL, "duplicate handle in batch");
        if (problems[q]->redraw)
            return fail(BSDE_EUNSUPPORTED, "points redrawn every iteration: use bsde_solve");
        if (problems[q]->kop)
            return fail(BSDE_EUNSUPPORTED, "the kernel operator: use bsde_solve");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    hipStream_t own = nullptr;
    const bool graph = (flags & BSDE_BATCH_GRAPH) != 0;
    if (graph && !s) { // capture needs a stream other than the null stream
        HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        s = own;
    }
    bsde_status st = run_batch(problems, count, s, 1 << 30, graph, true, ms);
    if (own) (void)hipStreamDestroy(own);
    return st;
}

} // extern "C"

// ---------------------------------------------------------------------------
// The no-allocation batched solve.  Its descriptor tables and tile counters
// live in this fixed array, one copy per device, held until the process
// ends.  In host code the array's name is not a device address: the
// address of the current device's copy comes from hipGetSymbolAddress on
// the first call on that device and is used everywhere after.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = size_t(4) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;            // one call per device at a time
std::map<int, void *> g_scratch;    // device -> address of its copy
} // namespace

extern "C" {

bsde_status bsde_solve_batch_noalloc(bsde_problem *problems, int count,
                                     void *hip_stream)
{
    if (!problems || count < 1) return fail(BSDE_EINVAL, "no problems");
    for (int q = 0; q < count; ++q) {
        if (!problems[q]) return fail(BSDE_EINVAL, "null handle in batch");
        for (int r = 0; r < q; ++r)
            if (problems[r] == problems[q]) return fail(BSDE_EINVAL, "duplicate handle in batch");
        if (problems[q]->redraw)
            return fail(BSDE_EUNSUPPORTED, "points redrawn every iteration: use bsde_solve");
        if (problems[q]->kop)
            return fail(BSDE_EUNSUPPORTED, "the kernel operator: use bsde_solve");
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(BSDE_EDEVICE, std::string("workspace address: ") + hipGetErrorString(e));
        it = g_scratch.emplace(dev, ptr).first;
    }
    return run_batch(problems, count, (hipStream_t)hip_stream, 1 << 30, false, true,
                     nullptr, nullptr, it->second, kNoAllocBytes);
}

bsde_status bsde_autotune(bsde_problem h, void *hip_stream, int *groups_out,
                          int *ppl_out, double *ms_out)
{
    if (!h) return fail(BSDE_EINVAL, "null handle");
    hipStream_t s = (hipStream_t)hip_stream;
    // candidates: paths per lane in powers of two, groups to cover M
    std::vector<std::pair<int, int>> cand;
    for (int ppl = 1; ppl <= 64; ppl *= 2) {
        const int groups = (h->M + kBlock * ppl - 1) / (kBlock * ppl);
        if (groups < 1) continue;
        if (!cand.empty() && cand.back().first == groups) continue;
        cand.push_back({groups, ppl});
        if (groups == 1) break;
    }
    size_t need = 0;
    for (auto &c : cand) need = std::max(need, (size_t)h->n * c.first * 2);
    if (need > h->partial_cap) {
        pool_free(h->d_partial);
        h->d_partial = nullptr;
        h->partial_cap = 0;
        HIP_TRY(pool_alloc((void **)&h->d_partial, sizeof(double) * need));
        h->partial_cap = need;
    }
    const int k = std::min(h->k_done, h->K_it - 1);
    if (!h->kop)
        HIP_TRY(launch_channels(h->p, h->n_live, s, h->d_alpha + (size_t)h->k_done * h->p,
                                h->d_rowptr, h->d_cols, h->d_vals, h->d_g64, h->d_g32));
    hipEvent_t e0, e1;
    HIP_TRY(event_get(&e0));
    HIP_TRY(event_get(&e1));
    double best = 1e300;
    std::pair<int, int> pick = cand.front();
    for (auto &c : cand) {
        PathParams prm = h->base;
        prm.k = (uint32_t)k;
        prm.groups = c.first;
        prm.paths_per_lane = c.second;
        prm.n = h->n;
        double t_min = 1e300;
        for (int rep = 0; rep < 5; ++rep) { // first launch warms up
            HIP_TRY(launch_problem_path(h, h->n * c.first, s, prm, e0, e1));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) t_min = std::min(t_min, (double)ms);
        }
        // a later candidate (fewer workgroups per point) must win by more
        // than timing noise, so that repeated tunings agree
        if (t_min < 0.98 * best) {
            best = t_min;
            pick = c;
        }
    }
    event_put(e0);
    event_put(e1);
    h->groups = pick.first;
    h->ppl = pick.second;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[tune_key(h)] = pick;
    }
    if (groups_out) *groups_out = pick.first;
    if (ppl_out) *ppl_out = pick.second;
    if (ms_out) *ms_out = best;
    return BSDE_OK;
}

// Architecture name of the current device ("gfx950"), the key under which
// recorded tilings are saved: a tiling measured on one architecture says
// nothing about another.
static bsde_status device_arch(std::string &arch)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    if (arch.empty()) return fail(BSDE_EDEVICE, "device reports no architecture name");
    return BSDE_OK;
}

bsde_status bsde_autotune_save(const char *path, int *count)
{
    if (!path) return fail(BSDE_EINVAL, "null path");
    std::string arch;
    const bsde_status st = device_arch(arch);
    if (st != BSDE_OK) return st;
    std::vector<std::pair<TuneKey, std::pair<int, int>>> rows;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        rows.assign(g_tuned.begin(), g_tuned.end());
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(BSDE_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "# bsde path tilings: arch d eta q10 precision vol M N size_class "
                    "groups_per_point paths_per_lane\n");
    for (const auto &r : rows) {
        const TuneKey &k = r.first;
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d\n", arch.c_str(), k.d, k.eta,
                     k.q10, k.prec, k.vol, k.M, k.N, k.nclass, r.second.first,
                     r.second.second);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) return fail(BSDE_EINVAL, std::string("cannot write ") + path);
    if (count) *count = (int)rows.size();
    return BSDE_OK;
}

bsde_status bsde_autotune_load(const char *path, int *count)
{
    if (!path) return fail(BSDE_EINVAL, "null path");
    std::string arch;
    const bsde_status st = device_arch(arch);
    if (st != BSDE_OK) return st;
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(BSDE_EINVAL, std::string("cannot read ") + path);
    // parse every line first: a malformed file changes nothing
    std::vector<std::pair<TuneKey, std::pair<int, int>>> rows;
    char line[512];
    int lineno = 0;
    bool bad = false;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        const char *q = line;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '#' || *q == '\n' || *q == '\0') continue;
        char a[64];
        TuneKey k;
        int groups = 0, ppl = 0;
        if (std::sscanf(q, "%63s %d %d %d %d %d %d %d %d %d %d", a, &k.d, &k.eta, &k.q10,
                        &k.prec, &k.vol, &k.M, &k.N, &k.nclass, &groups, &ppl) != 11 ||
            groups < 1 || ppl < 1 || k.M < 1 ||
            (long long)groups * ppl * kBlock < (long long)k.M) {
            bad = true;
            break;
        }
        if (arch == a) rows.push_back({k, {groups, ppl}});
    }
    std::fclose(f);
    if (bad)
        return fail(BSDE_EINVAL, std::string(path) + ": malformed tiling record on line " +
                                     std::to_string(lineno));
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        for (const auto &r : rows) g_tuned[r.first] = r.second;
    }
    if (count) *count = (int)rows.size();
    return BSDE_OK;
}

bsde_status bsde_get_tiling(bsde_problem h, int *groups_per_point, int *paths_per_lane)
{
    if (!h || !groups_per_point || !paths_per_lane) return fail(BSDE_EINVAL, "null argument");
    *groups_per_point = h->groups;
    *paths_per_lane = h->ppl;
    return BSDE_OK;
}

bsde_status bsde_set_timing(bsde_problem h, int level)
{
    if (!h) return fail(BSDE_EINVAL, "null handle");
    if (level < 0 || level > 2) return fail(BSDE_EINVAL, "timing level must be 0, 1 or 2");
    h->timing = level;
    return BSDE_OK;
}

bsde_status bsde_last_timings(bsde_problem h, double *ms5)
{
    if (!h || !ms5) return fail(BSDE_EINVAL, "null argument");
    for (int i = 0; i < 5; ++i) ms5[i] = h->timings[i];
    return BSDE_OK;
}

bsde_status bsde_problem_sizes(bsde_problem h, int *n, int *p, int *C)
{
    if (!h) return fail(BSDE_EINVAL, "null handle");
    if (n) *n = h->n;
    if (p) *p = h->p;
    if (C) *C = h->C;
    return BSDE_OK;
}

bsde_status bsde_get_points(bsde_problem h, double *pts)
{
    if (!h || !pts) return fail(BSDE_EINVAL, "null argument");
    std::memcpy(pts, h->pts.data(), sizeof(double) * h->pts.size());
    return BSDE_OK;
}

bsde_status bsde_get_coefficients(bsde_problem h, int k, double *alpha,
                                  int *k_done)
{
    if (!h || !alpha) return fail(BSDE_EINVAL, "null argument");
    if (k < 0) k = h->k_done;
    if (k > h->k_done) return fail(BSDE_ESTATE, "iteration not computed");
    std::memcpy(alpha, &h->alpha_hist[(size_t)k * h->p], sizeof(double) * h->p);
    if (k_done) *k_done = h->k_done;
    return BSDE_OK;
}

static bsde_status store_alpha(bsde_problem h, const double *alpha, int k_done)
{
    for (int l = 0; l < h->p; ++l)
        h->alpha_hist[(size_t)k_done * h->p + l] = h->active[l] ? alpha[l] : 0.0;
    HIP_TRY(hipMemcpy(h->d_alpha + (size_t)k_done * h->p,
                      &h->alpha_hist[(size_t)k_done * h->p],
                      sizeof(double) * h->p, hipMemcpyHostToDevice));
    h->k_done = k_done;
    h->have_alpha = true;
    return BSDE_OK;
}

bsde_status bsde_set_coefficients(bsde_problem h, const double *alpha,
                                  int k_done)
{
    if (!h || !alpha) return fail(BSDE_EINVAL, "null argument");
    if (k_done < 0 || k_done > h->K_it) return fail(BSDE_EINVAL, "bad k_done");
    if (h->kop) return fail(BSDE_EUNSUPPORTED, "the kernel operator runs whole solves");
    return store_alpha(h, alpha, k_done);
}

bsde_status bsde_fit_values(bsde_problem h, const double *y, int k_done)
{
    if (!h || !y) return fail(BSDE_EINVAL, "null argument");
    if (k_done < 0 || k_done > h->K_it) return fail(BSDE_EINVAL, "bad k_done");
    if (h->kop) return fail(BSDE_EUNSUPPORTED, "the kernel operator fits no basis");
    // alpha = R^{-1} Q' y with the device copy of W, evaluated on the host
    std::vector<double> W((size_t)h->p * h->n);
    HIP_TRY(hipMemcpy(W.data(), h->d_W, sizeof(double) * W.size(), hipMemcpyDeviceToHost));
    std::vector<double> a(h->p, 0.0);
    for (int l = 0; l < h->p; ++l) {
        double s = 0.0;
        for (int i = 0; i < h->n; ++i) s += W[(size_t)l * h->n + i] * y[i];
        a[l] = s;
    }
    return store_alpha(h, a.data(), k_done);
}

bsde_status bsde_get_corrections(bsde_problem h, int k, double *c, double *var)
{
    if (!h || !c) return fail(BSDE_EINVAL, "null argument");
    if (k < 0 || k >= h->k_done) return fail(BSDE_ESTATE, "iteration not computed");
    HIP_TRY(hipMemcpy(c, h->d_c + (size_t)k * h->n, sizeof(double) * h->n, hipMemcpyDeviceToHost));
    if (var)
        HIP_TRY(hipMemcpy(var, h->d_var + (size_t)k * h->n, sizeof(double) * h->n, hipMemcpyDeviceToHost));
    return BSDE_OK;
}

bsde_status bsde_query_price_delta(bsde_problem h, int nq, const double *t,
                                   const double *S, double *price,
                                   double *delta)
{
    if (!h || nq < 0 || (nq > 0 && (!t || !S || !price)))
        return fail(BSDE_EINVAL, "bad query arguments");
    if (!h->have_alpha) return fail(BSDE_ESTATE, "no coefficients yet");
    const int d = h->d, dp = d + 1, p = h->p;
    const double *alpha = &h->alpha_hist[(size_t)h->k_done * p];
    if (h->kop) {
        // u = h[y] = S1 / S0 and d_{x_j} u = scale_j (d_j S1 - u d_j S0) / S0
        // over the points (FP64, the clamped Gaussian weights)
        const double b2 = h->base.kbw * h->base.kbw;
        for (int qi = 0; qi < nq; ++qi) {
            double z[kMaxD + 1];
            z[0] = 2.0 * t[qi] / h->base.T - 1.0;
            for (int j = 0; j < d; ++j) {
                if (!(S[(size_t)qi * d + j] > 0.0)) return fail(BSDE_EINVAL, "price must be > 0");
                z[1 + j] = (std::log(S[(size_t)qi * d + j]) - h->base.mid[j]) * h->base.scale[j];
            }
            double S0 = 0.0, S1 = 0.0, D0[kMaxD] = {0}, D1[kMaxD] = {0};
            for (int i = 0; i < h->n; ++i) {
                double dz[kMaxD + 1], q = 0.0;
                dz[0] = z[0] - (2.0 * h->pts[(size_t)i * dp] / h->base.T - 1.0);
                q = dz[0] * dz[0];
                for (int j = 0; j < d; ++j) {
                    dz[1 + j] = z[1 + j] - (h->pts[(size_t)i * dp + 1 + j] - h->base.mid[j]) *
                                               h->base.scale[j];
                    q += dz[1 + j] * dz[1 + j];
                }
                const double e = q / (2.0 * b2);
                const bool flat = e > kKernelClamp;
                const double w = std::exp(-(flat ? kKernelClamp : e));
                S0 += w;
                S1 += alpha[i] * w;
                if (flat) continue;
                for (int j = 0; j < d; ++j) {
                    D0[j] += w * (-dz[1 + j] / b2);
                    D1[j] += alpha[i] * w * (-dz[1 + j] / b2);
                }
            }
            const double u = S1 / S0;
            price[qi] = u;
            if (delta)
                for (int j = 0; j < d; ++j)
                    delta[(size_t)qi * d + j] =
                        (D1[j] - u * D0[j]) / S0 * h->base.scale[j] / S[(size_t)qi * d + j];
        }
        return BSDE_OK;
    }
    std::vector<double> g((size_t)d * p, 0.0); // d_{x_j} coefficients
    for (int j = 0; j < d; ++j)
        for (int l = 0; l < p; ++l) {
            double s = 0.0;
            for (const auto &x : h->Dx[j][l]) s += x.second * alpha[x.first];
            g[(size_t)j * p + l] = s;
        }
    for (int qi = 0; qi < nq; ++qi) {
        double z[kMaxD + 1];
        z[0] = 2.0 * t[qi] / h->base.T - 1.0;
        for (int j = 0; j < d; ++j) {
            if (!(S[(size_t)qi * d + j] > 0.0)) return fail(BSDE_EINVAL, "price must be > 0");
            z[1 + j] = (std::log(S[(size_t)qi * d + j]) - h->base.mid[j]) * h->base.scale[j];
        }
        double u = 0.0, du[kMaxD] = {0};
        for (int l = 0; l < p; ++l) {
            double bv = 1.0;
            for (int w = 0; w < dp; ++w) bv *= cheb_value(h->nu[(size_t)l * dp + w], z[w]);
            u += alpha[l] * bv;
            for (int j = 0; j < d; ++j) du[j] += g[(size_t)j * p + l] * bv;
        }
        price[qi] = u;
        if (delta)
            for (int j = 0; j < d; ++j) delta[(size_t)qi * d + j] = du[j] / S[(size_t)qi * d + j];
    }
    return BSDE_OK;
}

void bsde_destroy(bsde_problem h)
{
    if (!h) return;
    free_device(h);
    delete h;
}

} // extern "C"
