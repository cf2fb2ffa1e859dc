// bsde_host.cpp -- C ABI of libbsde.so: problem set-up on the host (index
// set, grid, Chebyshev basis, rank-checked Householder QR, pseudo-inverse
// R^{-1} Q', derivative channel matrices), device buffers, the Picard loop
// that launches the HIP kernels, and the price/delta read-out.
//
// The method is Algorithm "algodetail" of Labart & Lelong (arXiv:1102.4666,
// Section 4.1); the least-squares extrapolating operator is that of
// Section 4.2 (eq. lspb) with polynomials centred and normalised to
// [-1, 1]^{d+1}; the model is Section 5 (eq. 4) with the correlation of
// Section 6.2.
#include "../../include/bsde.h"
#include "bsde_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace bsde {
bool kernel_exists(int d, int eta);
int index_table(int d, int eta, int8_t *nu, int cap);
hipError_t launch_path(int d, int eta, bool fp32, int blocks, hipStream_t s,
                       const PathParams &prm, const double *pts,
                       const void *gamma, double *partial);
hipError_t launch_update(int n, int groups, int M, int p, int C,
                         hipStream_t s, const double *partial, double *c,
                         double *var, const double *W, double *beta,
                         const double *alpha_in, double *alpha_out,
                         const double *Dmat, double *g64, float *g32,
                         hipEvent_t *ev);
hipError_t launch_channels(int p, int C, hipStream_t s, const double *alpha,
                           const double *Dmat, double *g64, float *g32);
} // namespace bsde

using namespace bsde;

static thread_local std::string g_last_error;

static bsde_status fail(bsde_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

struct bsde_problem_s {
    // parameters
    int d = 0, eta = 0, M = 0, N = 0, K_it = 0, precision = 0;
    double q = 1.0, omega = 0.0;
    PathParams base{};
    // sizes
    int n = 0, n_spatial = 0, p = 0, C = 0;
    std::vector<int8_t> nu;      // p x (d+1), kernel order
    std::vector<char> active;    // in the hyperbolic set
    std::vector<double> pts;     // n x (d+1)
    std::vector<double> lo, hi;
    std::vector<double> Dfirst;  // d x p x p: d_{x_j} channel matrices
    // device
    double *d_pts = nullptr, *d_W = nullptr, *d_D = nullptr,
           *d_alpha = nullptr, *d_beta = nullptr, *d_g64 = nullptr,
           *d_partial = nullptr, *d_c = nullptr, *d_var = nullptr;
    float *d_g32 = nullptr;
    size_t partial_cap = 0;
    // state
    int k_done = 0;
    bool have_alpha = false;
    std::vector<double> alpha_hist; // (K_it + 1) x p, host mirror
    int groups = 0, ppl = 0;       // tiling (0 = automatic)
    double timings[5] = {0, 0, 0, 0, 0};
};

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

// Householder QR of B (n x pa, row-major); returns W = R^{-1} Q' (pa x n)
// or false if rank deficient.
static bool pseudo_inverse(int n, int pa, std::vector<double> &A,
                           std::vector<double> &W, std::string &why)
{
    std::vector<double> vs((size_t)n * pa, 0.0), vnorm(pa), diag(pa);
    for (int j = 0; j < pa; ++j) {
        double nrm2 = 0.0;
        for (int i = j; i < n; ++i) nrm2 += A[(size_t)i * pa + j] * A[(size_t)i * pa + j];
        double nrm = std::sqrt(nrm2);
        if (nrm == 0.0) {
            why = "basis matrix has a zero column";
            return false;
        }
        double top = A[(size_t)j * pa + j];
        double beta = top >= 0.0 ? -nrm : nrm;
        double vv = 0.0;
        for (int i = j; i < n; ++i) {
            double v = A[(size_t)i * pa + j] - (i == j ? beta : 0.0);
            vs[(size_t)i * pa + j] = v;
            vv += v * v;
        }
        vnorm[j] = vv;
        diag[j] = beta;
        for (int c = j; c < pa; ++c) {
            double s = 0.0;
            for (int i = j; i < n; ++i) s += vs[(size_t)i * pa + j] * A[(size_t)i * pa + c];
            double f = 2.0 * s / vv;
            for (int i = j; i < n; ++i) A[(size_t)i * pa + c] -= f * vs[(size_t)i * pa + j];
        }
    }
    double dmax = 0.0, dmin = INFINITY;
    for (int j = 0; j < pa; ++j) {
        dmax = std::max(dmax, std::fabs(diag[j]));
        dmin = std::min(dmin, std::fabs(diag[j]));
    }
    if (!(dmin > 1e-12 * dmax)) {
        why = "basis matrix is numerically rank deficient on the grid";
        return false;
    }
    // Q' e_i for every i gives the columns of Q' (pa x n): apply H_p..H_1
    // in reverse to the unit vectors is costly; instead form thin Q = H_1..H_pa
    // [I; 0] column by column and transpose.
    std::vector<double> Q((size_t)n * pa, 0.0);
    for (int c = 0; c < pa; ++c) {
        std::vector<double> e(n, 0.0);
        e[c] = 1.0;
        for (int j = pa - 1; j >= 0; --j) {
            double s = 0.0;
            for (int i = j; i < n; ++i) s += vs[(size_t)i * pa + j] * e[i];
            double f = 2.0 * s / vnorm[j];
            for (int i = j; i < n; ++i) e[i] -= f * vs[(size_t)i * pa + j];
        }
        for (int i = 0; i < n; ++i) Q[(size_t)i * pa + c] = e[i];
    }
    // W = R^{-1} Q': back substitution for every column i of Q'
    W.assign((size_t)pa * n, 0.0);
    std::vector<double> col(pa);
    for (int i = 0; i < n; ++i) {
        for (int j = pa - 1; j >= 0; --j) {
            double s = Q[(size_t)i * pa + j];
            for (int c = j + 1; c < pa; ++c) s -= A[(size_t)j * pa + c] * col[c];
            col[j] = s / A[(size_t)j * pa + j];
        }
        for (int j = 0; j < pa; ++j) W[(size_t)j * n + i] = col[j];
    }
    return true;
}

static void free_device(bsde_problem_s *h)
{
    hipFree(h->d_pts);
    hipFree(h->d_W);
    hipFree(h->d_D);
    hipFree(h->d_alpha);
    hipFree(h->d_beta);
    hipFree(h->d_g64);
    hipFree(h->d_g32);
    hipFree(h->d_partial);
    hipFree(h->d_c);
    hipFree(h->d_var);
    h->d_pts = h->d_W = h->d_D = h->d_alpha = h->d_beta = h->d_g64 = nullptr;
    h->d_partial = h->d_c = h->d_var = nullptr;
    h->d_g32 = nullptr;
}

#define HIP_TRY(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(BSDE_EDEVICE, std::string(#expr) + ": " +              \
                                          hipGetErrorString(e_));              \
    } while (0)

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
    }
    return "unknown status";
}

const char *bsde_last_error(void) { return g_last_error.c_str(); }

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
    if (sigma->kind != BSDE_VOL_CONST && sigma->kind != BSDE_VOL_BUMP)
        return fail(BSDE_EINVAL, "bad volatility kind");
    if (sigma->kind == BSDE_VOL_BUMP && !(sigma->bump_c > 0.0))
        return fail(BSDE_EINVAL, "bump centre must be > 0");
    if (grid->kind != BSDE_GRID_TENSOR && grid->kind != BSDE_GRID_RANDOM)
        return fail(BSDE_EINVAL, "bad grid kind");
    if (grid->n_t < 2 || grid->n_x < 1 || !(grid->width > 0.0) ||
        grid->eta < 1 || !(grid->q > 0.0 && grid->q <= 1.0))
        return fail(BSDE_EINVAL, "bad grid (n_t >= 2, n_x >= 1, width > 0, "
                                 "eta >= 1, 0 < q <= 1)");
    if (precision != BSDE_FP64 && precision != BSDE_FP32_PATHS)
        return fail(BSDE_EINVAL, "bad precision");
    for (int j = 0; j < d; ++j)
        if (!(sigma->level[j] > 0.0) || !(payoff->S0[j] > 0.0))
            return fail(BSDE_EINVAL, "levels and spots must be > 0");
    if (!kernel_exists(d, grid->eta))
        return fail(BSDE_EUNSUPPORTED, "no kernel instantiated for d=" +
                                           std::to_string(d) + ", eta=" +
                                           std::to_string(grid->eta));
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
        b.div[j] = sigma->dividend ? sigma->dividend[j] : 0.0;
        double half = grid->width * sigma->level[j] * std::sqrt(payoff->T);
        h->lo[j] = std::log(payoff->S0[j]) - half;
        h->hi[j] = std::log(payoff->S0[j]) + half;
        b.mid[j] = 0.5 * (h->lo[j] + h->hi[j]);
        b.scale[j] = 2.0 / (h->hi[j] - h->lo[j]);
    }

    // index set in kernel order; hyperbolic subset marked active
    const int dp = d + 1;
    h->p = index_table(d, grid->eta, nullptr, 0);
    h->nu.resize((size_t)h->p * dp);
    index_table(d, grid->eta, h->nu.data(), h->p);
    h->active.assign(h->p, 1);
    if (grid->q < 1.0) {
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
    if ((long)ns * grid->n_t > (1L << 26)) {
        delete h;
        return fail(BSDE_EINVAL, "too many points");
    }
    h->n_spatial = (int)ns;
    h->n = (int)(ns * grid->n_t);
    h->pts.resize((size_t)h->n * dp);
    for (int a = 0; a < grid->n_t; ++a) {
        double t = a * payoff->T / (grid->n_t - 1);
        for (long s = 0; s < ns; ++s) {
            double *row = &h->pts[(size_t)(a * ns + s) * dp];
            row[0] = t;
            long rest = s;
            for (int j = 0; j < d; ++j) {
                double z;
                if (grid->kind == BSDE_GRID_TENSOR) {
                    long digit = rest % grid->n_x;
                    rest /= grid->n_x;
                    z = grid->n_x > 1 ? -1.0 + 2.0 * digit / (grid->n_x - 1) : 0.0;
                } else {
                    u32x4 w = philox10((uint32_t)s, 0, 0, (2u << 24) | (uint32_t)(j / 4),
                                       (uint32_t)seed, (uint32_t)(seed >> 32));
                    uint32_t word = j % 4 == 0 ? w.x : j % 4 == 1 ? w.y : j % 4 == 2 ? w.z : w.w;
                    z = 2.0 * (((double)word + 0.5) * 0x1p-32) - 1.0;
                }
                row[1 + j] = h->lo[j] + 0.5 * (z + 1.0) * (h->hi[j] - h->lo[j]);
            }
        }
    }

    // basis matrix over the active multi-indices and its pseudo-inverse
    std::vector<int> act;
    for (int l = 0; l < h->p; ++l)
        if (h->active[l]) act.push_back(l);
    const int pa = (int)act.size();
    if (h->n < pa) {
        delete h;
        return fail(BSDE_ERANK, "fewer points than basis functions");
    }
    std::vector<double> B((size_t)h->n * pa);
    for (int i = 0; i < h->n; ++i) {
        const double *row = &h->pts[(size_t)i * dp];
        double z[kMaxD + 1];
        z[0] = 2.0 * row[0] / payoff->T - 1.0;
        for (int j = 0; j < d; ++j) z[1 + j] = (row[1 + j] - b.mid[j]) * b.scale[j];
        for (int c = 0; c < pa; ++c) {
            const int8_t *e = &h->nu[(size_t)act[c] * dp];
            double v = 1.0;
            for (int w = 0; w < dp; ++w) v *= cheb_value(e[w], z[w]);
            B[(size_t)i * pa + c] = v;
        }
    }
    std::vector<double> Wa;
    std::string why;
    if (!pseudo_inverse(h->n, pa, B, Wa, why)) {
        delete h;
        return fail(BSDE_ERANK, why);
    }
    std::vector<double> W((size_t)h->p * h->n, 0.0);
    for (int c = 0; c < pa; ++c)
        std::memcpy(&W[(size_t)act[c] * h->n], &Wa[(size_t)c * h->n], sizeof(double) * h->n);

    // channel matrices: first derivatives in each variate, then products
    std::map<std::vector<int8_t>, int> pos;
    for (int l = 0; l < h->p; ++l)
        pos[std::vector<int8_t>(&h->nu[(size_t)l * dp], &h->nu[(size_t)l * dp] + dp)] = l;
    const size_t pp = (size_t)h->p * h->p;
    std::vector<double> Dv((size_t)dp * pp, 0.0); // d/dz_v, unscaled
    for (int v = 0; v < dp; ++v)
        for (int l = 0; l < h->p; ++l) {
            std::vector<int8_t> e(&h->nu[(size_t)l * dp], &h->nu[(size_t)l * dp] + dp);
            int a = e[v];
            for (int bb = 0; bb < a; ++bb) {
                double cf = cheb_deriv_coef(a, bb);
                if (cf == 0.0) continue;
                std::vector<int8_t> mu = e;
                mu[v] = (int8_t)bb;
                Dv[(size_t)v * pp + (size_t)pos[mu] * h->p + l] += cf;
            }
        }
    std::vector<double> Dm((size_t)(h->C - 1) * pp, 0.0);
    const double tfac = 2.0 / payoff->T;
    for (size_t e = 0; e < pp; ++e) Dm[e] = tfac * Dv[e]; // channel 1: d_t
    h->Dfirst.assign((size_t)d * pp, 0.0);
    for (int j = 0; j < d; ++j)
        for (size_t e = 0; e < pp; ++e) {
            double v = b.scale[j] * Dv[(size_t)(1 + j) * pp + e];
            Dm[(size_t)(1 + j) * pp + e] = v;
            h->Dfirst[(size_t)j * pp + e] = v;
        }
    int ch = 1 + d;
    for (int j = 0; j < d; ++j)
        for (int k = j; k < d; ++k, ++ch) {
            const double *A1 = &h->Dfirst[(size_t)j * pp];
            const double *A2 = &h->Dfirst[(size_t)k * pp];
            double *O = &Dm[(size_t)ch * pp];
            for (int l = 0; l < h->p; ++l)
                for (int mm = 0; mm < h->p; ++mm) {
                    double a1 = A1[(size_t)l * h->p + mm];
                    if (a1 == 0.0) continue;
                    for (int c = 0; c < h->p; ++c)
                        O[(size_t)l * h->p + c] += a1 * A2[(size_t)mm * h->p + c];
                }
        }

    // device buffers
    hipError_t alloc_err = hipSuccess;
    auto dalloc = [&](void **ptr, size_t bytes) {
        alloc_err = hipMalloc(ptr, bytes == 0 ? 8 : bytes);
        return alloc_err == hipSuccess;
    };
    bool ok = dalloc((void **)&h->d_pts, sizeof(double) * h->pts.size()) &&
              dalloc((void **)&h->d_W, sizeof(double) * W.size()) &&
              dalloc((void **)&h->d_D, sizeof(double) * Dm.size()) &&
              dalloc((void **)&h->d_alpha, sizeof(double) * (size_t)(h->K_it + 1) * h->p) &&
              dalloc((void **)&h->d_beta, sizeof(double) * h->p) &&
              dalloc((void **)&h->d_g64, sizeof(double) * (size_t)h->p * h->C) &&
              dalloc((void **)&h->d_g32, sizeof(float) * (size_t)h->p * h->C) &&
              dalloc((void **)&h->d_c, sizeof(double) * (size_t)h->K_it * h->n) &&
              dalloc((void **)&h->d_var, sizeof(double) * (size_t)h->K_it * h->n);
    if (!ok) {
        free_device(h);
        delete h;
        if (alloc_err == hipErrorOutOfMemory)
            return fail(BSDE_ENOMEM, "device allocation failed");
        return fail(BSDE_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(alloc_err));
    }
    hipError_t e = hipMemcpy(h->d_pts, h->pts.data(), sizeof(double) * h->pts.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_W, W.data(), sizeof(double) * W.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_D, Dm.data(), sizeof(double) * Dm.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->d_alpha, 0, sizeof(double) * (size_t)(h->K_it + 1) * h->p);
    if (e != hipSuccess) {
        free_device(h);
        delete h;
        return fail(BSDE_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    h->alpha_hist.assign((size_t)(h->K_it + 1) * h->p, 0.0);
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

bsde_status bsde_solve(bsde_problem h, void *hip_stream)
{
    if (!h) return fail(BSDE_EINVAL, "null handle");
    hipStream_t s = (hipStream_t)hip_stream;
    int groups = h->groups, ppl = h->ppl;
    if (groups == 0) auto_tiling(h, groups, ppl);
    const size_t need = (size_t)h->n * groups * 2;
    if (need > h->partial_cap) {
        hipFree(h->d_partial);
        h->d_partial = nullptr;
        h->partial_cap = 0;
        HIP_TRY(hipMalloc((void **)&h->d_partial, sizeof(double) * need));
        h->partial_cap = need;
    }
    const bool fp32 = h->precision == BSDE_FP32_PATHS;
    const int iters = h->K_it - h->k_done;
    // events: start, end, and 4 per iteration (before path, after path,
    // after reduction, after projection; the next iteration's first event
    // closes the channel update)
    std::vector<hipEvent_t> ev(2 + 4 * (size_t)iters + 1);
    for (auto &x : ev) HIP_TRY(hipEventCreate(&x));
    HIP_TRY(hipEventRecord(ev[0], s));
    // channel table of the starting coefficients
    HIP_TRY(launch_channels(h->p, h->C, s, h->d_alpha + (size_t)h->k_done * h->p,
                            h->d_D, h->d_g64, h->d_g32));
    for (int it = 0; it < iters; ++it) {
        const int k = h->k_done + it;
        hipEvent_t *e = &ev[2 + 4 * (size_t)it];
        PathParams prm = h->base;
        prm.k = (uint32_t)k;
        prm.groups = groups;
        prm.paths_per_lane = ppl;
        prm.n = h->n;
        HIP_TRY(hipEventRecord(e[0], s));
        HIP_TRY(launch_path(h->d, h->eta, fp32, h->n * groups, s, prm, h->d_pts,
                            fp32 ? (const void *)h->d_g32 : (const void *)h->d_g64,
                            h->d_partial));
        HIP_TRY(hipEventRecord(e[1], s));
        HIP_TRY(launch_update(h->n, groups, h->M, h->p, h->C, s, h->d_partial,
                              h->d_c + (size_t)k * h->n, h->d_var + (size_t)k * h->n,
                              h->d_W, h->d_beta, h->d_alpha + (size_t)k * h->p,
                              h->d_alpha + (size_t)(k + 1) * h->p, h->d_D, h->d_g64,
                              h->d_g32, e + 2));
    }
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipEventSynchronize(ev[1]));
    double t_path = 0, t_fin = 0, t_proj = 0, t_chan = 0;
    for (int it = 0; it < iters; ++it) {
        hipEvent_t *e = &ev[2 + 4 * (size_t)it];
        float ms;
        hipEventElapsedTime(&ms, e[0], e[1]); t_path += ms;
        hipEventElapsedTime(&ms, e[1], e[2]); t_fin += ms;
        hipEventElapsedTime(&ms, e[2], e[3]); t_proj += ms;
        hipEventElapsedTime(&ms, e[3], it + 1 < iters ? e[4] : ev[1]); t_chan += ms;
    }
    float tot;
    hipEventElapsedTime(&tot, ev[0], ev[1]);
    for (auto &x : ev) hipEventDestroy(x);
    HIP_TRY(hipMemcpy(h->alpha_hist.data(), h->d_alpha,
                      sizeof(double) * h->alpha_hist.size(), hipMemcpyDeviceToHost));
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
    return store_alpha(h, alpha, k_done);
}

bsde_status bsde_fit_values(bsde_problem h, const double *y, int k_done)
{
    if (!h || !y) return fail(BSDE_EINVAL, "null argument");
    if (k_done < 0 || k_done > h->K_it) return fail(BSDE_EINVAL, "bad k_done");
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
    const size_t pp = (size_t)p * p;
    std::vector<double> g((size_t)d * p, 0.0); // d_{x_j} coefficients
    for (int j = 0; j < d; ++j)
        for (int l = 0; l < p; ++l) {
            double s = 0.0;
            for (int m = 0; m < p; ++m) s += h->Dfirst[(size_t)j * pp + (size_t)l * p + m] * alpha[m];
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
