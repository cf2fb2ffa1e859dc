// bsde_kernels.hip -- gfx950 kernels of one Picard iteration of Algorithm
// "algodetail" (Labart & Lelong, arXiv:1102.4666, Section 4.1) other than
// the Monte Carlo path kernel (bsde_path.h), and the dispatch to it:
//
//   finalize_kernel c_i = (1/M) sum_m a_m (eq. chat) and the sample variance.
//   project_kernel  beta = R^{-1} Q' c, the least-squares increment: with
//                   y = u^k + c and u^k = B alpha^k in the span of B,
//                   argmin ||y - B a|| = alpha^k + B^+ c (eq. alpha).
//   channel_kernel  alpha^{k+1} = alpha^k + beta and the channel table
//                   Gamma[l][c] = (D_c alpha^{k+1})_l of u, d_t u, grad u and
//                   the upper-triangular hessian, in FP64 and FP32.
#include "bsde_common.h"

#include <hip/hip_runtime.h>

namespace bsde {

// c_i and sample variance from the per-workgroup sums (fixed order in g)
// the groups' means and sums of squared deviations combined in group order;
// group g holds the paths g ppg .. (g + 1) ppg - 1 below M
__device__ __forceinline__ void finalize_point(const double *__restrict__ partial,
                                               int i, int groups, int M, int ppg,
                                               double *__restrict__ c,
                                               double *__restrict__ var)
{
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int g = 0; g < groups; ++g) {
        const int ng = min(ppg, M - g * ppg);
        if (ng <= 0) break;
        combine_moments(n, mean, m2, (double)ng, partial[2 * ((size_t)i * groups + g)],
                        partial[2 * ((size_t)i * groups + g) + 1]);
    }
    c[i] = mean;
    var[i] = M > 1 ? m2 / (M - 1) : 0.0;
}

__global__ void finalize_kernel(const double *__restrict__ partial, int n,
                                int groups, int M, int ppg, double *__restrict__ c,
                                double *__restrict__ var)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) finalize_point(partial, i, groups, M, ppg, c, var);
}

// beta_l = sum_i W[l][i] c_i (W = R^{-1} Q', row-major p x n): lanes
// strided over i, fixed-order tree reduction; one workgroup of 256 lanes
__device__ __forceinline__ void project_row(const double *__restrict__ W,
                                            const double *__restrict__ c,
                                            int n, int l,
                                            double *__restrict__ beta)
{
    const double *w = W + (size_t)l * n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += w[i] * c[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) beta[l] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void project_kernel(
    const double *__restrict__ W, const double *__restrict__ c, int n,
    double *__restrict__ beta)
{
    project_row(W, c, n, blockIdx.x, beta);
}

constexpr int kMaxP = 512;

// Entry e of the packed channel table (layout in bsde_common.h):
// Gamma_e = sum_k vals[k] a[cols[k]], k in rowptr[e] .. rowptr[e+1]-1, with
// a = alpha_in + beta; the sparse rows are those of the derivative channels
// D_c alpha (channel 0, the first p entries, is a itself and also stores a
// as the next coefficients).  FP64 and FP32 copies.
__device__ __forceinline__ void channel_entries(
    const double *__restrict__ alpha_in, const double *__restrict__ beta,
    double *__restrict__ alpha_out, const int *__restrict__ rowptr,
    const int *__restrict__ cols, const double *__restrict__ vals, int p,
    int nnz, int blk, double *__restrict__ g64, float *__restrict__ g32)
{
    __shared__ double a[kMaxP];
    for (int m = threadIdx.x; m < p; m += 256)
        a[m] = alpha_in[m] + (beta ? beta[m] : 0.0);
    __syncthreads();
    const int e = blk * 256 + (int)threadIdx.x;
    if (e >= nnz) return;
    if (alpha_out && e < p) alpha_out[e] = a[e];
    double v = 0.0;
    for (int k = rowptr[e]; k < rowptr[e + 1]; ++k) v += vals[k] * a[cols[k]];
    g64[e] = v;
    g32[e] = (float)v;
}

// 256 entries per workgroup
__global__ __launch_bounds__(256) void channel_kernel(
    const double *__restrict__ alpha_in, const double *__restrict__ beta,
    double *__restrict__ alpha_out, const int *__restrict__ rowptr,
    const int *__restrict__ cols, const double *__restrict__ vals, int p, int nnz,
    double *__restrict__ g64, float *__restrict__ g32)
{
    channel_entries(alpha_in, beta, alpha_out, rowptr, cols, vals, p, nnz, blockIdx.x,
                    g64, g32);
}

// ---------------------------------------------------------------------------
// Batched forms: blockIdx.y selects the problem; each problem is reduced
// and updated by the same device functions as above.
// ---------------------------------------------------------------------------
__global__ void batch_finalize_kernel(const BatchUpdateDesc *__restrict__ d)
{
    const BatchUpdateDesc &q = d[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < q.n) finalize_point(q.partial, i, q.groups, q.M, q.ppg, q.c, q.var);
}

__global__ __launch_bounds__(256) void batch_project_kernel(
    const BatchUpdateDesc *__restrict__ d)
{
    const BatchUpdateDesc &q = d[blockIdx.y];
    if ((int)blockIdx.x < q.p) project_row(q.W, q.c, q.n, blockIdx.x, q.beta);
}

__global__ __launch_bounds__(256) void batch_channel_kernel(
    const BatchUpdateDesc *__restrict__ d, int with_beta)
{
    const BatchUpdateDesc &q = d[blockIdx.y];
    if ((int)blockIdx.x * 256 < q.nnz)
        channel_entries(q.alpha_in, with_beta ? q.beta : nullptr,
                        with_beta ? q.alpha_out : nullptr, q.rowptr, q.cols, q.vals,
                        q.p, q.nnz, blockIdx.x, q.g64, q.g32);
}

// Point values of the kernel operator (Section 3.2) for the next iteration:
// y^k_i = u^k(t_i, x_i) + c^k_i with u^k = h[y^{k-1}] = sum_j y_j w_j /
// sum_j w_j (FP64), w_j = exp(-min(|z_i - z_j|^2 / (2 b^2), clamp)) in the
// mapped coordinates; yprev null for u^k = 0.  Writes y^k (FP64) and the y
// column of the path kernel's table (FP32 or FP64).  One lane per point;
// the loop over the points j is uniform (scalar loads of their rows).
__global__ __launch_bounds__(256) void kernel_update_kernel(
    const PathParams prm, int d, const double *__restrict__ pts,
    const double *__restrict__ yprev, const double *__restrict__ c,
    double *__restrict__ ynew, void *__restrict__ table, int fp32)
{
    const int n = prm.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int dp = d + 1;
    const double inv2b2 = 0.5 / (prm.kbw * prm.kbw);
    double zi[kMaxD + 1];
    zi[0] = 2.0 * pts[(size_t)i * dp] / prm.T - 1.0;
    for (int j = 0; j < d; ++j)
        zi[1 + j] = (pts[(size_t)i * dp + 1 + j] - prm.mid[j]) * prm.scale[j];
    double u = 0.0;
    if (yprev) {
        double S0 = 0.0, S1 = 0.0;
        for (int q = 0; q < n; ++q) {
            const double *row = pts + (size_t)q * dp;
            double dz = zi[0] - (2.0 * row[0] / prm.T - 1.0);
            double qq = dz * dz;
            for (int j = 0; j < d; ++j) {
                dz = zi[1 + j] - (row[1 + j] - prm.mid[j]) * prm.scale[j];
                qq += dz * dz;
            }
            const double w = exp(-fmin(qq * inv2b2, kKernelClamp));
            S0 += w;
            S1 += yprev[q] * w;
        }
        u = S1 / S0;
    }
    const double y = u + c[i];
    ynew[i] = y;
    if (fp32)
        ((float *)table)[(size_t)i * kKernelRow + 1 + d] = (float)y;
    else
        ((double *)table)[(size_t)i * kKernelRow + 1 + d] = y;
}

hipError_t launch_kernel_update(const PathParams &prm, int d, const double *pts,
                                const double *yprev, const double *c, double *ynew,
                                void *table, int fp32, hipStream_t s)
{
    hipLaunchKernelGGL(kernel_update_kernel, dim3((prm.n + 255) / 256), dim3(256), 0, s,
                       prm, d, pts, yprev, c, ynew, table, fp32);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, int n, int groups, int M,
                           int ppg, double *c, double *var, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                       partial, n, groups, M, ppg, c, var);
    return hipGetLastError();
}

__global__ void reset_counters_kernel(unsigned int *c, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}

hipError_t launch_batch_update(int nprob, int max_n, int max_p, int max_cb,
                               hipStream_t s, const BatchUpdateDesc *d)
{
    hipLaunchKernelGGL(batch_finalize_kernel,
                       dim3((max_n + 255) / 256, nprob), dim3(256), 0, s, d);
    hipLaunchKernelGGL(batch_project_kernel, dim3(max_p, nprob), dim3(256), 0,
                       s, d);
    hipLaunchKernelGGL(batch_channel_kernel, dim3(max_cb, nprob), dim3(256), 0,
                       s, d, 1);
    return hipGetLastError();
}

hipError_t launch_batch_channels(int nprob, int max_cb, hipStream_t s,
                                 const BatchUpdateDesc *d)
{
    hipLaunchKernelGGL(batch_channel_kernel, dim3(max_cb, nprob), dim3(256), 0,
                       s, d, 0);
    return hipGetLastError();
}

hipError_t launch_reset_counters(unsigned int *c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counters_kernel, dim3((n + 255) / 256), dim3(256),
                       0, s, c, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dispatch over the translation units of path kernels: X(D, NAME) for the
// unit of dimension D whose functions are named launch_path_dNAME, ...
// (bsde_path.h).  d = 10 has a unit for its total-degree sets in FP32, one
// for them in FP64 and one per hyperbolic set (eta = 5, q = 0.5, 0.6, 0.7).
// ---------------------------------------------------------------------------
#define BSDE_UNITS(X)                                                          \
    X(1, 1) X(2, 2) X(3, 3) X(5, 5) X(10, 10) X(10, 10d) X(10, 10q5)           \
    X(10, 10q6) X(10, 10q7)
#define DECL(D, N)                                                             \
    hipError_t launch_path_d##N(int eta, int q10, bool fp32, int blocks,        \
                                hipStream_t s,                                 \
                                const PathParams &prm, const double *pts,      \
                                const void *gamma, double *partial,            \
                                hipEvent_t ev0, hipEvent_t ev1);               \
    int index_table_d##N(int eta, int q10, int8_t *nu, int cap);               \
    hipError_t launch_batch_d##N(int eta, int q10, bool fp32, int vol,         \
                                 int blocks,                                   \
                                 hipStream_t s, const BatchTileDesc *probs,    \
                                 int nprob, const long long *tile_begin,       \
                                 unsigned int *counter);                       \
    int batch_occupancy_d##N(int eta, int q10, bool fp32, int vol);            \
    bool has_variant_d##N(int eta, int q10, bool fp32, int vol);
BSDE_UNITS(DECL)
#undef DECL
hipError_t launch_kernel_path_d1(bool fp32, int blocks, hipStream_t s,
                                 const PathParams &prm, const double *pts,
                                 const void *table, double *partial,
                                 hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_kernel_path_d2(bool fp32, int blocks, hipStream_t s,
                                 const PathParams &prm, const double *pts,
                                 const void *table, double *partial,
                                 hipEvent_t ev0, hipEvent_t ev1);

// path kernels of the kernel operator exist for d <= 2, constant and bump
// volatility, FP32 and FP64 paths
bool kernel_op_exists(int d, int vol)
{
    return (d == 1 || d == 2) && (vol == kVolConst || vol == kVolBump);
}

hipError_t launch_kernel_path(int d, bool fp32, int blocks, hipStream_t s,
                              const PathParams &prm, const double *pts,
                              const void *table, double *partial,
                              hipEvent_t ev0, hipEvent_t ev1)
{
    if (d == 1)
        return launch_kernel_path_d1(fp32, blocks, s, prm, pts, table, partial, ev0, ev1);
    if (d == 2)
        return launch_kernel_path_d2(fp32, blocks, s, prm, pts, table, partial, ev0, ev1);
    return hipErrorInvalidValue;
}

int index_table(int d, int eta, int q10, int8_t *nu, int cap)
{
#define X(D, N)                                                                \
    if (d == D) {                                                              \
        const int p = index_table_d##N(eta, q10, nu, cap);                     \
        if (p > 0) return p;                                                   \
    }
    BSDE_UNITS(X)
#undef X
    return 0;
}

bool kernel_exists(int d, int eta, int q10)
{
    return index_table(d, eta, q10, nullptr, 0) > 0;
}

bool variant_exists(int d, int eta, int q10, bool fp32, int vol)
{
#define X(D, N)                                                                \
    if (d == D && has_variant_d##N(eta, q10, fp32, vol)) return true;
    BSDE_UNITS(X)
#undef X
    return false;
}

hipError_t launch_path(int d, int eta, int q10, bool fp32, int blocks, hipStream_t s,
                       const PathParams &prm, const double *pts,
                       const void *gamma, double *partial, hipEvent_t ev0,
                       hipEvent_t ev1)
{
#define X(D, N)                                                                \
    if (d == D && has_variant_d##N(eta, q10, fp32, prm.vol_kind))              \
        return launch_path_d##N(eta, q10, fp32, blocks, s, prm, pts, gamma,    \
                                partial, ev0, ev1);
    BSDE_UNITS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int d, int eta, int q10, bool fp32, int vol, int blocks,
                        hipStream_t s, const BatchTileDesc *probs, int nprob,
                        const long long *tile_begin, unsigned int *counter)
{
#define X(D, N)                                                                \
    if (d == D && has_variant_d##N(eta, q10, fp32, vol))                       \
        return launch_batch_d##N(eta, q10, fp32, vol, blocks, s, probs, nprob, \
                                 tile_begin, counter);
    BSDE_UNITS(X)
#undef X
    return hipErrorInvalidValue;
}

int batch_occupancy(int d, int eta, int q10, bool fp32, int vol)
{
#define X(D, N)                                                                \
    if (d == D && has_variant_d##N(eta, q10, fp32, vol))                       \
        return batch_occupancy_d##N(eta, q10, fp32, vol);
    BSDE_UNITS(X)
#undef X
    return 0;
}

hipError_t launch_update(int n, int groups, int M, int ppg, int p, int nnz,
                         hipStream_t s, const double *partial, double *c,
                         double *var, const double *W, double *beta,
                         const double *alpha_in, double *alpha_out,
                         const int *rowptr, const int *cols, const double *vals,
                         double *g64, float *g32, hipEvent_t *ev /* 3 events or NULL */)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       s, partial, n, groups, M, ppg, c, var);
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(project_kernel, dim3(p), dim3(256), 0, s, W, c, n,
                       beta);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(channel_kernel, dim3((nnz + 255) / 256), dim3(256), 0, s,
                       alpha_in, beta, alpha_out, rowptr, cols, vals, p, nnz, g64, g32);
    if (ev) (void)hipEventRecord(ev[2], s);
    return hipGetLastError();
}

hipError_t launch_channels(int p, int nnz, hipStream_t s, const double *alpha,
                           const int *rowptr, const int *cols, const double *vals,
                           double *g64, float *g32)
{
    hipLaunchKernelGGL(channel_kernel, dim3((nnz + 255) / 256), dim3(256), 0, s,
                       alpha, (const double *)nullptr, (double *)nullptr, rowptr,
                       cols, vals, p, nnz, g64, g32);
    return hipGetLastError();
}

} // namespace bsde
