// bsde_setup.hip -- gfx950 kernels of the least-squares set-up: the basis
// matrix B of the grid points (Section 3.2, the polynomial projection
// operator of eq. (3.1) restricted to the index set of Section 3.3) and the
// pieces of its pseudo-inverse B^+ = R^{-1} Q' by CholeskyQR2:
//
//   G1 = B'B,  R1 = chol(G1),  Q1 = B R1^{-1},
//   G2 = Q1'Q1, R2 = chol(G2),  B^+' = Q1 R2^{-1} R2^{-T} R1^{-T}.
//
// The Gram products and the tall-skinny products run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64).  The two p x p Cholesky factorisations,
// the triangular inverses and the p x p products run in one wave with
// the matrices in LDS when p <= kSmallFactorP (small_factor_kernel), so that
// the whole set-up is stream-ordered with one host synchronisation at the
// end; larger bases take them on the host.
//
// Matrices over the points are column-major with a leading dimension that
// is a multiple of 64 (each basis function's values over the points are
// contiguous); padding rows and columns hold zeros.
#include "bsde_common.h"

#include <hip/hip_runtime.h>

namespace bsde {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mma64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// B[c][i] = prod_v T_{nu_cv}(z_v(point i)) with z_0 = 2t/T - 1 and
// z_j = (x_j - mid_j) scale_j; zero for i >= n or c >= pa.  One lane per
// (point, column): the Chebyshev recurrence per factor costs eta FMAs.
__global__ __launch_bounds__(256) void basis_matrix_kernel(
    const double *__restrict__ pts, int n, int ld, int dp,
    const int8_t *__restrict__ nu, int pa, const double *__restrict__ mid,
    const double *__restrict__ scale, double T, double *__restrict__ B)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= ld) return;
    double v = 0.0;
    if (i < n && c < pa) {
        v = 1.0;
        const double *row = pts + (size_t)i * dp;
        for (int w = 0; w < dp; ++w) {
            const double z = w == 0 ? 2.0 * row[0] / T - 1.0
                                    : (row[w] - mid[w - 1]) * scale[w - 1];
            const int a = nu[(size_t)c * dp + w];
            double t0 = 1.0, t1 = z;
            for (int k = 1; k < a; ++k) {
                const double t2 = 2.0 * z * t1 - t0;
                t0 = t1;
                t1 = t2;
            }
            v *= a == 0 ? 1.0 : t1;
        }
    }
    B[(size_t)c * ld + i] = v;
}

// Partial Gram matrices: workgroup (pair, chunk) -- one wave -- forms the
// 64 x 64 block (bi, bj), bi <= bj, of A'A over the rows of its chunk.
// The rows assigned to the four k-slots of an MFMA are permuted so that
// each lane reads 4 consecutive rows of one column (32 contiguous bytes,
// a whole 128-byte line per 4 lanes): in step t of a 16-row group at s,
// k-slot kk takes row s + 4 kk + t, the same for both operands.
// partial[chunk][r][c] holds the block's entries (r in bi's rows).
__global__ __launch_bounds__(64) void gram_partial_kernel(
    const double *__restrict__ A, int ld, int pap, int rows_per_chunk,
    const int2 *__restrict__ pairs, double *__restrict__ partial)
{
    const int2 pr = pairs[blockIdx.x];
    const int chunk = blockIdx.y;
    const int lane = threadIdx.x;
    const int r0 = chunk * rows_per_chunk;
    const int r1 = min(ld, r0 + rows_per_chunk);
    const int tiles = pap >> 4;
    int nti = 0, ntj = 0;
    const double *pa[4], *pb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ti = pr.x * 4 + t, tj = pr.y * 4 + t;
        nti += ti < tiles;
        ntj += tj < tiles;
        pa[t] = A + (size_t)(min(ti, tiles - 1) * 16 + (lane & 15)) * ld + 4 * (lane >> 4);
        pb[t] = A + (size_t)(min(tj, tiles - 1) * 16 + (lane & 15)) * ld + 4 * (lane >> 4);
    }
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int s = r0; s < r1; s += 16) {
        double va[4][4], vb[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < nti) {
                const double2 x = *(const double2 *)(pa[t] + s);
                const double2 y = *(const double2 *)(pa[t] + s + 2);
                va[t][0] = x.x; va[t][1] = x.y; va[t][2] = y.x; va[t][3] = y.y;
            }
            if (t < ntj) {
                const double2 x = *(const double2 *)(pb[t] + s);
                const double2 y = *(const double2 *)(pb[t] + s + 2);
                vb[t][0] = x.x; vb[t][1] = x.y; vb[t][2] = y.x; vb[t][3] = y.y;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (a < nti && b < ntj) acc[a][b] = mma64(va[a][k], vb[b][k], acc[a][b]);
    }
    double *out = partial + (size_t)chunk * pap * pap;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (a < nti && b < ntj) {
                const int col = (pr.y * 4 + b) * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = (pr.x * 4 + a) * 16 + (lane >> 4) + 4 * v;
                    out[(size_t)row * pap + col] = acc[a][b][v];
                }
            }
}

// G[r][c] (pa x pa, row-major) = sum over chunks, in chunk order, of the
// partial entry of the upper block holding (r, c) or (c, r)
__global__ void gram_reduce_kernel(const double *__restrict__ partial,
                                   int chunks, int pap, int pa,
                                   double *__restrict__ G)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= pa * pa) return;
    int r = idx / pa, c = idx % pa;
    if ((r >> 6) > (c >> 6)) {
        const int x = r;
        r = c;
        c = x;
    }
    double s = 0.0;
    for (int k = 0; k < chunks; ++k) s += partial[((size_t)k * pap + r) * pap + c];
    G[idx] = s;
}

// Y = A X for A (ld x pap, column-major, rows >= n zero) and X (pap x pap,
// row-major): one wave per 64 x 64 block of Y', so that the A operand is
// X' (coalesced rows of X) and the B operand is A' (16 consecutive rows of
// A per k).  Column c of the result goes to Y + colmap[c] * ldy (c < ncols)
// for rows < nrows.
__global__ __launch_bounds__(64) void gemm_ax_kernel(
    const double *__restrict__ A, int ld, const double *__restrict__ X,
    int pap, double *__restrict__ Y, int ldy, int nrows,
    const int *__restrict__ colmap, int ncols, const int *__restrict__ skip)
{
    // a failed factorisation upstream (skip != 0) leaves Y untouched
    if (skip && *skip != 0) return;
    const int lane = threadIdx.x;
    const int i0 = blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    const int tiles = pap >> 4;
    const int ntc = min(4, tiles - (c0 >> 4));
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double *xa = X + (size_t)(lane >> 4) * pap + c0 + (lane & 15);
    const double *ab = A + (size_t)(lane >> 4) * ld + i0 + (lane & 15);
    for (int k = 0; k < pap; k += 4) {
        double va[4], vb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            va[a] = a < ntc ? xa[(size_t)k * pap + 16 * a] : 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) vb[b] = ab[(size_t)k * ld + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (a < ntc) acc[a][b] = mma64(va[a], vb[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + 16 * b + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * a + (lane >> 4) + 4 * v;
                if (a < ntc && c < ncols && i < nrows)
                    Y[(size_t)(colmap ? colmap[c] : c) * ldy + i] = acc[a][b][v];
            }
        }
}

// ---------------------------------------------------------------------------
// Small factorisations in LDS, one wave: a wave's LDS operations complete in
// issue order, so the steps are ordered by wavefront-scope fences (which
// keep the compiler from moving LDS accesses across them) instead of
// workgroup barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Upper Cholesky factor of the symmetric pa x pa matrix in R (row-major, in
// LDS), in place: R'R = G.  The rank test is that of the host version: every
// pivot must be positive and its square root above rel_tol times the square
// root of the largest diagonal entry of G.  Returns false in every lane when
// a pivot fails.
__device__ bool chol_upper_lds(double *R, int pa, double rel_tol)
{
    const int t = threadIdx.x;
    double dmax = 0.0;
    for (int j = 0; j < pa; ++j) dmax = fmax(dmax, R[j * pa + j]);
    dmax = sqrt(fmax(dmax, 0.0));
    for (int j = 0; j < pa; ++j) {
        const double piv = R[j * pa + j];
        if (!(piv > 0.0) || !(sqrt(piv) > rel_tol * dmax)) return false;
        const double r = sqrt(piv);
        wave_sync();
        for (int c = j + t; c < pa; c += 64) R[j * pa + c] /= r;
        wave_sync();
        // trailing update of the upper triangle: rows rr > j, columns c >= rr
        const int m = pa - j - 1;
        for (int e = t; e < m * m; e += 64) {
            const int rr = j + 1 + e / m, c = j + 1 + e % m;
            if (c >= rr) R[rr * pa + c] -= R[j * pa + rr] * R[j * pa + c];
        }
        wave_sync();
    }
    for (int e = t; e < pa * pa; e += 64)
        if (e % pa < e / pa) R[e] = 0.0;
    wave_sync();
    return true;
}

// X = R^{-1} for upper triangular R (pa x pa, row-major, LDS): one lane per
// column, back substitution from the diagonal up
__device__ void tri_inv_upper_lds(const double *R, double *X, int pa)
{
    for (int c = threadIdx.x; c < pa; c += 64) {
        X[c * pa + c] = 1.0 / R[c * pa + c];
        for (int r = c - 1; r >= 0; --r) {
            double s = 0.0;
            for (int k = r + 1; k <= c; ++k) s += R[r * pa + k] * X[k * pa + c];
            X[r * pa + c] = -s / R[r * pa + r];
        }
        for (int r = c + 1; r < pa; ++r) X[r * pa + c] = 0.0;
    }
    wave_sync();
}

// Stage 1 (R1 from G1): X1 = R1^{-1} to X1 (pa x pa) and, zero-padded, to Xp
// (pap x pap), the right factor of Q1 = B X1.  Stage 2 (R2 from G2): Xp =
// P' with P = R2^{-1} R2^{-T} R1^{-T}, the right factor of B^+' = Q1 P.
// status: 0, or the stage whose rank test failed (stage 2 does nothing when
// stage 1 failed).  One wave.
__global__ __launch_bounds__(64) void small_factor_kernel(
    const double *__restrict__ G, int pa, int pap, double rel_tol, int stage,
    double *__restrict__ X1, double *__restrict__ Xp, int *__restrict__ status)
{
    __shared__ double A[kSmallFactorP * kSmallFactorP];
    __shared__ double Y[kSmallFactorP * kSmallFactorP];
    const int t = threadIdx.x;
    if (stage == 2 && *status != 0) return;
    for (int e = t; e < pa * pa; e += 64) A[e] = G[e];
    wave_sync();
    if (!chol_upper_lds(A, pa, rel_tol)) {
        if (t == 0) *status = stage;
        return;
    }
    tri_inv_upper_lds(A, Y, pa); // Y = R^{-1}
    if (stage == 1) {
        for (int e = t; e < pa * pa; e += 64) X1[e] = Y[e];
        for (int e = t; e < pap * pap; e += 64) {
            const int r = e / pap, c = e % pap;
            Xp[e] = (r < pa && c < pa) ? Y[r * pa + c] : 0.0;
        }
        if (t == 0) *status = 0;
        return;
    }
    // T2 = Y2 Y2' (upper factors: the sum starts at max(r, c)) into A
    for (int e = t; e < pa * pa; e += 64) {
        const int r = e / pa, c = e % pa;
        double v = 0.0;
        for (int k = max(r, c); k < pa; ++k) v += Y[r * pa + k] * Y[c * pa + k];
        A[e] = v;
    }
    wave_sync();
    for (int e = t; e < pa * pa; e += 64) Y[e] = X1[e];
    wave_sync();
    // Xp[r][c] = sum_k T2[r][k] X1[c][k] (X1 upper: k >= c)
    for (int e = t; e < pap * pap; e += 64) {
        const int r = e / pap, c = e % pap;
        double v = 0.0;
        if (r < pa && c < pa)
            for (int k = c; k < pa; ++k) v += A[r * pa + k] * Y[c * pa + k];
        Xp[e] = v;
    }
    if (t == 0) *status = 0;
}

hipError_t launch_small_factor(const double *G, int pa, int pap, double rel_tol,
                               int stage, double *X1, double *Xp, int *status,
                               hipStream_t s)
{
    if (pa > kSmallFactorP || pa < 1 || (stage != 1 && stage != 2))
        return hipErrorInvalidValue;
    small_factor_kernel<<<1, 64, 0, s>>>(G, pa, pap, rel_tol, stage, X1, Xp, status);
    return hipGetLastError();
}

hipError_t launch_basis_matrix(const double *pts, int n, int ld, int dp,
                               const int8_t *nu, int pa, int pap,
                               const double *mid, const double *scale,
                               double T, double *B, hipStream_t s)
{
    dim3 grid((ld + 255) / 256, pap);
    basis_matrix_kernel<<<grid, 256, 0, s>>>(pts, n, ld, dp, nu, pa, mid, scale, T, B);
    return hipGetLastError();
}

hipError_t launch_gram(const double *A, int ld, int pap, int rows_per_chunk,
                       int chunks, const int2 *pairs, int npairs,
                       double *partial, int pa, double *G, hipStream_t s)
{
    gram_partial_kernel<<<dim3(npairs, chunks), 64, 0, s>>>(A, ld, pap, rows_per_chunk,
                                                          pairs, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    gram_reduce_kernel<<<(pa * pa + 255) / 256, 256, 0, s>>>(partial, chunks, pap, pa, G);
    return hipGetLastError();
}

hipError_t launch_gemm_ax(const double *A, int ld, const double *X, int pap,
                          double *Y, int ldy, int nrows, const int *colmap,
                          int ncols, hipStream_t s, const int *skip)
{
    dim3 grid(ld / 64, (pap + 63) / 64);
    gemm_ax_kernel<<<grid, 64, 0, s>>>(A, ld, X, pap, Y, ldy, nrows, colmap, ncols, skip);
    return hipGetLastError();
}

} // namespace bsde
