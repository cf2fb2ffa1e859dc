// bsde_common.h -- definitions shared by the host set-up and the HIP kernels
// of the BSDE library: the counter-based generator, the compile-time index
// sets of the polynomial basis and the per-launch parameter block.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

namespace bsde {

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1, so
// that table reads indexed by I are constant expressions.
template <typename F, int... Is>
__host__ __device__ __forceinline__ void static_for_impl(
    F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}

template <int N, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int kMaxD = 10;
constexpr int kBlock = 256; // lanes per workgroup of the path kernel
// largest basis whose set-up factorisations run on the device (two
// kSmallFactorP^2 FP64 matrices in the LDS of one wave's workgroup)
constexpr int kSmallFactorP = 56;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter words:
// (path m, point i, iteration k, substream << 24 | block); key: the seed.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t x, y, z, w;
};

// one round: two 32x32->64 products, the high halves mixed with the other
// words and the round key, then the key bumped by the Weyl constants
__host__ __device__ __forceinline__ void philox_round(u32x4 &c, uint32_t &k0,
                                                      uint32_t &k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    c = {n0, (uint32_t)p1, n2, (uint32_t)p0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
}

__host__ __device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1,
                                                   uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1)
{
    u32x4 c{c0, c1, c2, c3};
#pragma unroll
    for (int r = 0; r < 10; ++r) philox_round(c, k0, k1);
    return c;
}

// ---------------------------------------------------------------------------
// Index set of the basis (Section 4.2, the hyperbolic sets of eq.
// hyper_set): {nu in N^{DP} : (sum_j nu_j^q)^{1/q} <= ETA} with q = Q / 10
// (Q = 10: the total-degree set |nu| <= ETA), graded, and within a degree
// lexicographically decreasing.  For every multi-index the table gives the
// "parent" obtained by zeroing its last non-zero entry (the sets are
// downward closed, so it is in the set), the variate of that entry and its
// degree: B_nu = B_parent * T_deg(z_var).
// ---------------------------------------------------------------------------
constexpr int binom(int n, int k)
{
    long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

// compile-time exp and log (series, to double rounding) for the q-norms
constexpr double c_exp(double x)
{
    int k = 0;
    while (x > 0.5 || x < -0.5) {
        x *= 0.5;
        ++k;
    }
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 30; ++i) {
        term *= x / i;
        sum += term;
    }
    for (int i = 0; i < k; ++i) sum *= sum;
    return sum;
}
constexpr double c_log(double x)
{
    int e = 0;
    while (x > 1.5) {
        x *= 0.5;
        ++e;
    }
    while (x < 0.75) {
        x *= 2.0;
        --e;
    }
    const double y = (x - 1.0) / (x + 1.0), y2 = y * y;
    double term = y, sum = 0.0;
    for (int i = 1; i < 80; i += 2) {
        sum += term / i;
        term *= y2;
    }
    return 2.0 * sum + e * 0.693147180559945309417232121458;
}
// n^(Q/10) for a non-negative integer n
constexpr double qpow(int n, int Q)
{
    return n == 0 ? 0.0 : Q == 10 ? (double)n : c_exp(Q / 10.0 * c_log((double)n));
}
template <int DP>
constexpr bool in_index_set(const int *nu, int eta, int Q)
{
    if (Q == 10) return true; // the total degree is bounded by the enumeration
    double s = 0.0;
    for (int v = 0; v < DP; ++v) s += qpow(nu[v], Q);
    return s <= qpow(eta, Q) * (1.0 + 1e-12);
}

// visits the multi-indices of total degree <= ETA in table order
template <int DP, int ETA, typename F>
constexpr void for_each_total_degree(F &&f)
{
    for (int g = 0; g <= ETA; ++g) {
        // odometer over compositions of g into DP parts, first part largest
        int cur[DP] = {};
        cur[0] = g;
        while (true) {
            f(cur);
            // next composition in lexicographically decreasing order
            int j = DP - 2;
            while (j >= 0 && cur[j] == 0) --j;
            if (j < 0) break;
            cur[j] -= 1;
            int rest = 0;
            for (int v = j + 1; v < DP; ++v) rest += cur[v];
            for (int v = j + 1; v < DP; ++v) cur[v] = 0;
            cur[j + 1] = rest + 1;
        }
    }
}

template <int DP, int ETA, int Q>
constexpr int index_set_size()
{
    int count = 0;
    for_each_total_degree<DP, ETA>([&](const int *nu) {
        if (in_index_set<DP>(nu, ETA, Q)) ++count;
    });
    return count;
}

template <int DP, int ETA, int Q>
struct IndexTable {
    static constexpr int P = index_set_size<DP, ETA, Q>();
    int8_t nu[P][DP];
    int16_t parent[P];
    int8_t var[P];
    int8_t deg[P];
};

template <int DP, int ETA, int Q>
constexpr IndexTable<DP, ETA, Q> make_index_table()
{
    IndexTable<DP, ETA, Q> t{};
    int count = 0;
    for_each_total_degree<DP, ETA>([&](const int *cur) {
        if (!in_index_set<DP>(cur, ETA, Q)) return;
        for (int v = 0; v < DP; ++v) t.nu[count][v] = (int8_t)cur[v];
        ++count;
    });
    for (int l = 0; l < t.P; ++l) {
        int last = -1;
        for (int v = 0; v < DP; ++v)
            if (t.nu[l][v]) last = v;
        if (last < 0) {
            t.parent[l] = -1;
            t.var[l] = 0;
            t.deg[l] = 0;
            continue;
        }
        int8_t want[DP] = {};
        for (int v = 0; v < DP; ++v) want[v] = t.nu[l][v];
        want[last] = 0;
        int par = -1;
        for (int m = 0; m < l; ++m) {
            bool eq = true;
            for (int v = 0; v < DP; ++v) eq = eq && (t.nu[m][v] == want[v]);
            if (eq) par = m;
        }
        t.parent[l] = (int16_t)par;
        t.var[l] = (int8_t)last;
        t.deg[l] = t.nu[l][last];
    }
    return t;
}

template <int DP, int ETA, int Q = 10>
struct Basis {
    static constexpr int P = IndexTable<DP, ETA, Q>::P;
    static constexpr IndexTable<DP, ETA, Q> tab = make_index_table<DP, ETA, Q>();
};

// number of derivative channels: u, d_t u, d d_x u, d(d+1)/2 d_xx u
__host__ __device__ constexpr int num_channels(int d)
{
    return 2 + d + d * (d + 1) / 2;
}

// the set-up's basis and Gram matrices have pad16(p) columns, zero beyond
// p, so that 16 x 16 matrix-core tiles read them in bounds
__host__ __device__ constexpr int pad16(int x) { return (x + 15) & ~15; }

// The channel table the path kernels read (FP64 and FP32 alike) holds the
// live rows of the p x C table packed (see channel_row_live) in three
// blocks: channel 0 over every row (p entries); each second-derivative
// channel over its live rows, channel after channel; then row after row the
// live entries of channels 1 .. 1 + d (the time derivative and the
// gradient), in channel order -- at most p C entries in all.
__host__ __device__ constexpr size_t table_entries(int p, int C)
{
    return (size_t)p * C;
}

// channel 2 + d + idx holds d^2 u / dx_j dx_k for the idx-th pair j <= k
// (row-major upper triangle)
__host__ __device__ constexpr int hess_j(int d, int idx)
{
    int j = 0;
    while (idx >= d - j) {
        idx -= d - j;
        ++j;
    }
    return j;
}
__host__ __device__ constexpr int hess_k(int d, int idx)
{
    int j = 0;
    while (idx >= d - j) {
        idx -= d - j;
        ++j;
    }
    return j + idx;
}

// The channel table Gamma = D alpha holds derivatives of u = sum_l alpha_l
// B_l (Section 4.2, the derivatives of the basis functions).  The
// derivative of a Chebyshev factor has lower degree (T_a' is a combination
// of the T_b with b < a and a - b odd), so over a downward-closed index set
// Lambda the row of basis function nu in channel c can be non-zero only if
// nu + e_v is in Lambda, c the derivative in variate v (v = 0 the time), or
// nu + e_v + e_w is, c the second derivative in v and w (v = w included).
// Channel 0, u itself, has every row.  in_set tests a multi-index (int[dp])
// for membership in Lambda.
template <int MAXDP, typename InSet>
__host__ __device__ constexpr bool channel_row_live(const int8_t *nu, int dp, int c,
                                                    const InSet &in_set)
{
    if (c == 0) return true;
    const int d = dp - 1;
    int mu[MAXDP] = {};
    for (int v = 0; v < dp; ++v) mu[v] = nu[v];
    if (c < 2 + d) {
        mu[c - 1] += 1; // c = 1: the time; c = 2 + j: x_j, variate 1 + j
    } else {
        mu[1 + hess_j(d, c - 2 - d)] += 1;
        mu[1 + hess_k(d, c - 2 - d)] += 1;
    }
    return in_set(mu);
}

// Membership in the kernel's index set {nu : |nu| <= ETA, sum_v nu_v^q <=
// ETA^q} (the same test as in_index_set, with the powers tabulated)
template <int DP, int ETA, int Q>
struct IndexSetTest {
    double qp[ETA + 3] = {};
    double lim = 0.0;
    constexpr IndexSetTest()
    {
        for (int n = 0; n < ETA + 3; ++n) qp[n] = qpow(n, Q);
        lim = qpow(ETA, Q) * (1.0 + 1e-12);
    }
    constexpr bool operator()(const int *mu) const
    {
        int g = 0;
        double s = 0.0;
        for (int v = 0; v < DP; ++v) {
            if (mu[v] > ETA) return false;
            g += mu[v];
            s += qp[mu[v]];
        }
        return g <= ETA && (Q == 10 || s <= lim);
    }
};

// Packed positions of the kernel's live rows (layout above): hpos[h][l] is
// the entry of row l in second-derivative channel 2 + d + h (-1: not
// live); row l of the last block holds entries goff[l] .. goff[l+1]-1, entry
// e of channel gch[e - goff[0]].
template <int DP, int ETA, int Q>
constexpr int channel_rows_count(int c_lo, int c_hi)
{
    using BS = Basis<DP, ETA, Q>;
    constexpr IndexSetTest<DP, ETA, Q> in_set{};
    int n = 0;
    for (int l = 0; l < BS::P; ++l)
        for (int c = c_lo; c < c_hi; ++c)
            n += channel_row_live<DP>(BS::tab.nu[l], DP, c, in_set) ? 1 : 0;
    return n;
}

template <int DP, int ETA, int Q>
struct ChannelRowTable {
    static constexpr int P = Basis<DP, ETA, Q>::P;
    static constexpr int D = DP - 1;
    static constexpr int NH = num_channels(D) - 2 - D; // second derivatives
    static constexpr int NG = channel_rows_count<DP, ETA, Q>(1, 2 + D);
    int16_t hpos[NH][P];
    int16_t goff[P + 1];
    uint8_t gch[NG];
};

template <int DP, int ETA, int Q>
constexpr ChannelRowTable<DP, ETA, Q> make_channel_rows()
{
    using BS = Basis<DP, ETA, Q>;
    using T = ChannelRowTable<DP, ETA, Q>;
    constexpr IndexSetTest<DP, ETA, Q> in_set{};
    T t{};
    int e = BS::P; // after channel 0
    for (int h = 0; h < T::NH; ++h)
        for (int l = 0; l < BS::P; ++l)
            t.hpos[h][l] = channel_row_live<DP>(BS::tab.nu[l], DP, 2 + T::D + h, in_set)
                               ? (int16_t)e++ : (int16_t)-1;
    const int g0 = e;
    for (int l = 0; l < BS::P; ++l) {
        t.goff[l] = (int16_t)e;
        for (int c = 1; c < 2 + T::D; ++c)
            if (channel_row_live<DP>(BS::tab.nu[l], DP, c, in_set)) t.gch[e++ - g0] = (uint8_t)c;
    }
    t.goff[BS::P] = (int16_t)e;
    return t;
}

template <int DP, int ETA, int Q = 10>
struct ChannelRows {
    static constexpr ChannelRowTable<DP, ETA, Q> tab = make_channel_rows<DP, ETA, Q>();
};

// ---------------------------------------------------------------------------
// Per-launch parameters of the path kernel (passed by value).
// ---------------------------------------------------------------------------
enum VolKind { kVolConst = 0, kVolBump = 1, kVolDupire = 2 };
enum PayoffKind {
    kPutArith = 0,
    kCallArith = 1,
    kPutGeom = 2,
    kCallGeom = 3,
    kFwdArith = 4,
    kQuad = 5
};

// Per-asset constants of the path kernel in the path precision, rounded
// once on the host: the kernel reads them as uniform scalar operands instead
// of converting them into vector registers.
template <typename Real>
struct AssetConsts {
    Real level[kMaxD];   // volatility level
    Real level_a[kMaxD]; // level x bump height
    Real drift[kMaxD];   // r - dividend
    Real mid[kMaxD];     // domain centre
    Real scale[kMaxD];   // 2 / (hi - lo)
    Real Ldiag[kMaxD];   // Cholesky diagonal L_jj
    Real Lcol[kMaxD];    // L_{j+1, j}: column j below the diagonal (constant)
    Real spot[kMaxD];    // S0_j: the smile centre of the Dupire-type volatility
};

struct PathParams {
    uint64_t seed;
    uint32_t k;          // Picard iteration (counter word 2)
    int M, N;            // paths per point, Euler steps
    int groups;          // workgroups per point
    int paths_per_lane;  // paths run by one lane
    int n;               // number of points
    int vol_kind, payoff;
    double r, omega, K, T;
    double level[kMaxD];
    double div[kMaxD];
    double bump_a, log_bump_c;
    double L[kMaxD * kMaxD];   // Cholesky factor, row-major lower
    double rho;
    double mid[kMaxD];         // domain centre
    double scale[kMaxD];       // 2 / (hi - lo)
    double spot[kMaxD];        // S0_j
    AssetConsts<float> cf;     // the per-asset constants in FP32
    AssetConsts<double> cd;    // and in FP64
    double kbw;                // kernel operator: bandwidth in z (0: least squares)
};

// Extrapolating operators: least squares on the polynomial basis, or the
// kernel operator of Section 3.2 (path kernels with OP = kOpKernel read a
// table of rows {z_0, .., z_d, y} of kKernelRow entries instead of Gamma)
enum { kOpBasis = 0, kOpKernel = 1 };
constexpr int kKernelRow = 4;
// weights beyond this exponent are constant (the clamp of the kernel)
constexpr double kKernelClamp = 60.0;

template <typename Real>
__host__ __device__ __forceinline__ const AssetConsts<Real> &asset_consts(const PathParams &p);
template <>
__host__ __device__ __forceinline__ const AssetConsts<float> &asset_consts<float>(const PathParams &p)
{
    return p.cf;
}
template <>
__host__ __device__ __forceinline__ const AssetConsts<double> &asset_consts<double>(const PathParams &p)
{
    return p.cd;
}

// fills cf and cd from the FP64 parameters (level, div, bump_a, mid,
// scale, L, spot and r must be set; d assets)
__host__ inline void fill_asset_consts(PathParams &p, int d)
{
    for (int j = 0; j < kMaxD; ++j) {
        const bool on = j < d;
        const double v[8] = {on ? p.level[j] : 0.0,
                             on ? p.level[j] * p.bump_a : 0.0,
                             on ? p.r - p.div[j] : 0.0,
                             on ? p.mid[j] : 0.0,
                             on ? p.scale[j] : 0.0,
                             on ? p.L[j * kMaxD + j] : 0.0,
                             j + 1 < d ? p.L[(j + 1) * kMaxD + j] : 0.0,
                             on ? p.spot[j] : 0.0};
        double *dd[8] = {p.cd.level, p.cd.level_a, p.cd.drift, p.cd.mid,
                         p.cd.scale, p.cd.Ldiag, p.cd.Lcol, p.cd.spot};
        float *ff[8] = {p.cf.level, p.cf.level_a, p.cf.drift, p.cf.mid,
                        p.cf.scale, p.cf.Ldiag, p.cf.Lcol, p.cf.spot};
        for (int c = 0; c < 8; ++c) {
            dd[c][j] = v[c];
            ff[c][j] = (float)v[c];
        }
    }
}

// One problem of a batched launch (see batch_path_kernel).
struct BatchTileDesc {
    PathParams prm;        // prm.k is the problem's own iteration
    const double *pts;     // n x (d+1) points
    const void *gamma;     // channel table (float or double)
    double *partial;       // n x groups x 2 sums
};

// Count, mean and sum of squared deviations of two sets of samples
// combined into those of their union (the pairwise update of Chan, Golub and
// LeVeque): with d = mean_b - mean_a and n = n_a + n_b,
// mean = mean_a + d n_b / n, M2 = M2_a + M2_b + d^2 n_a n_b / n.  Both sums of
// squares stay sums of squared deviations from a mean, so the variance does
// not come from the difference of two large sums.
__host__ __device__ inline void combine_moments(double &n, double &mean, double &m2,
                                                double nb, double meanb, double m2b)
{
    if (nb == 0.0) return;
    if (n == 0.0) {
        n = nb;
        mean = meanb;
        m2 = m2b;
        return;
    }
    const double nt = n + nb;
    const double d = meanb - mean;
    const double f = nb / nt;
    mean = __builtin_fma(d, f, mean);
    m2 = __builtin_fma(d * d, n * f, m2 + m2b);
    n = nt;
}

// One problem of the batched reduction / update kernels (one iteration).
struct BatchUpdateDesc {
    const double *partial; // n x groups x 2: mean and M2 of each group's paths
    int n, groups, M, p;
    int ppg;               // paths per group (256 x paths per lane)
    int nnz;               // entries of the packed channel table
    double *c, *var;       // this iteration's slices
    const double *W;       // p x n pseudo-inverse
    double *beta;          // p
    const double *alpha_in;
    double *alpha_out;
    const int *rowptr;     // the channel update (sparse rows of the packed table)
    const int *cols;
    const double *vals;
    double *g64;
    float *g32;            // FP32 table
};

} // namespace bsde
