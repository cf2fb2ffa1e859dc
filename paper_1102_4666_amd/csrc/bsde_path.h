// bsde_path.h -- the Monte Carlo path kernel of one Picard iteration of
// Algorithm "algodetail" (Labart & Lelong, arXiv:1102.4666, Section 4.1),
// templated on the dimension d, the basis degree eta and the path precision.
// Instantiated per dimension in bsde_inst_d*.hip.
//
//   a_m for every (point i, path m): Philox4x32-10 normals in registers,
//   Box-Muller, Euler scheme of the log-price (eq. 4) with coefficients
//   frozen at the last node (eq. eqs3), the interpolated state at the random
//   time tau = t_i + (T - t_i) U (eq. psiN), the Chebyshev basis row at
//   (tau, X_tau) contracted with the derivative channels of u^k, the
//   penalised driver (eq. bsde-penal-2) and the frozen generator; per-lane
//   FP64 sums reduced through wavefront shuffles and LDS in a fixed order.
#pragma once

#include "bsde_common.h"
#include "bsde_f64_math.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace bsde {

// The FP64 kernels' tables of sines, cosines and powers of two
// (bsde_f64_math.h), one copy per workgroup, filled at the start of each
// tile (run_tile).
static __shared__ f64::Tables f64_tables;

// ---------------------------------------------------------------------------
// Precision-specific arithmetic.  FP32: hardware transcendentals (v_log_f32
// is log2, v_sin/v_cos take revolutions); FP64: the device math library.
// ---------------------------------------------------------------------------
template <typename Real>
struct Arith;

template <>
struct Arith<float> {
    static __device__ __forceinline__ float u01(uint32_t w)
    {
        return fmaf((float)w, 0x1p-32f, 0x1p-33f); // (w + 1/2) 2^-32
    }
    // Box-Muller pair scaled by sqrt(v): R = sqrt(-2 v ln ua), computed as
    // sqrt((-2 ln2 v) log2 ua); angle 2 pi ub (v_sin/v_cos take revolutions)
    static __device__ __forceinline__ float bm_scale(float v)
    {
        return -1.38629436111989061883f * v;
    }
    // c32, c33: 2^-32 and 2^-33 of u01, passed in so that the caller can
    // hold them in vector registers
    static __device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb,
                                                      float scale, float &n0,
                                                      float &n1, float c32 = 0x1p-32f,
                                                      float c33 = 0x1p-33f)
    {
        const float ua = fmaf((float)wa, c32, c33);
        float R = __builtin_amdgcn_sqrtf(scale * __builtin_amdgcn_logf(ua));
        // angle: 1 + (top 23 bits of wb) 2^-23 in [1, 2) revolutions, built
        // by one funnel shift that puts the exponent of 1.0 above them
        // (sine and cosine have period one revolution)
        const float ub = __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, wb, 9u));
        n0 = R * __builtin_amdgcn_cosf(ub);
        n1 = R * __builtin_amdgcn_sinf(ub);
    }
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
    static __device__ __forceinline__ float exp_nonpos(float x) { return __expf(x); }
    static __device__ __forceinline__ float sqrt(float x)
    {
        return __builtin_amdgcn_sqrtf(x); // v_sqrt_f32, no refinement
    }
    static __device__ __forceinline__ float frac33(uint64_t num)
    {
        // (num mod 2^33) 2^-33 from the top 32 of the low 33 bits
        return (float)(uint32_t)((num & 0x1FFFFFFFFull) >> 1) * 0x1p-32f;
    }
};

template <>
struct Arith<double> {
    static __device__ __forceinline__ double u01(uint32_t w)
    {
        return ((double)w + 0.5) * 0x1p-32;
    }
    static __device__ __forceinline__ double bm_scale(double v)
    {
        return -2.0 * v;
    }
    // Box-Muller pair scaled by sqrt(v), scale = -2 v: R = sqrt(-2 v ln ua);
    // ln ua and the sine and cosine of the angle 2 pi ub from the words
    // themselves (bsde_f64_math.h)
    static __device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb,
                                                      double scale, double &n0,
                                                      double &n1, double = 0.0,
                                                      double = 0.0)
    {
        double R = f64::sqrt_nonneg(scale * f64::log_word(wa));
        double s, c;
        f64::sincos_turn_tab(wb, f64_tables, s, c);
        n0 = R * c;
        n1 = R * s;
    }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    // e^x for x <= 0 (the volatilities' Gaussian factors)
    static __device__ __forceinline__ double exp_nonpos(double x)
    {
        return f64::exp_nonpos_tab(x, f64_tables);
    }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double frac33(uint64_t num)
    {
        return (double)(num & 0x1FFFFFFFFull) * 0x1p-33;
    }
};

// Time factors of the Dupire-type volatility of eq. vol_locale, uniform
// across the paths of a point at one Euler step: with S = e^x,
// sigma(t, S) = A(t) - B(t) e^{-0.001 (S e^{r t} - s)^2}, A = 0.72 e^{-0.05
// sqrt t}, B = 0.6 e^{-0.1 t} e^{-0.05 sqrt t}, rt = r t.
template <typename Real>
struct VolTime {
    Real A, B, rt;
};
template <int VOL, typename Real>
__device__ __forceinline__ VolTime<Real> vol_time(Real t, Real r)
{
    VolTime<Real> v{Real(0), Real(0), Real(0)};
    if constexpr (VOL == kVolDupire) {
        const Real damp = Arith<Real>::exp(Real(-0.05) * Arith<Real>::sqrt(t));
        v.A = Real(0.72) * damp;
        v.B = Real(0.6) * damp * Arith<Real>::exp(Real(-0.1) * t);
        v.rt = r * t;
    }
    return v;
}

// sigma_j of log-price x: constant; bump level (1 + a e^{-(x - log c)^2})
// = level + (level a) e^{...}; or the Dupire-type form above
template <int VOL, typename Real>
__device__ __forceinline__ Real local_vol(Real level, Real level_a, Real lc,
                                          Real spot, const VolTime<Real> &vt,
                                          Real x)
{
    if constexpr (VOL == kVolBump) {
        Real dx = x - lc;
        return fma(level_a, Arith<Real>::exp_nonpos(-dx * dx), level);
    } else if constexpr (VOL == kVolDupire) {
        const Real dev = Arith<Real>::exp(x + vt.rt) - spot;
        return fma(-vt.B, Arith<Real>::exp_nonpos(Real(-0.001) * dev * dev), vt.A);
    }
    return level;
}

// Coordinates of the Euler state.  With the bump volatility the paths carry
// y = kappa (x - log c) -- kappa^2 = log2 e in FP32, 256 log2 e in FP64 at
// d = 10, 1 in the other FP64 kernels -- so that the volatility costs a
// square, one exponential and one fused multiply-add per asset and step:
// level + (level a) 2^{-y^2} (FP32), level + (level a) 2^{-y^2/256} (FP64,
// d = 10: the table exponential needs no reduction by ln 2), level +
// (level a) e^{-y^2} (other FP64; there the scaled form saves nothing: the
// vector instruction it takes off the volatility comes back as 64-bit
// literal moves in the rest of the step).  Every increment of x is scaled
// by kappa as well.  The other volatility kinds keep y = x.
template <int VOL, typename Real, int D>
struct EulerState {
    static constexpr bool kShift = VOL == kVolBump;
    static constexpr bool kExp2F64 = kShift && sizeof(Real) == 8 && D >= 10;
    static constexpr Real kappa =
        !kShift ? Real(1)
                : (sizeof(Real) == 4 ? Real(1.2011224087864498)
                                     : (kExp2F64 ? Real(19.217958540583197) : Real(1)));
    static __device__ __forceinline__ Real to(Real x, Real lc)
    {
        if constexpr (kShift) return (x - lc) * kappa;
        else return x;
    }
    static __device__ __forceinline__ Real from(Real y, Real lc)
    {
        if constexpr (kShift) return fma(y, Real(1) / kappa, lc);
        else return y;
    }
    static __device__ __forceinline__ Real vol(Real level, Real level_a, Real spot,
                                               const VolTime<Real> &vt, Real y)
    {
        if constexpr (kShift) {
            if constexpr (sizeof(Real) == 4)
                return fmaf(level_a, __builtin_amdgcn_exp2f(-y * y), level);
            else if constexpr (kExp2F64)
                return fma(level_a, f64::exp2_neg_tab(y * y, f64_tables), level);
            else
                return fma(level_a, f64::exp_nonpos_tab(-y * y, f64_tables), level);
        } else {
            return local_vol<VOL>(level, level_a, Real(0), spot, vt, y);
        }
    }
};

template <int D, typename Real>
__device__ __forceinline__ Real payoff(int kind, Real K, const Real *x)
{
    Real s = 0;
    if (kind == kPutArith || kind == kCallArith || kind == kFwdArith) {
#pragma unroll
        for (int j = 0; j < D; ++j) s += Arith<Real>::exp(x[j]);
        s *= Real(1.0 / D);
    } else {
#pragma unroll
        for (int j = 0; j < D; ++j) s += x[j];
        if (kind == kQuad) return s * s;
        s = Arith<Real>::exp(s * Real(1.0 / D));
    }
    switch (kind) {
    case kPutArith:
    case kPutGeom: return fmax(K - s, Real(0));
    case kCallArith:
    case kCallGeom: return fmax(s - K, Real(0));
    default: return s - K; // kFwdArith
    }
}

// Chebyshev values T_0..T_ETA of z
template <int ETA, typename Real>
__device__ __forceinline__ void cheb(Real z, Real *Tz)
{
    Tz[0] = Real(1);
    if (ETA >= 1) Tz[1] = z;
#pragma unroll
    for (int a = 1; a < ETA; ++a) Tz[a + 1] = Real(2) * z * Tz[a] - Tz[a - 1];
}

// One Philox4x32-10 round in the path kernel (the function of philox_round).
// Bit 0 / bit 1 of X3 select, for the new word 0 / word 2, the three-way
// XOR (high half ^ counter word ^ key) as one v_bitop3_b32 with truth table
// 0x96 (a ^ b ^ c) instead of two v_xor_b32.  That pays only where the
// counter word varies across the wave: with a uniform counter word the two
// uniform operands combine on the scalar unit and leave one vector XOR,
// while v_bitop3_b32 (one scalar operand at most) would need a move too.
template <int X3>
__device__ __forceinline__ void philox_round_dev(u32x4 &c, uint32_t &k0, uint32_t &k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t h1 = (uint32_t)(p1 >> 32), h0 = (uint32_t)(p0 >> 32);
    const uint32_t n0 = (X3 & 1) ? __builtin_amdgcn_bitop3_b32(h1, c.y, k0, 0x96)
                                 : h1 ^ c.y ^ k0;
    const uint32_t n2 = (X3 & 2) ? __builtin_amdgcn_bitop3_b32(h0, c.w, k1, 0x96)
                                 : h0 ^ c.w ^ k1;
    c = {n0, (uint32_t)p1, n2, (uint32_t)p0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
}

// One Philox4x32-10 block in the path kernel (the same function as
// philox10) on the counter (m, i, k, word 3): m varies across the wave, the
// other three words are uniform.  Rounds 1 and 2 keep their hoistable work
// on the uniform words; after round 2 only word 3 is still uniform, and from
// round 4 on every word varies, so with kXor3 round 3 takes the three-input
// XOR for word 0 and rounds 4-10 for both.  All kernels but the FP64 d = 1
// ones take it (10 fewer of the ~53 vector instructions of a block; the
// d = 10 launches 3-5% faster); the FP64 d = 1 kernels keep the two-XOR
// form, under which they fit 128 registers (four waves per SIMD).
// After the second round the key passes through an empty asm statement, so
// that the keys of rounds 3-10, k + r (W0, W1), are formed on the scalar
// unit per block instead of being hoisted out of the path loops, where
// sixteen of them would stay live in scalar registers (at d >= 5 the
// compiler parks the excess in vector-register lanes and reads it back with
// one vector instruction per use).
// Keys of rounds 3-10, k + r (W0, W1) for r = 2..9, held in vector
// registers: v_bitop3_b32 with all three operands in vector registers
// issues in about three cycles instead of four.
struct PhiloxKeys {
    uint32_t a[8], b[8];
};

__device__ __forceinline__ PhiloxKeys philox_vector_keys(uint32_t k0, uint32_t k1)
{
    PhiloxKeys kv;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        kv.a[r] = k0 + (uint32_t)(r + 2) * 0x9E3779B9u;
        kv.b[r] = k1 + (uint32_t)(r + 2) * 0xBB67AE85u;
        asm volatile("" : "+v"(kv.a[r]), "+v"(kv.b[r]));
    }
    return kv;
}

template <bool kXor3>
__device__ __forceinline__ u32x4 philox_block(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1)
{
    u32x4 c{c0, c1, c2, c3};
    philox_round_dev<0>(c, k0, k1);
    philox_round_dev<0>(c, k0, k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
    philox_round_dev<kXor3 ? 1 : 0>(c, k0, k1);
#pragma unroll
    for (int r = 3; r < 10; ++r) philox_round_dev<kXor3 ? 3 : 0>(c, k0, k1);
    return c;
}

// The same block with the keys of rounds 3-10 taken from vector registers
// (every XOR of those rounds one v_bitop3_b32; in round 3 the uniform word
// 3 is its one scalar operand).
__device__ __forceinline__ u32x4 philox_block(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1,
                                              const PhiloxKeys &kv)
{
    u32x4 c{c0, c1, c2, c3};
    philox_round_dev<0>(c, k0, k1);
    philox_round_dev<0>(c, k0, k1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        uint32_t ka = kv.a[r], kb = kv.b[r];
        philox_round_dev<3>(c, ka, kb);
    }
    return c;
}

// The per-asset constants of a launch as a constant-address-space object
// at the uniform address cbase of its PathParams (the kernel-argument
// segment, or the batch's descriptor table), through an address the
// compiler cannot see through, so that their scalar loads are issued where
// they are used instead of being hoisted out of the loop.
template <typename Real>
using ConstAssets = const __attribute__((address_space(4))) AssetConsts<Real>;

template <typename Real>
__device__ __forceinline__ ConstAssets<Real> &reload_consts(uint64_t cbase)
{
    uint64_t a = cbase + (sizeof(Real) == 8 ? offsetof(PathParams, cd)
                                            : offsetof(PathParams, cf));
    asm volatile("" : "+s"(a));
    return *(ConstAssets<Real> *)a;
}

// ---------------------------------------------------------------------------
// The Monte Carlo path kernel.
// Grid: n * groups workgroups of kBlock lanes; workgroup (i, g) runs the
// paths m = (g * ppl + r) * kBlock + lane, r < ppl, m < M, of point i and
// writes the mean and the sum of squared deviations of its FP64 path terms
// to partial[2 (i groups + g)].
// ---------------------------------------------------------------------------
// Gamma is read-only, uniform across the workgroup and read once per basis
// function and channel per path: its loads must stay scalar (SGPR) loads,
// so GammaPtr is a global restrict pointer or a constant-address-space one.
template <int D, int ETA, typename Real, int VOL, int Q, typename GammaPtr,
          int OP = kOpBasis, bool RELOAD = false>
__device__ __forceinline__ void run_tile(const PathParams &prm, uint64_t cbase,
                                         const double *__restrict__ pts,
                                         GammaPtr gamma, const int i,
                                         const int g, double *__restrict__ out)
{
    constexpr int DP = D + 1;
    [[maybe_unused]] constexpr int C = num_channels(D);
    using BS = Basis<DP, ETA, Q>;
    constexpr int NP = BS::P;
    // steps per group so that a group uses whole Philox blocks
    constexpr int SG = (D % 4 == 0) ? 1 : ((D % 2 == 0) ? 2 : 4);
    constexpr int NB = SG * D / 4;
    constexpr int NBB = (D + 3) / 4; // bridge blocks
    constexpr bool kXor3 = sizeof(Real) == 4 || D >= 2; // Philox XOR form
    // FP32 round keys in vector registers (16 of them): at d = 1, and at
    // d = 2 from eta = 5 on, where the kernel's own registers already hold
    // it to four waves per SIMD and the keys still fit (below, they would
    // cost waves).  Not in the kernel operator, whose pair loop, not the
    // Euler loop, sets the time and which would lose waves.
    constexpr bool kVKeys = sizeof(Real) == 4 && OP == kOpBasis &&
                            (D == 1 || (D == 2 && ETA >= 5));

    const uint32_t k0 = (uint32_t)prm.seed, k1 = (uint32_t)(prm.seed >> 32);
    PhiloxKeys kv{};
    if constexpr (kVKeys) kv = philox_vector_keys(k0, k1);
    auto block = [&](uint32_t m, uint32_t w3) -> u32x4 {
        if constexpr (kVKeys) return philox_block((uint32_t)m, (uint32_t)i, prm.k, w3, k0, k1, kv);
        else return philox_block<kXor3>((uint32_t)m, (uint32_t)i, prm.k, w3, k0, k1);
    };

    const double *row = pts + (size_t)i * DP;
    const Real T = (Real)prm.T;
    const Real t0 = (Real)row[0];
    const Real h = (T - t0) / (Real)prm.N;
    // Euler state coordinates y = kappa (x - off); step normals come out of
    // Box-Muller already scaled by kappa sqrt(h)
    using ES = EulerState<VOL, Real, D>;
    const Real step_scale = Arith<Real>::bm_scale(h * (ES::kappa * ES::kappa));
    const Real r = (Real)prm.r, omega = (Real)prm.omega, K = (Real)prm.K;
    const Real lc = (Real)prm.log_bump_c;
    const Real rho = (Real)prm.rho;
    // per-asset constants, read as uniform scalars where they are used.
    // The Cholesky factor of the uniform correlation rho 11' + (1 - rho) I
    // has columns constant below the diagonal (Lcol[k] = L[j][k], j > k),
    // so (L G)_j = S_j + L_jj G_j with S_{j+1} = S_j + Lcol[j] G_j -- the
    // terms of sum_k L_jk G_k in the same order, O(d) instead of O(d^2)
    const AssetConsts<Real> &ac = asset_consts<Real>(prm);
    // FP64 one-problem kernels read the per-asset constants of the Euler
    // step again for every group of steps (RELOAD; cbase is then the
    // address of prm in constant memory)
    constexpr bool kReloadConsts = RELOAD && sizeof(Real) == 8;
    const Real tscale = Real(2) / T;
    const Real neg_half_hk = Real(-0.5) * ES::kappa * h;
    const Real hk = ES::kappa * h;
    // The volatility levels as vector operands: the volatility's fused
    // multiply-add has another scalar operand (level a) already, and a
    // second one costs a register move per asset and step.  At d = 10 the
    // vector registers are the scarcer ones (the moves are cheaper than the
    // spills that ten more live registers cause).
    Real lev[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lev[j] = ac.level[j];
        if constexpr (D <= 5) asm volatile("" : "+v"(lev[j]));
    }
    // gfx950 issues a 32-bit vector instruction whose operands are all
    // vector registers in two cycles, one with a scalar or literal operand
    // in four.  The FP32 kernels up to d = 5 therefore also hold the other
    // loop-invariant operands of the Euler step (level a, (r - delta) h
    // kappa) and the constants of the uniform map in vector registers.
    constexpr bool kVecConst = sizeof(Real) == 4 && D <= 5;
    Real lva[D], dhk[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lva[j] = ac.level_a[j];
        dhk[j] = ac.drift[j] * hk;
        if constexpr (kVecConst) asm volatile("" : "+v"(lva[j]), "+v"(dhk[j]));
    }
    Real c32 = Real(0x1p-32), c33 = Real(0x1p-33);
    if constexpr (kVecConst) asm volatile("" : "+v"(c32), "+v"(c33));
    // X and the normals G at the step j* of each path: written to LDS by
    // the one step that matches, a store under the lane mask, where a
    // select in every step would take two vector-ALU slots per asset
    struct alignas(2 * sizeof(Real)) Rec {
        Real y, g;
    };
    __shared__ Rec rec[D][kBlock];

    if constexpr (sizeof(Real) == 8) {
        f64::fill_tables(f64_tables, (int)threadIdx.x, kBlock);
        __syncthreads();
    }

    // this lane's paths: count, mean and sum of squared deviations, updated
    // path by path (Welford), so the sum of squares never dwarfs the spread
    int cnt = 0;
    double mean = 0.0, m2 = 0.0;
    for (int rr = 0; rr < prm.paths_per_lane; ++rr) {
        int m = (g * prm.paths_per_lane + rr) * kBlock + (int)threadIdx.x;
        const bool valid = m < prm.M;
        if (!valid) break;

        // U, j* = floor(U N) and theta = U N - j* in integer arithmetic
        const u32x4 wu = block((uint32_t)m, 1u << 24);
        const uint64_t num = (2ull * wu.x + 1ull) * (uint64_t)prm.N;
        const int jstar = (int)(num >> 33);
        const Real theta = Arith<Real>::frac33(num);
        const Real U = Arith<Real>::u01(wu.x);
        const Real tau = t0 + (T - t0) * U;

        Real X[D];
#pragma unroll
        for (int j = 0; j < D; ++j) X[j] = ES::to((Real)row[1 + j], lc);
        const int ngroups = (prm.N + SG - 1) / SG;
        for (int grp = 0; grp < ngroups; ++grp) {
            // FP64: the per-asset constants of the step are read again for
            // every group of steps through an address the compiler cannot
            // see through (scalar loads from the constant cache); held
            // across the loop they overflow the scalar registers and come
            // back from vector-register lanes with one vector instruction
            // per use
            Real G[4 * NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const u32x4 w = block((uint32_t)m, (uint32_t)(grp * NB + b));
                Arith<Real>::box_muller(w.x, w.y, step_scale, G[4 * b],
                                        G[4 * b + 1], c32, c33);
                Arith<Real>::box_muller(w.z, w.w, step_scale, G[4 * b + 2],
                                        G[4 * b + 3], c32, c33);
            }
            auto steps = [&](auto &acs) {
#pragma unroll
            for (int ss = 0; ss < SG; ++ss) {
                const int s = grp * SG + ss;
                if (s < prm.N) {
                    if (s == jstar) {
#pragma unroll
                        for (int j = 0; j < D; ++j)
                            rec[j][threadIdx.x] = Rec{X[j], G[ss * D + j]};
                    }
                    const VolTime<Real> vt = vol_time<VOL>(t0 + Real(s) * h, r);
                    Real S = Real(0);
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        // kappa sqrt(h) (L G)_j; the first row of the Cholesky
                        // factor of a correlation matrix is (1, 0, ..., 0)
                        Real lg = G[ss * D];
                        if (j > 0) lg = fma(acs.Ldiag[j], G[ss * D + j], S);
                        if (j + 1 < D) S = j == 0 ? acs.Lcol[0] * G[ss * D]
                                                  : fma(acs.Lcol[j], G[ss * D + j], S);
                        const Real sig = ES::vol(lev[j],
                                                 kReloadConsts ? acs.level_a[j] : lva[j],
                                                 acs.spot[j], vt, X[j]);
                        // X += (r - delta - sigma^2/2) h + sigma sqrt(h) (L G)
                        //    = X + (r - delta) h + sigma (sqrt(h) (L G) - h sigma / 2),
                        // every term times kappa
                        const Real inner = fma(sig, fma(neg_half_hk, sig, lg), X[j]);
                        if constexpr (kVecConst) X[j] = inner + dhk[j];
                        else X[j] = fma(acs.drift[j], hk, inner);
                    }
                }
            }
            };
            if constexpr (kReloadConsts) steps(reload_consts<Real>(cbase));
            else steps(ac);
        }

        // frozen coefficients at the last node t_{j*} and X at tau: the
        // bridge normals are scaled by sqrt(theta (1 - theta) h)
        const Real bridge_scale =
            Arith<Real>::bm_scale(theta * (Real(1) - theta) * h);
        Real Gb[4 * NBB];
#pragma unroll
        for (int b = 0; b < NBB; ++b) {
            const u32x4 w = block((uint32_t)m, (1u << 24) | (uint32_t)(1 + b));
            Arith<Real>::box_muller(w.x, w.y, bridge_scale, Gb[4 * b],
                                    Gb[4 * b + 1]);
            Arith<Real>::box_muller(w.z, w.w, bridge_scale, Gb[4 * b + 2],
                                    Gb[4 * b + 3]);
        }
        // back to x: the state at T and at t_{j*} with sqrt(h) (L G) of the
        // step j* (every j* < N is a step of the path, so each lane has
        // written its own record)
        Real Xs[D], LGs[D];
        {
            Real Sr = Real(0);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const Rec rj = rec[j][threadIdx.x];
                Xs[j] = ES::from(rj.y, lc);
                Real lg = rj.g;
                if (j > 0) lg = fma(ac.Ldiag[j], rj.g, Sr);
                if (j + 1 < D) Sr = j == 0 ? ac.Lcol[0] * rj.g : fma(ac.Lcol[j], rj.g, Sr);
                LGs[j] = lg * (Real(1) / ES::kappa);
                X[j] = ES::from(X[j], lc);
            }
        }
        Real sgs[D], bst[D], Xt[D];
        Real Sb = Real(0);
        const VolTime<Real> vts = vol_time<VOL>(t0 + Real(jstar) * h, r);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            Real lgb = Gb[0];
            if (j > 0) lgb = fma(ac.Ldiag[j], Gb[j], Sb);
            if (j + 1 < D) Sb = j == 0 ? ac.Lcol[0] * Gb[0] : fma(ac.Lcol[j], Gb[j], Sb);
            sgs[j] = local_vol<VOL>(ac.level[j], ac.level_a[j], lc, ac.spot[j], vts,
                                    Xs[j]);
            bst[j] = fma(Real(-0.5) * sgs[j], sgs[j], ac.drift[j]);
            Xt[j] = Xs[j] + bst[j] * theta * h +
                    sgs[j] * fma(theta, LGs[j], lgb);
        }

        // basis row at (tau, X_tau) contracted with the channel table, and
        // the value u^k(T, X_T) (z_0 = 1 there, so every T_a(z_0) = 1)
        Real Tz[DP][ETA + 1], TzT[DP][ETA + 1];
        cheb<ETA>(tau * tscale - Real(1), Tz[0]);
#pragma unroll
        for (int a = 0; a <= ETA; ++a) TzT[0][a] = Real(1);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            cheb<ETA>((Xt[j] - ac.mid[j]) * ac.scale[j], Tz[1 + j]);
            cheb<ETA>((X[j] - ac.mid[j]) * ac.scale[j], TzT[1 + j]);
        }
        // payoff at tau (for the penalty) and the terminal term
        // Phi(X_T) - u^k(T, X_T)
        Real phi_tau = payoff<D>(prm.payoff, K, Xt);
        Real u = Real(0), gen = Real(0), uT = Real(0), terminal;
        if constexpr (OP == kOpKernel) {
            // u^k = h[y] of the kernel operator (Section 3.2) in its
            // normalised form h = S1 / S0, S0 = sum_i w_i, S1 = sum_i y_i w_i,
            // w_i = exp(-min(|z - z_i|^2 / (2 b^2), clamp)) in the mapped
            // coordinates z; a clamped weight is constant (no derivative).
            // With L the frozen generator (d_t + b*.grad + sum_jk a_jk d_jk,
            // a_jk = sigma*_j sigma*_k C_jk / 2), in z units,
            //   L h = [L S1 - h L S0 - 2 sum_jk a_jk d_j h d_k S0] / S0,
            //   d_j h = (d_j S1 - h d_j S0) / S0,
            // and L w_i / w_i = l(dz), the polynomial below.  The table rows
            // {z_0, .., z_d, y} are uniform across the workgroup (scalar loads).
            const Real b2 = Real(prm.kbw * prm.kbw);
            const Real invb2 = Real(1) / b2;
            // FP32: the exponent in base 2 (log2 e folded into the scale and
            // the clamp), so that a weight is one v_exp_f32
            constexpr bool kF32 = sizeof(Real) == 4;
            const Real kq = Real(0.5 / (prm.kbw * prm.kbw) * (kF32 ? 1.4426950408889634 : 1.0));
            const Real clamp = Real(kKernelClamp * (kF32 ? 1.4426950408889634 : 1.0));
            auto weight = [&](Real e) {
                if constexpr (kF32) return __builtin_amdgcn_exp2f(-fminf(e, clamp));
                else return ::exp(-fmin(e, clamp));
            };
            Real zt[DP], zT[DP];
            zt[0] = tau * tscale - Real(1);
            zT[0] = Real(1);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                zt[1 + j] = (Xt[j] - ac.mid[j]) * ac.scale[j];
                zT[1 + j] = (X[j] - ac.mid[j]) * ac.scale[j];
            }
            // l(dz) = c0 + ct dz_0 + sum_j cj dz_j + sum_{j<=k} cjk dz_j dz_k
            Real ajk[D][D];
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int k = 0; k < D; ++k)
                    ajk[j][k] = Real(0.5) * sgs[j] * sgs[k] * (j == k ? Real(1) : rho) *
                                ac.scale[j] * ac.scale[k];
            const Real ct = -tscale * invb2;
            Real cj[D], cjk[D][D], c0 = Real(0);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                cj[j] = -bst[j] * ac.scale[j] * invb2;
                c0 -= ajk[j][j] * invb2;
#pragma unroll
                for (int k = j; k < D; ++k)
                    cjk[j][k] = (j == k ? ajk[j][j] : Real(2) * ajk[j][k]) * invb2 * invb2;
            }
            Real S0 = 0, S1 = 0, L0 = 0, L1 = 0, S0T = 0, S1T = 0;
            Real G0[D], G1[D]; // sum w dz_j and sum y w dz_j (unclamped weights)
#pragma unroll
            for (int j = 0; j < D; ++j) G0[j] = G1[j] = Real(0);
#pragma unroll 4
            for (int q = 0; q < prm.n; ++q) {
                const auto row = gamma + (size_t)q * kKernelRow;
                Real dz[DP], qq = Real(0), qT = Real(0);
#pragma unroll
                for (int v = 0; v < DP; ++v) {
                    dz[v] = zt[v] - row[v];
                    qq = fma(dz[v], dz[v], qq);
                    const Real dT = zT[v] - row[v];
                    qT = fma(dT, dT, qT);
                }
                const Real y = row[1 + D];
                const Real e = qq * kq;
                const bool flat = e > clamp;
                const Real w = weight(e);
                const Real wy = w * y;
                S0 += w;
                S1 += wy;
                const Real wd = flat ? Real(0) : w, wyd = flat ? Real(0) : wy;
                Real l = fma(ct, dz[0], c0);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    l = fma(cj[j], dz[1 + j], l);
#pragma unroll
                    for (int k = j; k < D; ++k) l = fma(cjk[j][k], dz[1 + j] * dz[1 + k], l);
                    G0[j] = fma(wd, dz[1 + j], G0[j]);
                    G1[j] = fma(wyd, dz[1 + j], G1[j]);
                }
                L0 = fma(wd, l, L0);
                L1 = fma(wyd, l, L1);
                const Real wT = weight(qT * kq);
                S0T += wT;
                S1T = fma(wT, y, S1T);
            }
            u = S1 / S0;
            // d_j S = -G_j / b^2 (z units), d_j h = (d_j S1 - h d_j S0) / S0
            Real hj[D];
#pragma unroll
            for (int j = 0; j < D; ++j) hj[j] = -(G1[j] - u * G0[j]) * invb2 / S0;
            Real acc = L1 - u * L0;
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int k = 0; k < D; ++k)
                    acc -= Real(2) * ajk[j][k] * hj[j] * (-G0[k] * invb2);
            gen = acc / S0;
            uT = S1T / S0T;
            terminal = payoff<D>(prm.payoff, K, X) - uT;
        } else {
            if constexpr (D >= 5) asm volatile("" : "+v"(phi_tau));
            // basis function l as the product of its non-zero Chebyshev
            // factors (at most eta of them), so that no earlier basis value
            // has to stay live in registers
            auto basis = [&](auto lc, const Real(&Tv)[DP][ETA + 1]) {
                constexpr int l = decltype(lc)::value;
                Real v = Real(1);
                static_for<DP>([&](auto vc) {
                    constexpr int w = decltype(vc)::value;
                    constexpr int e = BS::tab.nu[l][w];
                    if constexpr (e > 0) v *= Tv[w][e];
                });
                return v;
            };
            // fold of channel c of V (this lane's path) into u and the
            // frozen generator
            auto fold = [&](auto cc, Real vc) {
                constexpr int c = decltype(cc)::value;
                if constexpr (c == 0) {
                    u = vc;
                } else if constexpr (c == 1) {
                    gen += vc;
                } else if constexpr (c < 2 + D) {
                    gen += bst[c - 2] * vc;
                } else {
                    constexpr int j = hess_j(D, c - 2 - D);
                    constexpr int k = hess_k(D, c - 2 - D);
                    const Real cov = (j == k) ? Real(0.5) * sgs[j] * sgs[j]
                                              : rho * sgs[j] * sgs[k];
                    gen += cov * vc;
                }
            };
            {
                // V = B Gamma over the live rows of the channel table only
                // (channel_row_live): the derivative channels of a
                // polynomial over a downward-closed set have lower degree,
                // so the 67 channels of d = 10, eta = 3 need 1,882 of the
                // 364 x 67 products and the 22 of d = 5, eta = 3 need 357 of
                // 84 x 22.  The packed table is uniform across the wave:
                // each fused multiply-add takes its entry as a scalar
                // operand and the basis value as the vector one.  The
                // table's address is made opaque once per path, so that its
                // loads stay in the path's iteration instead of being
                // hoisted out of the path loop into registers.
                using CR = ChannelRows<DP, ETA, Q>;
                uint64_t pa = (uint64_t)(uintptr_t)&gamma[0];
                asm volatile("" : "+s"(pa));
                const auto pk = (const __attribute__((address_space(4))) Real *)pa;
                // u^k(T, X_T): channel 0
                static_for<NP>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    uT = fma(basis(lc, TzT), pk[l], uT);
                });
                terminal = payoff<D>(prm.payoff, K, X) - uT;
                // second derivatives first, one channel at a time, each
                // folded as soon as it is complete: their live rows are
                // those of degree at most eta - 2 (at total degree 3 the
                // constant and the linear ones, whose basis values are the
                // coordinates themselves), so no accumulator of theirs
                // stays live through the rest of the rows
                static_for<CR::tab.NH>([&](auto hc) {
                    constexpr int h = decltype(hc)::value;
                    Real vc = Real(0);
                    static_for<NP>([&](auto lc) {
                        constexpr int e = CR::tab.hpos[h][decltype(lc)::value];
                        if constexpr (e >= 0) vc = fma(basis(lc, Tz), pk[e], vc);
                    });
                    fold(std::integral_constant<int, 2 + D + h>{}, vc);
                });
                // then u, d_t u and the gradient over every row in order
                Real V[2 + D];
#pragma unroll
                for (int c = 0; c < 2 + D; ++c) V[c] = Real(0);
                static_for<NP>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    constexpr int e0 = CR::tab.goff[l];
                    const Real b = basis(lc, Tz);
                    V[0] = fma(b, pk[l], V[0]);
                    static_for<CR::tab.goff[l + 1] - e0>([&](auto ec) {
                        constexpr int e = e0 + decltype(ec)::value;
                        constexpr int c = CR::tab.gch[e - CR::tab.goff[0]];
                        V[c] = fma(b, pk[e], V[c]);
                    });
                });
                static_for<2 + D>([&](auto cc) { fold(cc, V[decltype(cc)::value]); });
            }
        }

        // penalised driver f = -r u + omega (Phi - u)_+ and the path term
        const Real f = -r * u + omega * fmax(phi_tau - u, Real(0));
        const Real a = (T - t0) * (f + gen) + terminal;
        const double ad = (double)a;
        cnt += 1;
        const double dev = ad - mean;
        mean += dev / (double)cnt;
        m2 = fma(dev, ad - mean, m2);
    }

    // fixed-order reduction of the lanes' moments (combine_moments):
    // butterfly within the wavefront, then waves in order through LDS
    double n = (double)cnt;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double nb = __shfl_xor(n, off), mb = __shfl_xor(mean, off),
                     m2b = __shfl_xor(m2, off);
        combine_moments(n, mean, m2, nb, mb, m2b);
    }
    __shared__ double red[3][kBlock / 64];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = n;
        red[1][wave] = mean;
        red[2][wave] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nw = 0.0, mw = 0.0, m2w = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w)
            combine_moments(nw, mw, m2w, red[0][w], red[1][w], red[2][w]);
        out[0] = mw;
        out[1] = m2w;
    }
    __syncthreads(); // red[] may be reused by the next tile
}

// Waves per SIMD the register allocation must allow.  The d = 10 (FP32)
// and d = 5 (FP32 and FP64) kernels are held to three waves (168 registers
// a lane): left to themselves they take 180-240 and run at two, and at
// three they run 10-17% faster (d = 10 serving shape, d = 5 FP64), with
// what does not fit (up to 340 bytes a lane) stored and reloaded once per
// path, outside the Euler loop.  At four waves (128 registers) the FP64
// d = 5 kernel spills inside the Euler loop and takes 60% longer, and the
// FP32 d = 10 one gains 2%.  d = 10 in FP64 runs at two waves.  d = 2 in
// FP64 (eta = 5 wants over 256 registers) runs at two waves, 29% faster than
// at one.
template <int D, typename Real>
constexpr int min_waves()
{
    if (D >= 10) return sizeof(Real) == 4 ? 3 : 2;
    if (D == 5) return 3;
    if (D == 2) return sizeof(Real) == 4 ? 1 : 2;
    return 1;
}

// One problem: workgroup b runs tile (i, g) = (b / groups, b % groups) and
// writes its sums to partial[2 b].
template <int D, int ETA, typename Real, int VOL, int Q, int OP = kOpBasis>
__global__ __launch_bounds__(kBlock, (min_waves<D, Real>())) void path_kernel(
    const PathParams prm, const double *__restrict__ pts,
    const Real *__restrict__ gamma, double *__restrict__ partial)
{
    const int i = blockIdx.x / prm.groups;
    const int g = blockIdx.x - i * prm.groups;
    // prm is the first kernel argument: its copy at the start of the
    // kernel-argument segment is the one the scalar loads read
    run_tile<D, ETA, Real, VOL, Q, const Real *__restrict__, OP, true>(
        prm, (uint64_t)(uintptr_t)__builtin_amdgcn_kernarg_segment_ptr(), pts,
        gamma, i, g, partial + 2 * (size_t)blockIdx.x);
}

// Many problems of one kernel signature in one persistent launch.  Tiles
// of problem q are tile_begin[q] .. tile_begin[q+1]-1 (problems ordered by
// decreasing tile cost); every workgroup takes the next tile from an
// atomic counter until none is left -- dynamic per-tile dispatch.  A tile
// computes exactly what the one-problem kernel computes for the same
// (i, g), so a problem's result does not depend on the batch.
template <int D, int ETA, typename Real, int VOL, int Q>
__global__ __launch_bounds__(kBlock, (min_waves<D, Real>())) void batch_path_kernel(
    const BatchTileDesc *__restrict__ probs, int nprob,
    const long long *__restrict__ tile_begin, unsigned int *counter)
{
    __shared__ long long next;
    const long long total = tile_begin[nprob];
    for (;;) {
        if (threadIdx.x == 0) next = (long long)atomicAdd(counter, 1u);
        __syncthreads();
        // the tile index is the same in every lane: keep it (and the
        // problem lookup and parameter loads that follow) scalar
        const long long tl = next;
        const long long t =
            (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                             (int)(tl >> 32))
                         << 32) |
                        (unsigned)__builtin_amdgcn_readfirstlane((int)tl));
        __syncthreads();
        if (t >= total) break;
        int lo = 0, hi = nprob - 1; // last q with tile_begin[q] <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_begin[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchTileDesc &q = probs[lo];
        const long long local = t - tile_begin[lo];
        const int i = (int)(local / q.prm.groups);
        const int g = (int)(local - (long long)i * q.prm.groups);
        using ConstReal = const __attribute__((address_space(4))) Real *;
        run_tile<D, ETA, Real, VOL, Q>(q.prm, 0, q.pts, (ConstReal)q.gamma, i, g,
                                    q.partial + 2 * local);
    }
}

// ---------------------------------------------------------------------------
// Instantiation and dispatch.  For one (d, eta) the kernels exist for FP32
// paths and, when FP64 is set, FP64 paths; for the constant and bump
// volatilities and, when DUP is set, the Dupire-type one.
// ---------------------------------------------------------------------------
template <typename T>
struct TypeTag {
    using type = T;
};

// Path precisions a set is instantiated for (a bit set)
enum PrecisionSet { kPrecF32 = 1, kPrecF64 = 2, kPrecBoth = 3 };

// calls f(TypeTag<Real>, integral_constant<VOL>) for the variant at hand;
// hipErrorInvalidValue when it is not instantiated
template <int D, int E, int PREC, bool DUP, typename F>
hipError_t dispatch_variant(bool fp32, int vol, F &&f)
{
    auto by_vol = [&](auto rt) -> hipError_t {
        if (vol == kVolConst) return f(rt, std::integral_constant<int, kVolConst>{});
        if (vol == kVolBump) return f(rt, std::integral_constant<int, kVolBump>{});
        if constexpr (DUP) {
            if (vol == kVolDupire) return f(rt, std::integral_constant<int, kVolDupire>{});
        }
        return hipErrorInvalidValue;
    };
    if (fp32) {
        if constexpr ((PREC & kPrecF32) != 0) return by_vol(TypeTag<float>{});
    } else {
        if constexpr ((PREC & kPrecF64) != 0) return by_vol(TypeTag<double>{});
    }
    return hipErrorInvalidValue;
}

template <int D, int E, int Q>
int copy_index_table(int8_t *nu, int cap)
{
    constexpr int DP = D + 1;
    constexpr auto &t = Basis<DP, E, Q>::tab;
    constexpr int P = Basis<DP, E, Q>::P;
    if (nu && cap >= P)
        for (int l = 0; l < P; ++l)
            for (int v = 0; v < DP; ++v) nu[l * DP + v] = t.nu[l][v];
    return P;
}

} // namespace bsde

// Defines launch_path_dD, index_table_dD, launch_batch_dD,
// batch_occupancy_dD and has_variant_dD for the (eta, q-norm, precisions,
// Dupire) sets listed by SETS(X) as X(E, Q, PREC, DUP), with q = Q / 10 and
// PREC a PrecisionSet.
// Path kernels of the kernel operator (Section 3.2) for d = D: FP32 and
// FP64 paths, constant and bump volatility; table = rows {z, y}
#define BSDE_DEFINE_KERNEL_OP(D)                                               \
    hipError_t launch_kernel_path_d##D(bool fp32, int blocks, hipStream_t s,   \
                                       const PathParams &prm,                  \
                                       const double *pts, const void *table,   \
                                       double *partial, hipEvent_t ev0,        \
                                       hipEvent_t ev1)                         \
    {                                                                          \
        return dispatch_variant<D, 1, kPrecBoth, false>(                            \
            fp32, prm.vol_kind, [&](auto rt, auto vt) -> hipError_t {          \
                using R = typename decltype(rt)::type;                         \
                hipExtLaunchKernelGGL(                                         \
                    (path_kernel<D, 1, R, decltype(vt)::value, 10, kOpKernel>), \
                    dim3(blocks), dim3(kBlock), 0, s, ev0, ev1, 0u, prm, pts,  \
                    (const R *)table, partial);                                \
                return hipGetLastError();                                      \
            });                                                                \
    }

#define BSDE_DEFINE_DIMENSION(D, SETS) BSDE_DEFINE_DIMENSION_NAMED(D, D, SETS)
// the same for a second group of sets of dimension D in a translation unit
// of its own: the functions are named with NAME (launch_path_dNAME, ...)
#define BSDE_DEFINE_DIMENSION_NAMED(D, NAME, SETS)                             \
    hipError_t launch_path_d##NAME(int eta, int q10, bool fp32, int blocks,    \
                                hipStream_t s,                                 \
                                const PathParams &prm, const double *pts,      \
                                const void *gamma, double *partial,            \
                                hipEvent_t ev0, hipEvent_t ev1)                \
    {                                                                          \
        constexpr int D_ = D;                                                  \
        SETS(BSDE_PATH_SET)                                                    \
        return hipErrorInvalidValue;                                           \
    }                                                                          \
    int index_table_d##NAME(int eta, int q10, int8_t *nu, int cap)                \
    {                                                                          \
        constexpr int D_ = D;                                                  \
        SETS(BSDE_TABLE_SET)                                                   \
        return 0;                                                              \
    }                                                                          \
    hipError_t launch_batch_d##NAME(int eta, int q10, bool fp32, int vol,         \
                                 int blocks,                                   \
                                 hipStream_t s, const BatchTileDesc *probs,    \
                                 int nprob, const long long *tile_begin,       \
                                 unsigned int *counter)                        \
    {                                                                          \
        constexpr int D_ = D;                                                  \
        SETS(BSDE_BATCH_SET)                                                   \
        return hipErrorInvalidValue;                                           \
    }                                                                          \
    int batch_occupancy_d##NAME(int eta, int q10, bool fp32, int vol)             \
    {                                                                          \
        constexpr int D_ = D;                                                  \
        int nb = 0;                                                            \
        SETS(BSDE_OCC_SET)                                                     \
        return nb;                                                             \
    }                                                                          \
    bool has_variant_d##NAME(int eta, int q10, bool fp32, int vol)                \
    {                                                                          \
        constexpr int D_ = D;                                                  \
        SETS(BSDE_HAS_SET)                                                     \
        return false;                                                          \
    }

#define BSDE_PATH_SET(E, Q, PREC, DUP)                                          \
    if (eta == E && q10 == Q)                                                  \
        return dispatch_variant<D_, E, PREC, DUP>(                              \
            fp32, prm.vol_kind, [&](auto rt, auto vt) -> hipError_t {          \
                using R = typename decltype(rt)::type;                         \
                /* ev0/ev1 (may be null) take the start and end times   \
                   of the dispatch itself: no marker packets around it */  \
                hipExtLaunchKernelGGL(                                         \
                    (path_kernel<D_, E, R, decltype(vt)::value, Q>),           \
                    dim3(blocks), dim3(kBlock), 0, s, ev0, ev1, 0u, prm, pts,  \
                    (const R *)gamma, partial);                                \
                return hipGetLastError();                                      \
            });
#define BSDE_TABLE_SET(E, Q, PREC, DUP)                                         \
    if (eta == E && q10 == Q) return copy_index_table<D_, E, Q>(nu, cap);
#define BSDE_BATCH_SET(E, Q, PREC, DUP)                                         \
    if (eta == E && q10 == Q)                                                  \
        return dispatch_variant<D_, E, PREC, DUP>(                              \
            fp32, vol, [&](auto rt, auto vt) -> hipError_t {                   \
                using R = typename decltype(rt)::type;                         \
                hipLaunchKernelGGL(                                            \
                    (batch_path_kernel<D_, E, R, decltype(vt)::value, Q>),     \
                    dim3(blocks), dim3(kBlock), 0, s, probs, nprob,            \
                    tile_begin, counter);                                      \
                return hipGetLastError();                                      \
            });
#define BSDE_OCC_SET(E, Q, PREC, DUP)                                           \
    if (eta == E && q10 == Q)                                                  \
        (void)dispatch_variant<D_, E, PREC, DUP>(                               \
            fp32, vol, [&](auto rt, auto vt) -> hipError_t {                   \
                using R = typename decltype(rt)::type;                         \
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(           \
                    &nb, batch_path_kernel<D_, E, R, decltype(vt)::value, Q>,  \
                    kBlock, 0);                                                \
            });
#define BSDE_HAS_SET(E, Q, PREC, DUP)                                           \
    if (eta == E && q10 == Q)                                                  \
        return dispatch_variant<D_, E, PREC, DUP>(                              \
                   fp32, vol, [](auto, auto) { return hipSuccess; }) ==        \
               hipSuccess;
