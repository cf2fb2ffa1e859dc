// bsde_f64_math.h -- FP64 elementary functions of the FP64 path kernels,
// specialised to the arguments the Box-Muller transform hands them.
//
// The angle of a Box-Muller pair is 2 pi u with u = (w + 1/2) 2^-32 for a
// 32-bit Philox word w, so its reduction to a quarter turn is exact integer
// arithmetic on w: with q the nearest quarter turn and the remainder
// rho = w - q 2^30 in [-2^29, 2^29), the reduced angle is
// x = 2 pi (rho + 1/2) 2^-32 in [-pi/4, pi/4] (one rounding), and
// sin(2 pi u), cos(2 pi u) are sin x, cos x permuted and negated by q.  On
// [-pi/4, pi/4] the Maclaurin series of sine to degree 17 and of cosine to
// degree 16 leave remainders below 1e-19 and 3e-18, under a quarter of an
// ulp of the results (|cos x| >= 0.707, |sin x| >= 0.637 |x|), so the
// results are within a few ulps.  The general-argument library sincos
// spends most of its instructions on a double-word reduction by pi/2 that
// this angle does not need.
//
// The radius of the pair needs ln u for the same u: with v = w + 1/2 =
// 2^e m, m in [1/sqrt 2, sqrt 2) split off the bits of v, ln u =
// (e - 32) ln 2 + ln m and ln m = 2 atanh(s), s = (m - 1) / (m + 1),
// |s| <= 0.1716, whose odd series 2 s (1 + s^2/3 + s^4/5 + ...) is taken
// as 2 s + s z q(z), z = s^2, with q a degree-6 polynomial fitted to the
// series' tail (relative error 4.7e-16 of a term below 1% of 2 s).  The
// quotient s takes one hardware reciprocal and two residual corrections.
//
// The local volatility needs e^x for x = -y^2 <= 0: x clamped at -708
// (e^-708 is already below the volatility's rounding), x = n ln 2 + r with
// |r| <= ln 2 / 2 (ln 2 in two parts, so r is exact to the last bits), e^r
// by its Maclaurin series to degree 13 (remainder below 6e-18 of e^r), and
// the power 2^n applied to the exponent.
//
// The radius takes the square root from the hardware reciprocal square
// root and Newton steps (sqrt_nonneg).
//
// Plain double and 32-bit integer arithmetic (and the hardware reciprocal
// and reciprocal-square-root seeds on the device), so the same code also
// compiles for the host: the test suite checks it there against
// high-precision references.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define BSDE_F64_HD __host__ __device__
#else
#define BSDE_F64_HD
#endif

namespace bsde {
namespace f64 {

// Maclaurin coefficients (-1)^k / (2k+1)! of sine and (-1)^k / (2k)! of
// cosine, k = 1..8
constexpr double kS[8] = {-1.0 / 6.0,
                          1.0 / 120.0,
                          -1.0 / 5040.0,
                          1.0 / 362880.0,
                          -1.0 / 39916800.0,
                          1.0 / 6227020800.0,
                          -1.0 / 1307674368000.0,
                          1.0 / 355687428096000.0};
constexpr double kC[8] = {-1.0 / 2.0,
                          1.0 / 24.0,
                          -1.0 / 720.0,
                          1.0 / 40320.0,
                          -1.0 / 3628800.0,
                          1.0 / 479001600.0,
                          -1.0 / 87178291200.0,
                          1.0 / 20922789888000.0};
// 2 pi 2^-32 (the ulp of u in radians)
constexpr double kTwoPiUlp = 6.283185307179586476925286766559 / 4294967296.0;

// sin x and cos x for |x| <= pi/4 (Maclaurin series to degrees 17 and 16)
BSDE_F64_HD inline void sincos_reduced(double x, double &s, double &c)
{
    const double x2 = x * x;
    double ps = kS[7], pc = kC[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) {
        ps = __builtin_fma(ps, x2, kS[k]);
        pc = __builtin_fma(pc, x2, kC[k]);
    }
    s = __builtin_fma(x * x2, ps, x);
    c = __builtin_fma(x2, pc, 1.0);
}

// sin and cos of q pi/2 + x from sx = sin x, cx = cos x:
// sin(q pi/2 + x) = sin x, cos x, -sin x, -cos x;
// cos(q pi/2 + x) = cos x, -sin x, -cos x, sin x
BSDE_F64_HD inline void rotate_quarters(uint32_t q, double sx, double cx, double &s, double &c)
{
    const bool odd = (q & 1u) != 0;
    const double a = odd ? cx : sx;
    const double b = odd ? sx : cx;
    s = (q & 2u) ? -a : a;
    c = ((q + 1u) & 2u) ? -b : b;
}

// sin and cos of the angle 2 pi (w + 1/2) 2^-32 (w a 32-bit word)
BSDE_F64_HD inline void sincos_turn(uint32_t w, double &s, double &c)
{
    // nearest quarter turn (mod 4) and the signed remainder; the 32-bit
    // wrap-around of the sum gives q = 0 for the last eighth of the turn
    const uint32_t q = (w + 0x20000000u) >> 30;
    const int32_t rho = (int32_t)(w - (q << 30));
    const double x = __builtin_fma((double)rho, kTwoPiUlp, 0.5 * kTwoPiUlp);
    double sx, cx;
    sincos_reduced(x, sx, cx);
    rotate_quarters(q, sx, cx, s, c);
}

// ln 2 in two parts: kLn2Hi has 42 significant bits, so e kLn2Hi is exact
// for |e| < 2^11
constexpr double kLn2Hi = 0.693147180559890330187045037746429443359375;
constexpr double kLn2Lo = 5.4979230187083711552420206887e-14;

BSDE_F64_HD inline uint64_t to_bits(double x) { return __builtin_bit_cast(uint64_t, x); }
BSDE_F64_HD inline double from_bits(uint64_t b) { return __builtin_bit_cast(double, b); }

// Hardware seeds: v_rcp_f64 and v_rsq_f64 on the device.  The host build
// (tests only) takes seeds of single-precision accuracy, no better than the
// hardware's, so that the refinement steps below are tested as the device
// needs them.
BSDE_F64_HD inline double reciprocal_seed(double d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(d);
#else
    return (1.0 / d) * (1.0 - 0x1p-24); // single-precision accuracy
#endif
}
BSDE_F64_HD inline double rsqrt_seed(double a)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(a);
#else
    // single-precision accuracy, also below the single-precision range
    const double y = 1.0 / __builtin_sqrt(a);
    return y * (1.0 + 0x1p-24);
#endif
}

// sqrt(a) for a = 0 or a normal number above 2^-900 (the Box-Muller radius
// sqrt(-2 v ln u), whose argument is zero or above 1e-25): from the
// reciprocal square root seed y of a + 2^-1000 (which is a itself unless a
// is zero, where y stays finite and g comes out 0), two coupled Newton steps
// on g ~ sqrt(a), h ~ 1/(2 sqrt(a)) (each squares the relative error:
// 2^-23 -> 2^-46 -> 2^-92) and one residual correction g + (a - g^2) h.
BSDE_F64_HD inline double sqrt_nonneg(double a)
{
    const double y = rsqrt_seed(a + 0x1p-1000);
    double g = a * y, h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    return __builtin_fma(__builtin_fma(-g, g, a), h, g);
}

// ln((w + 1/2) 2^-32) for a 32-bit word w
BSDE_F64_HD inline double log_word(uint32_t w)
{
    const double v = (double)w + 0.5; // exact, in [1/2, 2^32)
    const uint64_t b = to_bits(v);
    const uint32_t hi = (uint32_t)(b >> 32);
    const uint32_t frac_hi = hi & 0x000FFFFFu;
    // mantissas at or above sqrt 2 (its top fraction bits are 0x6A09E)
    // take the next exponent and m in [1/sqrt 2, 1)
    const uint32_t up = frac_hi >= 0x6A09Fu ? 1u : 0u;
    const int e = (int)(hi >> 20) - 1023 + (int)up - 32;
    const double m = from_bits(((uint64_t)(frac_hi | ((0x3FFu - up) << 20)) << 32) |
                               (b & 0xFFFFFFFFull));
    const double f = m - 1.0; // exact
    const double d = m + 1.0;
    // s = f / d from the reciprocal seed y and two residual corrections
    // s += (f - s d) y (each squares the relative error)
    const double y = reciprocal_seed(d);
    double sq = f * y;
    sq = __builtin_fma(__builtin_fma(-sq, d, f), y, sq);
    sq = __builtin_fma(__builtin_fma(-sq, d, f), y, sq);
    const double z = sq * sq;
    // q(z) = 2/3 + 2z/5 + 2z^2/7 + ... by a degree-6 polynomial fitted to its
    // relative error on [0, s_max^2] (Chebyshev nodes, least squares; at most
    // 4.7e-16 with the coefficients in double), in place of the series to
    // z^8: s z q is below 1% of 2 s, so this adds under 5e-18 to ln m
    double q = 0.14616233499191306;
    q = __builtin_fma(q, z, 0.15331740686457643);
    q = __builtin_fma(q, z, 0.18182888493505678);
    q = __builtin_fma(q, z, 0.22222211144430887);
    q = __builtin_fma(q, z, 0.2857142862590908);
    q = __builtin_fma(q, z, 0.3999999999989967);
    q = __builtin_fma(q, z, 0.666666666666667);
    const double ed = (double)e;
    const double hi_part = __builtin_fma(ed, kLn2Hi, 2.0 * sq);
    const double lo_part = __builtin_fma(ed, kLn2Lo, (sq * z) * q);
    return hi_part + lo_part;
}

// e^x for x <= 0 (the local volatility's e^{-y^2})
BSDE_F64_HD inline double exp_nonpos(double x)
{
    x = __builtin_fmax(x, -708.0);
    const double n = __builtin_rint(x * 1.4426950408889634073599246810019);
    double r = __builtin_fma(-n, kLn2Hi, x);
    r = __builtin_fma(-n, kLn2Lo, r);
    double p = 1.0 / 6227020800.0; // 1/13!
    p = __builtin_fma(p, r, 1.0 / 479001600.0);
    p = __builtin_fma(p, r, 1.0 / 39916800.0);
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    // times 2^n, n in [-1022, 0]: exponent field of a normal number
    return p * from_bits((uint64_t)(1023 + (int)n) << 52);
}

// ---------------------------------------------------------------------------
// Table-driven forms for the FP64 path kernels, with the tables in LDS
// (filled by each workgroup at the start of a tile):
//  - sine and cosine of the Box-Muller angle: the turn in 1024 sectors
//    centred at j/1024 turns (the axes are centres, so results near zero
//    keep their relative accuracy); the word's remainder rho = w - j 2^22
//    is exact, r = 2 pi (rho + 1/2) 2^-32 lies in [-pi/1024, pi/1024],
//    where sin r and cos r to degrees 5 and 4 leave remainders below 2e-19
//    of r and 2e-18; then the angle-addition formulas with the table's sine
//    and cosine of 2 pi j / 1024;
//  - e^x for x <= 0: x = (256 n + j) ln 2 / 256 + r, |r| <= ln 2 / 512, e^r
//    to degree 4 (remainder below 4e-17 of e^r), times the table entry
//    2^(j/256) and 2^n.
// The larger tables (18 KB of LDS a workgroup) take one degree off each
// series: two fused multiply-adds fewer per Box-Muller pair and one fewer
// per volatility.
// ---------------------------------------------------------------------------
constexpr int kSinCosBins = 1024;
constexpr int kExpBins = 256;
struct Tables {
    double sc[kSinCosBins][2]; // sin, cos of 2 pi j / 1024
    double ex[kExpBins];       // 2^(j/256)
};
// ln 2 / 256 in two parts: the first has 35 significant bits, so
// n kLn2_256Hi is exact for |n| < 2^18 (x >= -708 gives |n| < 261,500)
constexpr double kLn2_256Hi = 0.0027076061741126978;
constexpr double kLn2_256Lo = -5.0411407304988844e-14;

// entries first, first + stride, ... of both tables
BSDE_F64_HD inline void fill_tables(Tables &T, int first, int stride)
{
    for (int t = first; t < kSinCosBins + kExpBins; t += stride) {
        if (t < kSinCosBins) {
            // j/1024 turns = q/4 + f/1024, f in [-128, 128)
            const uint32_t q = ((uint32_t)(t + 128) >> 8) & 3u;
            const int f = t - (int)(((uint32_t)(t + 128) >> 8) << 8);
            double sx, cx;
            sincos_reduced((double)f * (6.283185307179586476925286766559 / 1024.0), sx, cx);
            rotate_quarters(q, sx, cx, T.sc[t][0], T.sc[t][1]);
        } else {
            T.ex[t - kSinCosBins] = exp2((double)(t - kSinCosBins) / (double)kExpBins);
        }
    }
}

BSDE_F64_HD inline void sincos_turn_tab(uint32_t w, const Tables &T, double &s, double &c)
{
    // nearest sector centre j 2^22 (mod 2^32) and the signed remainder
    const uint32_t j = (w + 0x00200000u) >> 22;
    const int32_t rho = (int32_t)(w - (j << 22));
    const double r = __builtin_fma((double)rho, kTwoPiUlp, 0.5 * kTwoPiUlp);
    const double r2 = r * r;
    // sin r = r + r^3 (-1/6 + r^2/120), cos r = 1 + r^2 (-1/2 + r^2/24)
    const double ps = __builtin_fma(r2, kS[1], kS[0]);
    const double pc = __builtin_fma(r2, kC[1], kC[0]);
    const double sr = __builtin_fma(r * r2, ps, r);
    const double cr = __builtin_fma(r2, pc, 1.0);
    const double sa = T.sc[j & (kSinCosBins - 1)][0], ca = T.sc[j & (kSinCosBins - 1)][1];
    s = __builtin_fma(sa, cr, ca * sr);
    c = __builtin_fma(ca, cr, -(sa * sr));
}

BSDE_F64_HD inline double exp_nonpos_tab(double x, const Tables &T)
{
    x = __builtin_fmax(x, -708.0);
    const double N = __builtin_rint(x * 369.32993046757465); // 256 / ln 2
    double r = __builtin_fma(-N, kLn2_256Hi, x);
    r = __builtin_fma(-N, kLn2_256Lo, r);
    // e^r - 1 = r + r^2 (1/2 + r (1/6 + r / 24))
    double q = __builtin_fma(r, 1.0 / 24.0, 1.0 / 6.0);
    q = __builtin_fma(q, r, 0.5);
    const double em1 = __builtin_fma(q * r, r, r);
    const int Ni = (int)N;
    const double t = T.ex[Ni & (kExpBins - 1)];
    // times 2^n, n = floor(N / 256) in [-1022, 0] (the result stays normal)
    return __builtin_ldexp(__builtin_fma(t, em1, t), Ni >> 8);
}

// 2^(-t/256) for t >= 0: the bump volatility's e^{-(x - log c)^2} when the
// FP64 paths carry y = kappa (x - log c) with kappa^2 = 256 log2 e, so that
// t = y^2 needs no reduction constant: t clamped at 261,485 (2^-1021.4, far
// below the volatility's rounding), N = rint(t) and f = t - N (exact, in
// [-1/2, 1/2]), 2^(-f/256) = e^{-f ln 2 / 256} by its Maclaurin series in f
// to degree 4 (remainder below 4e-17), times the table entry 2^(j/256) and
// 2^n for -N = 256 n + j.
// Coefficients (-ln 2 / 256)^k / k!, k = 1..4
constexpr double kE2m[4] = {-0.0027076061740622863, 3.6655655969101062e-06,
                            -3.3083026805413713e-09, 2.239395190875157e-12};
BSDE_F64_HD inline double exp2_neg_tab(double t, const Tables &T)
{
    t = __builtin_fmin(t, 261485.0);
    const double N = __builtin_rint(t);
    const double f = t - N; // exact
    double q = __builtin_fma(f, kE2m[3], kE2m[2]);
    q = __builtin_fma(q, f, kE2m[1]);
    q = __builtin_fma(q, f, kE2m[0]);
    const double em1 = q * f;
    const int Ni = -(int)N;
    const double e = T.ex[Ni & (kExpBins - 1)];
    // times 2^n, n = floor(-N / 256) in [-1022, 0] (the result stays normal)
    return __builtin_ldexp(__builtin_fma(e, em1, e), Ni >> 8);
}

} // namespace f64
} // namespace bsde
