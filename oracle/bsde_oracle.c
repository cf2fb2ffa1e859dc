/*
 * bsde_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see the
 * header for what it computes and the readings it takes).
 *
 * Written for readability, not speed: single thread, no blocking, no fusion,
 * the loops of Algorithm "algodetail" (Section 4.1) in the paper's order.
 */
#define _GNU_SOURCE
#include "bsde_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ===================================================================== */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:   */
/* as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies    */
/* with a Weyl-sequence key schedule.                                     */
/* ===================================================================== */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in (0, 1) from one 32-bit word */
static double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

static void philox_block(uint64_t seed, uint32_t m, uint32_t i, uint32_t k,
                         uint32_t sub, uint32_t block, uint32_t w[4])
{
    uint32_t ctr[4] = { m, i, k, (sub << 24) | block };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    oracle_philox4x32_10(ctr, key, w);
}

/* Box-Muller (1958): two uniforms -> two independent standard normals. */
static void box_muller(uint32_t wa, uint32_t wb, double *n0, double *n1)
{
    double R = sqrt(-2.0 * log(u01(wa)));
    double phi = 2.0 * 3.14159265358979323846 * u01(wb);
    *n0 = R * cos(phi);
    *n1 = R * sin(phi);
}

/* A stream of normals of one (m, i, k, substream), caching the last block. */
typedef struct {
    uint64_t seed;
    uint32_t m, i, k, sub, first_block;
    int64_t cached; /* block index held in nrm[], -1 = none */
    double nrm[4];
} normal_stream;

static void ns_init(normal_stream *s, uint64_t seed, uint32_t m, uint32_t i,
                    uint32_t k, uint32_t sub, uint32_t first_block)
{
    s->seed = seed; s->m = m; s->i = i; s->k = k; s->sub = sub;
    s->first_block = first_block;
    s->cached = -1;
}

/* normal number q of the stream (normals 4b..4b+3 live in block b) */
static double ns_get(normal_stream *s, uint32_t q)
{
    uint32_t block = s->first_block + q / 4;
    if (s->cached != (int64_t)block) {
        uint32_t w[4];
        philox_block(s->seed, s->m, s->i, s->k, s->sub, block, w);
        box_muller(w[0], w[1], &s->nrm[0], &s->nrm[1]);
        box_muller(w[2], w[3], &s->nrm[2], &s->nrm[3]);
        s->cached = block;
    }
    return s->nrm[q % 4];
}

void oracle_normals(uint64_t seed, uint32_t m, uint32_t i, uint32_t k,
                    uint32_t sub, uint32_t first_block, int count,
                    double *out)
{
    normal_stream s;
    ns_init(&s, seed, m, i, k, sub, first_block);
    for (int q = 0; q < count; ++q) out[q] = ns_get(&s, (uint32_t)q);
}

/* ===================================================================== */
/* Index set (eq. hyper_set): nu in N^{d'} with (sum nu_j^q)^{1/q} <= eta. */
/* Listed by total degree, then lexicographically decreasing.             */
/* ===================================================================== */
static int in_hyperbolic_set(const int *nu, int dp, int eta, double q)
{
    int total = 0;
    for (int j = 0; j < dp; ++j) total += nu[j];
    if (total > eta) return 0;          /* q <= 1: q-norm >= 1-norm */
    if (q >= 1.0) return 1;
    double s = 0.0;
    for (int j = 0; j < dp; ++j)
        if (nu[j] > 0) s += pow((double)nu[j], q);
    return s <= pow((double)eta, q) * (1.0 + 1e-12);
}

static void enumerate_degree(int *cur, int j, int dp, int remaining, int eta,
                             double q, int *nu, int cap, int *count)
{
    if (j == dp - 1) {
        cur[j] = remaining;
        if (in_hyperbolic_set(cur, dp, eta, q)) {
            if (*count < cap && nu)
                memcpy(nu + (size_t)(*count) * dp, cur, sizeof(int) * dp);
            ++*count;
        }
        return;
    }
    for (int v = remaining; v >= 0; --v) {
        cur[j] = v;
        enumerate_degree(cur, j + 1, dp, remaining - v, eta, q, nu, cap,
                         count);
    }
}

int oracle_index_set(int dp, int eta, double q, int *nu, int cap)
{
    int cur[ORACLE_DMAX + 1];
    int count = 0;
    if (dp < 1 || dp > ORACLE_DMAX + 1 || eta < 0) return 0;
    for (int g = 0; g <= eta; ++g)
        enumerate_degree(cur, 0, dp, g, eta, q, nu, cap, &count);
    return count;
}

int oracle_num_basis(const oracle_problem *pb)
{
    return oracle_index_set(pb->d + 1, pb->eta, pb->q, NULL, 0);
}

/* ===================================================================== */
/* Domain, grid, correlation                                              */
/* ===================================================================== */
void oracle_domain(const oracle_problem *pb, double *lo, double *hi)
{
    for (int j = 0; j < pb->d; ++j) {
        double half = pb->width * pb->vol_level[j] * sqrt(pb->T);
        lo[j] = log(pb->S0[j]) - half;
        hi[j] = log(pb->S0[j]) + half;
    }
}

static long n_spatial(const oracle_problem *pb)
{
    if (pb->grid == ORACLE_GRID_TENSOR) {
        long s = 1;
        for (int j = 0; j < pb->d; ++j) s *= pb->n_x;
        return s;
    }
    return pb->n_x;
}

int oracle_num_points(const oracle_problem *pb)
{
    if (pb->grid == ORACLE_GRID_UNIFORM) return pb->n_x;
    return (int)(n_spatial(pb) * pb->n_t);
}

int oracle_points(const oracle_problem *pb, double *pts)
{
    return oracle_points_k(pb, 0, pts);
}

/* Algorithm 1 draws the n points uniformly at every iteration; with the
 * fixed time nodes of the grid reading only the spatial coordinates are
 * redrawn, from the counter (b, 0, k, substream 2 | block). */
int oracle_points_k(const oracle_problem *pb, uint32_t k, double *pts)
{
    int d = pb->d;
    uint32_t kdraw = (pb->redraw && pb->grid != ORACLE_GRID_TENSOR) ? k : 0;
    if (pb->grid == ORACLE_GRID_UNIFORM) {
        /* point i: word q of the counter (i, 0, k, substream 3 | q / 4) is
         * t for q = 0 and x_j for q = 1 + j, each uniform on its range */
        double lo[ORACLE_DMAX], hi[ORACLE_DMAX];
        oracle_domain(pb, lo, hi);
        for (int i = 0; i < pb->n_x; ++i) {
            double *row = pts + (size_t)i * (d + 1);
            for (int q = 0; q <= d; ++q) {
                uint32_t w[4];
                philox_block(pb->seed, (uint32_t)i, 0, kdraw, 3, (uint32_t)(q / 4), w);
                double u = u01(w[q % 4]);
                row[q] = q == 0 ? pb->T * u : lo[q - 1] + u * (hi[q - 1] - lo[q - 1]);
            }
        }
        return pb->n_x;
    }
    long ns = n_spatial(pb);
    double lo[ORACLE_DMAX], hi[ORACLE_DMAX];
    oracle_domain(pb, lo, hi);
    for (int a = 0; a < pb->n_t; ++a) {
        double t = (double)a * pb->T / (double)(pb->n_t - 1);
        for (long b = 0; b < ns; ++b) {
            double *row = pts + (size_t)(a * ns + b) * (d + 1);
            row[0] = t;
            for (int j = 0; j < d; ++j) {
                double z;
                if (pb->grid == ORACLE_GRID_TENSOR) {
                    long digit = b;
                    for (int jj = 0; jj < j; ++jj) digit /= pb->n_x;
                    digit %= pb->n_x;
                    z = pb->n_x > 1
                            ? -1.0 + 2.0 * (double)digit / (pb->n_x - 1)
                            : 0.0;
                } else {
                    uint32_t w[4];
                    philox_block(pb->seed, (uint32_t)b, 0, kdraw, 2,
                                 (uint32_t)(j / 4), w);
                    z = 2.0 * u01(w[j % 4]) - 1.0;
                }
                row[1 + j] = lo[j] + 0.5 * (z + 1.0) * (hi[j] - lo[j]);
            }
        }
    }
    return (int)(ns * pb->n_t);
}

int oracle_cholesky(int d, double rho, double *L)
{
    /* C_jk = rho for j != k, 1 on the diagonal (Section 6.2) */
    for (int j = 0; j < d * d; ++j) L[j] = 0.0;
    for (int j = 0; j < d; ++j) {
        for (int k = 0; k <= j; ++k) {
            double c = (j == k) ? 1.0 : rho;
            double s = c;
            for (int l = 0; l < k; ++l) s -= L[j * d + l] * L[k * d + l];
            if (j == k) {
                if (s <= 0.0) return ORACLE_EINVAL;
                L[j * d + j] = sqrt(s);
            } else {
                L[j * d + k] = s / L[k * d + k];
            }
        }
    }
    return ORACLE_OK;
}

/* ===================================================================== */
/* Least squares by Householder QR (in place of LAPACK dgelsy).           */
/* ===================================================================== */
int oracle_lstsq(int n, int p, const double *B, const double *y,
                 double *alpha)
{
    if (n < p || p < 1) return ORACLE_ERANK;
    double *A = (double *)malloc(sizeof(double) * (size_t)n * p);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(A, B, sizeof(double) * (size_t)n * p);
    memcpy(b, y, sizeof(double) * (size_t)n);
    int status = ORACLE_OK;
    for (int j = 0; j < p; ++j) {
        double norm2 = 0.0;
        for (int i = j; i < n; ++i) norm2 += A[(size_t)i * p + j] * A[(size_t)i * p + j];
        double norm = sqrt(norm2);
        if (norm == 0.0) { status = ORACLE_ERANK; break; }
        double top = A[(size_t)j * p + j];
        double beta = top >= 0.0 ? -norm : norm; /* new diagonal entry */
        for (int i = j; i < n; ++i) v[i] = A[(size_t)i * p + j];
        v[j] -= beta;
        double vv = 0.0;
        for (int i = j; i < n; ++i) vv += v[i] * v[i];
        /* apply H = I - 2 v v' / (v' v) to columns j..p-1 and to b */
        for (int c = j; c < p; ++c) {
            double s = 0.0;
            for (int i = j; i < n; ++i) s += v[i] * A[(size_t)i * p + c];
            double f = 2.0 * s / vv;
            for (int i = j; i < n; ++i) A[(size_t)i * p + c] -= f * v[i];
        }
        double s = 0.0;
        for (int i = j; i < n; ++i) s += v[i] * b[i];
        double f = 2.0 * s / vv;
        for (int i = j; i < n; ++i) b[i] -= f * v[i];
    }
    if (status == ORACLE_OK) {
        double dmax = 0.0, dmin = INFINITY;
        for (int j = 0; j < p; ++j) {
            double a = fabs(A[(size_t)j * p + j]);
            if (a > dmax) dmax = a;
            if (a < dmin) dmin = a;
        }
        if (!(dmin > 1e-12 * dmax)) status = ORACLE_ERANK;
    }
    if (status == ORACLE_OK) {
        for (int j = p - 1; j >= 0; --j) { /* back substitution R a = Q'y */
            double s = b[j];
            for (int c = j + 1; c < p; ++c) s -= A[(size_t)j * p + c] * alpha[c];
            alpha[j] = s / A[(size_t)j * p + j];
        }
    }
    free(A); free(b); free(v);
    return status;
}

/* ===================================================================== */
/* Model pieces (Section 5, eq. 4; payoffs eq. put_payoff, call_payoff)   */
/* ===================================================================== */
double oracle_payoff(const oracle_problem *pb, const double *x)
{
    int d = pb->d;
    double mean_e = 0.0, mean_x = 0.0, sum_x = 0.0;
    for (int j = 0; j < d; ++j) {
        mean_e += exp(x[j]);
        mean_x += x[j];
        sum_x += x[j];
    }
    mean_e /= d;
    mean_x /= d;
    switch (pb->payoff) {
    case ORACLE_PUT_ARITH: return fmax(pb->K - mean_e, 0.0);
    case ORACLE_CALL_ARITH: return fmax(mean_e - pb->K, 0.0);
    case ORACLE_PUT_GEOM: return fmax(pb->K - exp(mean_x), 0.0);
    case ORACLE_CALL_GEOM: return fmax(exp(mean_x) - pb->K, 0.0);
    case ORACLE_FWD_ARITH: return mean_e - pb->K;
    case ORACLE_QUAD: return sum_x * sum_x;
    }
    return NAN;
}

double oracle_vol(const oracle_problem *pb, int j, double t, double x_j)
{
    if (pb->vol_kind == ORACLE_VOL_BUMP) {
        double dx = x_j - log(pb->bump_c);
        return pb->vol_level[j] * (1.0 + pb->bump_a * exp(-dx * dx));
    }
    if (pb->vol_kind == ORACLE_VOL_DUPIRE) {
        /* eq. vol_locale with the price S = e^{x_j} and s the spot S0_j */
        double S = exp(x_j);
        double dev = S * exp(pb->r * t) - pb->S0[j];
        return 0.6 * (1.2 - exp(-0.1 * t) * exp(-0.001 * dev * dev)) *
               exp(-0.05 * sqrt(t));
    }
    return pb->vol_level[j];
}

/* ===================================================================== */
/* u^k and its derivatives from the monomial expansion (Section 4.2:      */
/* u = sum alpha_l B_l, B_l = t^{nu_0} prod x_j^{nu_j} in mapped variables) */
/* ===================================================================== */
static double ipow(double z, int e)
{
    double r = 1.0;
    for (int a = 0; a < e; ++a) r *= z;
    return r;
}

void oracle_eval(const oracle_problem *pb, const int *nu, int p,
                 const double *alpha, double t, const double *x, double *u,
                 double *ut, double *ux, double *uxx)
{
    int d = pb->d, dp = d + 1;
    double lo[ORACLE_DMAX], hi[ORACLE_DMAX];
    double z[ORACLE_DMAX + 1], scale[ORACLE_DMAX + 1];
    oracle_domain(pb, lo, hi);
    z[0] = 2.0 * t / pb->T - 1.0;
    scale[0] = 2.0 / pb->T;
    for (int j = 0; j < d; ++j) {
        scale[1 + j] = 2.0 / (hi[j] - lo[j]);
        z[1 + j] = (x[j] - lo[j]) * scale[1 + j] - 1.0;
    }
    *u = 0.0;
    *ut = 0.0;
    for (int j = 0; j < d; ++j) ux[j] = 0.0;
    for (int j = 0; j < d * d; ++j) uxx[j] = 0.0;
    for (int l = 0; l < p; ++l) {
        const int *e = nu + (size_t)l * dp;
        double a = alpha[l];
        /* value */
        double val = 1.0;
        for (int v = 0; v < dp; ++v) val *= ipow(z[v], e[v]);
        *u += a * val;
        /* first derivatives: d/dz_v z_v^e = e z_v^{e-1} */
        for (int v = 0; v < dp; ++v) {
            if (e[v] == 0) continue;
            double g = scale[v] * e[v] * ipow(z[v], e[v] - 1);
            for (int w = 0; w < dp; ++w)
                if (w != v) g *= ipow(z[w], e[w]);
            if (v == 0) *ut += a * g;
            else ux[v - 1] += a * g;
        }
        /* second derivatives in x */
        for (int j = 1; j < dp; ++j) {
            for (int k = 1; k < dp; ++k) {
                double g;
                if (j == k) {
                    if (e[j] < 2) continue;
                    g = scale[j] * scale[j] * e[j] * (e[j] - 1) *
                        ipow(z[j], e[j] - 2);
                    for (int w = 0; w < dp; ++w)
                        if (w != j) g *= ipow(z[w], e[w]);
                } else {
                    if (e[j] < 1 || e[k] < 1) continue;
                    g = scale[j] * e[j] * ipow(z[j], e[j] - 1) * scale[k] *
                        e[k] * ipow(z[k], e[k] - 1);
                    for (int w = 0; w < dp; ++w)
                        if (w != j && w != k) g *= ipow(z[w], e[w]);
                }
                uxx[(j - 1) * d + (k - 1)] += a * g;
            }
        }
    }
}

/* ===================================================================== */
/* One Euler path from (t0, x0) (eq. eqs3 with N equal steps on [t0,T]),  */
/* the random time tau = t0 + (T - t0) U (eq. psiN) and X^N_tau by the    */
/* continuous-time Euler interpolation inside step j*.                    */
/* ===================================================================== */
void oracle_path(const oracle_problem *pb, double t0, const double *x0,
                 uint32_t i, uint32_t m, uint32_t k, oracle_path_out *out)
{
    int d = pb->d, N = pb->N;
    double T = pb->T;
    double h = (T - t0) / N;
    double L[ORACLE_DMAX * ORACLE_DMAX];
    oracle_cholesky(d, pb->rho, L);

    /* U from word 0 of substream 1, block 0; j* = floor(U N) and
     * theta = U N - j*, both exact in integer arithmetic. */
    uint32_t w[4];
    philox_block(pb->seed, m, i, k, 1, 0, w);
    uint64_t num = (2ull * w[0] + 1ull) * (uint64_t)N; /* U N = num / 2^33 */
    out->U = u01(w[0]);
    out->jstar = (uint32_t)(num >> 33);
    out->theta = (double)(num & ((1ull << 33) - 1)) * 0x1p-33;
    out->tau = t0 + (T - t0) * out->U;

    normal_stream steps, bridge;
    ns_init(&steps, pb->seed, m, i, k, 0, 0);
    ns_init(&bridge, pb->seed, m, i, k, 1, 1);

    double X[ORACLE_DMAX];
    for (int j = 0; j < d; ++j) X[j] = x0[j];
    for (int s = 0; s < N; ++s) {
        double ts = t0 + s * h;
        double G[ORACLE_DMAX], LG[ORACLE_DMAX], sig[ORACLE_DMAX],
            b[ORACLE_DMAX];
        for (int j = 0; j < d; ++j) G[j] = ns_get(&steps, (uint32_t)(s * d + j));
        for (int j = 0; j < d; ++j) {
            LG[j] = 0.0;
            for (int l = 0; l <= j; ++l) LG[j] += L[j * d + l] * G[l];
        }
        for (int j = 0; j < d; ++j) {
            sig[j] = oracle_vol(pb, j, ts, X[j]);
            b[j] = pb->r - pb->div[j] - 0.5 * sig[j] * sig[j];
        }
        if ((uint32_t)s == out->jstar) {
            double th = out->theta;
            double Gb[ORACLE_DMAX], LGb[ORACLE_DMAX];
            for (int j = 0; j < d; ++j) Gb[j] = ns_get(&bridge, (uint32_t)j);
            for (int j = 0; j < d; ++j) {
                LGb[j] = 0.0;
                for (int l = 0; l <= j; ++l) LGb[j] += L[j * d + l] * Gb[l];
            }
            for (int j = 0; j < d; ++j) {
                out->xstar[j] = X[j];
                out->sigstar[j] = sig[j];
                out->bstar[j] = b[j];
                out->xtau[j] = X[j] + b[j] * th * h +
                               sig[j] * (th * sqrt(h) * LG[j] +
                                         sqrt(th * (1.0 - th) * h) * LGb[j]);
            }
        }
        for (int j = 0; j < d; ++j) X[j] += b[j] * h + sig[j] * sqrt(h) * LG[j];
    }
    for (int j = 0; j < d; ++j) out->xT[j] = X[j];
}

/* a_m = psi^N(t_i, x_i, f_{u^k} + (d_t + L^N) u^k, Phi - u^k, W, U)
 * (Algorithm line "MC"; eq. psiN), with f(t,x,y,z) = -r y + omega (Phi(x) - y)_+
 * (eq. bsde-penal-2) and L^N frozen at the last Euler node. */
/* a_m from the path and u^k (value, derivatives at (tau, X_tau), value at
 * (T, X_T)): eq. (3.3) with the penalised driver */
static double path_term_from(const oracle_problem *pb, const oracle_path_out *pp,
                             double t0, double u, double ut, const double *ux,
                             const double *uxx, double uT);

double oracle_path_term(const oracle_problem *pb, const int *nu, int p,
                        const double *alpha, double t0, const double *x0,
                        uint32_t i, uint32_t m, uint32_t k)
{
    int d = pb->d;
    double T = pb->T;
    oracle_path_out P;
    oracle_path(pb, t0, x0, i, m, k, &P);

    double u = 0.0, ut = 0.0, ux[ORACLE_DMAX] = { 0 },
           uxx[ORACLE_DMAX * ORACLE_DMAX] = { 0 };
    double uT = 0.0, dummy_t, dummy_x[ORACLE_DMAX],
           dummy_xx[ORACLE_DMAX * ORACLE_DMAX];
    if (alpha) {
        oracle_eval(pb, nu, p, alpha, P.tau, P.xtau, &u, &ut, ux, uxx);
        oracle_eval(pb, nu, p, alpha, T, P.xT, &uT, &dummy_t, dummy_x,
                    dummy_xx);
    }
    (void)d;
    return path_term_from(pb, &P, t0, u, ut, ux, uxx, uT);
}

static double path_term_from(const oracle_problem *pb, const oracle_path_out *pp,
                             double t0, double u, double ut, const double *ux,
                             const double *uxx, double uT)
{
    const oracle_path_out P = *pp;
    int d = pb->d;
    double T = pb->T;
    double f = -pb->r * u + pb->omega * fmax(oracle_payoff(pb, P.xtau) - u, 0.0);
    double gen = ut;
    for (int j = 0; j < d; ++j) gen += P.bstar[j] * ux[j];
    for (int j = 0; j < d; ++j)
        for (int l = 0; l < d; ++l) {
            double cjl = (j == l) ? 1.0 : pb->rho;
            gen += 0.5 * P.sigstar[j] * P.sigstar[l] * cjl * uxx[j * d + l];
        }
    double g1 = f + gen;
    double g2 = oracle_payoff(pb, P.xT) - uT;
    return (T - t0) * g1 + g2;
}

/* c_i = (1/M) sum_m a_m (eq. chat) and the sample variance of the a_m */
static void correction_at_point(const oracle_problem *pb, const int *nu,
                                int p, const double *alpha,
                                const double *row, uint32_t i, uint32_t k,
                                double *a, double *c, double *var)
{
    double sum = 0.0;
    for (int m = 0; m < pb->M; ++m) {
        a[m] = oracle_path_term(pb, nu, p, alpha, row[0], row + 1, i,
                                (uint32_t)m, k);
        sum += a[m];
    }
    double mean = sum / pb->M;
    double ss = 0.0;
    for (int m = 0; m < pb->M; ++m) ss += (a[m] - mean) * (a[m] - mean);
    *c = mean;
    if (var) *var = pb->M > 1 ? ss / (pb->M - 1) : 0.0;
}

void oracle_corrections(const oracle_problem *pb, const double *alpha,
                        uint32_t k, int i_begin, int i_end, double *c,
                        double *var)
{
    int d = pb->d, n = oracle_num_points(pb);
    int p = oracle_num_basis(pb);
    int *nu = (int *)malloc(sizeof(int) * (size_t)p * (d + 1));
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    double *a = (double *)malloc(sizeof(double) * (size_t)pb->M);
    oracle_index_set(d + 1, pb->eta, pb->q, nu, p);
    oracle_points_k(pb, k, pts);
    for (int i = i_begin; i < i_end; ++i)
        correction_at_point(pb, nu, p, alpha, pts + (size_t)i * (d + 1),
                            (uint32_t)i, k, a, &c[i - i_begin],
                            var ? &var[i - i_begin] : NULL);
    free(nu); free(pts); free(a);
}

/* ===================================================================== */
/* Algorithm "algodetail": the Picard loop with the least-squares         */
/* extrapolating operator (eq. lspb).                                     */
/* ===================================================================== */
static void basis_matrix(const oracle_problem *pb, const int *nu, int p,
                         const double *pts, int n, double *B)
{
    int d = pb->d, dp = d + 1;
    double lo[ORACLE_DMAX], hi[ORACLE_DMAX];
    oracle_domain(pb, lo, hi);
    for (int i = 0; i < n; ++i) {
        const double *row = pts + (size_t)i * dp;
        double z[ORACLE_DMAX + 1];
        z[0] = 2.0 * row[0] / pb->T - 1.0;
        for (int j = 0; j < d; ++j)
            z[1 + j] = 2.0 * (row[1 + j] - lo[j]) / (hi[j] - lo[j]) - 1.0;
        for (int l = 0; l < p; ++l) {
            double v = 1.0;
            for (int w = 0; w < dp; ++w) v *= ipow(z[w], nu[(size_t)l * dp + w]);
            B[(size_t)i * p + l] = v;
        }
    }
}

void oracle_basis_matrix(const oracle_problem *pb, double *B)
{
    oracle_basis_matrix_k(pb, 0, B);
}

void oracle_basis_matrix_k(const oracle_problem *pb, uint32_t k, double *B)
{
    int d = pb->d, n = oracle_num_points(pb), p = oracle_num_basis(pb);
    int *nu = (int *)malloc(sizeof(int) * (size_t)p * (d + 1));
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    oracle_index_set(d + 1, pb->eta, pb->q, nu, p);
    oracle_points_k(pb, k, pts);
    basis_matrix(pb, nu, p, pts, n, B);
    free(nu); free(pts);
}

int oracle_fit(const oracle_problem *pb, const double *y, double *alpha)
{
    int d = pb->d, n = oracle_num_points(pb), p = oracle_num_basis(pb);
    int *nu = (int *)malloc(sizeof(int) * (size_t)p * (d + 1));
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    double *B = (double *)malloc(sizeof(double) * (size_t)n * p);
    oracle_index_set(d + 1, pb->eta, pb->q, nu, p);
    oracle_points(pb, pts);
    basis_matrix(pb, nu, p, pts, n, B);
    int st = oracle_lstsq(n, p, B, y, alpha);
    free(nu); free(pts); free(B);
    return st;
}

int oracle_solve(const oracle_problem *pb, int k_start,
                 const double *alpha_start, int k_end, double *alpha_hist,
                 double *c_hist, double *var_hist, double *u_hist)
{
    int d = pb->d;
    if (d < 1 || d > ORACLE_DMAX || pb->N < 1 || pb->M < 1 ||
        (pb->grid != ORACLE_GRID_UNIFORM && pb->n_t < 2) ||
        pb->n_x < 1 || k_start < 0 || k_end < k_start)
        return ORACLE_EINVAL;
    double Ltest[ORACLE_DMAX * ORACLE_DMAX];
    if (oracle_cholesky(d, pb->rho, Ltest) != ORACLE_OK) return ORACLE_EINVAL;
    int n = oracle_num_points(pb), p = oracle_num_basis(pb);
    if (n < p) return ORACLE_ERANK;

    int *nu = (int *)malloc(sizeof(int) * (size_t)p * (d + 1));
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    double *B = (double *)malloc(sizeof(double) * (size_t)n * p);
    double *alpha = (double *)malloc(sizeof(double) * (size_t)p);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *var = (double *)malloc(sizeof(double) * (size_t)n);
    double *uvec = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *abuf = (double *)malloc(sizeof(double) * (size_t)pb->M);
    oracle_index_set(d + 1, pb->eta, pb->q, nu, p);
    oracle_points(pb, pts);
    basis_matrix(pb, nu, p, pts, n, B);

    /* u^0 = 0, alpha^0 = 0 (Algorithm, first line) unless resuming */
    for (int l = 0; l < p; ++l) alpha[l] = alpha_start ? alpha_start[l] : 0.0;
    if (alpha_hist) memcpy(alpha_hist, alpha, sizeof(double) * (size_t)p);

    int status = ORACLE_OK;
    int have_alpha = alpha_start != NULL;
    int redraw = pb->redraw && pb->grid != ORACLE_GRID_TENSOR;
    for (int k = k_start; k < k_end; ++k) {
        /* the points of this iteration (Algorithm 1: new uniform points at
         * every iteration) and their basis matrix */
        if (redraw) {
            oracle_points_k(pb, (uint32_t)k, pts);
            basis_matrix(pb, nu, p, pts, n, B);
        }
        /* c_i for every point (eq. chat) */
        for (int i = 0; i < n; ++i)
            correction_at_point(pb, nu, p, have_alpha ? alpha : NULL,
                                pts + (size_t)i * (d + 1), (uint32_t)i,
                                (uint32_t)k, abuf, &c[i], &var[i]);
        /* u_i = sum_l alpha_l B_l(t_i, x_i) (eq. cu) */
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int l = 0; l < p; ++l) s += alpha[l] * B[(size_t)i * p + l];
            uvec[i] = s;
            y[i] = uvec[i] + c[i];
        }
        /* alpha^{k+1} = argmin sum_i |u_i + c_i - sum_l alpha_l B_l|^2 (eq. alpha) */
        status = oracle_lstsq(n, p, B, y, alpha);
        if (status != ORACLE_OK) break;
        have_alpha = 1;
        int kk = k - k_start;
        if (alpha_hist)
            memcpy(alpha_hist + (size_t)(kk + 1) * p, alpha, sizeof(double) * (size_t)p);
        if (c_hist) memcpy(c_hist + (size_t)kk * n, c, sizeof(double) * (size_t)n);
        if (var_hist) memcpy(var_hist + (size_t)kk * n, var, sizeof(double) * (size_t)n);
        if (u_hist) memcpy(u_hist + (size_t)kk * n, uvec, sizeof(double) * (size_t)n);
    }
    free(nu); free(pts); free(B); free(alpha); free(c); free(var); free(uvec);
    free(y); free(abuf);
    return status;
}

void oracle_price_delta(const oracle_problem *pb, const double *alpha,
                        int nq, const double *t, const double *S,
                        double *price, double *delta)
{
    int d = pb->d, p = oracle_num_basis(pb);
    int *nu = (int *)malloc(sizeof(int) * (size_t)p * (d + 1));
    oracle_index_set(d + 1, pb->eta, pb->q, nu, p);
    for (int qi = 0; qi < nq; ++qi) {
        double x[ORACLE_DMAX], u, ut, ux[ORACLE_DMAX],
            uxx[ORACLE_DMAX * ORACLE_DMAX];
        for (int j = 0; j < d; ++j) x[j] = log(S[(size_t)qi * d + j]);
        oracle_eval(pb, nu, p, alpha, t[qi], x, &u, &ut, ux, uxx);
        price[qi] = u;
        /* Delta = grad_x V in price units: d u / d S_j = e^{-x_j} d_{x_j} u */
        for (int j = 0; j < d; ++j)
            delta[(size_t)qi * d + j] = ux[j] / S[(size_t)qi * d + j];
    }
    free(nu);
}

/* ===================================================================== */
/* The kernel operator of Section 3.2 ("A kernel operator", the first      */
/* version of the method): h(t, x) = sum_i y_i K_t(t - t_i) K_x(x - x_i),  */
/* taken in its normalised form h = sum_i y_i k_i / sum_i k_i (so that it  */
/* reproduces constants up to the edges of the domain) with Gaussian k_i   */
/* of one bandwidth b in the mapped coordinates z.  With S_0 = sum k_i and */
/* S_1 = sum y_i k_i, h = S_1 / S_0 and, for derivatives in z,             */
/*   d_v h = (d_v S_1 - h d_v S_0) / S_0,                                  */
/*   d_vw h = (d_vw S_1 - h d_vw S_0 - d_v h d_w S_0 - d_w h d_v S_0) / S_0. */
/* ===================================================================== */
static void map_z(const oracle_problem *pb, const double *lo, const double *hi,
                  double t, const double *x, double *z)
{
    z[0] = 2.0 * t / pb->T - 1.0;
    for (int j = 0; j < pb->d; ++j)
        z[1 + j] = 2.0 * (x[j] - lo[j]) / (hi[j] - lo[j]) - 1.0;
}

void oracle_kernel_eval(const oracle_problem *pb, const double *pts,
                        const double *y, int n, double t, const double *x,
                        double *u, double *ut, double *ux, double *uxx)
{
    const int d = pb->d, dp = d + 1;
    const double b2 = pb->kernel_bw * pb->kernel_bw;
    double lo[ORACLE_DMAX], hi[ORACLE_DMAX], z[ORACLE_DMAX + 1];
    oracle_domain(pb, lo, hi);
    map_z(pb, lo, hi, t, x, z);
    double S0 = 0.0, S1 = 0.0;
    double S0v[ORACLE_DMAX + 1] = { 0 }, S1v[ORACLE_DMAX + 1] = { 0 };
    double S0vw[(ORACLE_DMAX + 1) * (ORACLE_DMAX + 1)] = { 0 };
    double S1vw[(ORACLE_DMAX + 1) * (ORACLE_DMAX + 1)] = { 0 };
    for (int i = 0; i < n; ++i) {
        const double *row = pts + (size_t)i * dp;
        double zi[ORACLE_DMAX + 1], dz[ORACLE_DMAX + 1], q = 0.0;
        map_z(pb, lo, hi, row[0], row + 1, zi);
        for (int v = 0; v < dp; ++v) {
            dz[v] = z[v] - zi[v];
            q += dz[v] * dz[v];
        }
        const double e = q / (2.0 * b2);
        const int flat = e > 60.0; /* clamped: constant weight */
        const double w = exp(-(flat ? 60.0 : e));
        const double yi = y ? y[i] : 0.0;
        S0 += w;
        S1 += yi * w;
        if (flat) continue;
        for (int v = 0; v < dp; ++v) {
            const double g = -dz[v] / b2; /* d/dz_v of the Gaussian, / w */
            S0v[v] += w * g;
            S1v[v] += yi * w * g;
            for (int ww = 0; ww < dp; ++ww) {
                const double g2 = dz[v] * dz[ww] / (b2 * b2) - (v == ww ? 1.0 / b2 : 0.0);
                S0vw[v * dp + ww] += w * g2;
                S1vw[v * dp + ww] += yi * w * g2;
            }
        }
    }
    const double h = S1 / S0;
    double hv[ORACLE_DMAX + 1];
    for (int v = 0; v < dp; ++v) hv[v] = (S1v[v] - h * S0v[v]) / S0;
    /* chain rule: dz_0/dt = 2/T, dz_j/dx_j = 2/(hi_j - lo_j) */
    double sc[ORACLE_DMAX + 1];
    sc[0] = 2.0 / pb->T;
    for (int j = 0; j < d; ++j) sc[1 + j] = 2.0 / (hi[j] - lo[j]);
    *u = h;
    *ut = hv[0] * sc[0];
    for (int j = 0; j < d; ++j) {
        ux[j] = hv[1 + j] * sc[1 + j];
        for (int l = 0; l < d; ++l) {
            const int v = 1 + j, ww = 1 + l;
            const double hvw = (S1vw[v * dp + ww] - h * S0vw[v * dp + ww] -
                                hv[v] * S0v[ww] - hv[ww] * S0v[v]) / S0;
            uxx[j * d + l] = hvw * sc[v] * sc[ww];
        }
    }
}

void oracle_kernel_corrections(const oracle_problem *pb, const double *y,
                               uint32_t k, int i_begin, int i_end, double *c,
                               double *var)
{
    const int d = pb->d, n = oracle_num_points(pb);
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    double *a = (double *)malloc(sizeof(double) * (size_t)pb->M);
    oracle_points(pb, pts);
    for (int i = i_begin; i < i_end; ++i) {
        const double *row = pts + (size_t)i * (d + 1);
        double sum = 0.0;
        for (int m = 0; m < pb->M; ++m) {
            oracle_path_out P;
            oracle_path(pb, row[0], row + 1, (uint32_t)i, (uint32_t)m, k, &P);
            double u = 0.0, ut = 0.0, ux[ORACLE_DMAX] = { 0 },
                   uxx[ORACLE_DMAX * ORACLE_DMAX] = { 0 }, uT = 0.0;
            if (y) {
                double dt, dx[ORACLE_DMAX], dxx[ORACLE_DMAX * ORACLE_DMAX];
                oracle_kernel_eval(pb, pts, y, n, P.tau, P.xtau, &u, &ut, ux, uxx);
                oracle_kernel_eval(pb, pts, y, n, pb->T, P.xT, &uT, &dt, dx, dxx);
            }
            a[m] = path_term_from(pb, &P, row[0], u, ut, ux, uxx, uT);
            sum += a[m];
        }
        const double mean = sum / pb->M;
        double ss = 0.0;
        for (int m = 0; m < pb->M; ++m) ss += (a[m] - mean) * (a[m] - mean);
        c[i - i_begin] = mean;
        if (var) var[i - i_begin] = pb->M > 1 ? ss / (pb->M - 1) : 0.0;
    }
    free(pts); free(a);
}

int oracle_kernel_solve(const oracle_problem *pb, double *y_hist,
                        double *c_hist, double *var_hist, double *u_hist)
{
    const int d = pb->d;
    if (d < 1 || d > ORACLE_DMAX || pb->N < 1 || pb->M < 1 ||
        !(pb->kernel_bw > 0.0) || pb->redraw ||
        (pb->grid != ORACLE_GRID_UNIFORM && pb->n_t < 2) || pb->n_x < 1)
        return ORACLE_EINVAL;
    double Ltest[ORACLE_DMAX * ORACLE_DMAX];
    if (oracle_cholesky(d, pb->rho, Ltest) != ORACLE_OK) return ORACLE_EINVAL;
    const int n = oracle_num_points(pb);
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    double *y = (double *)calloc((size_t)n, sizeof(double));
    double *ynew = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *var = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_points(pb, pts);
    if (y_hist) memset(y_hist, 0, sizeof(double) * (size_t)n);
    for (int k = 0; k < pb->K_it; ++k) {
        /* c_i with u^k = h[y^{k-1}] (u^0 = 0) */
        oracle_kernel_corrections(pb, k ? y : NULL, (uint32_t)k, 0, n, c, var);
        /* y^k_i = u^k(t_i, x_i) + c^k_i */
        for (int i = 0; i < n; ++i) {
            double u = 0.0, ut, ux[ORACLE_DMAX], uxx[ORACLE_DMAX * ORACLE_DMAX];
            const double *row = pts + (size_t)i * (d + 1);
            if (k) oracle_kernel_eval(pb, pts, y, n, row[0], row + 1, &u, &ut, ux, uxx);
            ynew[i] = u + c[i];
            if (u_hist) u_hist[(size_t)k * n + i] = u;
        }
        memcpy(y, ynew, sizeof(double) * (size_t)n);
        if (y_hist) memcpy(y_hist + (size_t)(k + 1) * n, y, sizeof(double) * (size_t)n);
        if (c_hist) memcpy(c_hist + (size_t)k * n, c, sizeof(double) * (size_t)n);
        if (var_hist) memcpy(var_hist + (size_t)k * n, var, sizeof(double) * (size_t)n);
    }
    free(pts); free(y); free(ynew); free(c); free(var);
    return ORACLE_OK;
}

void oracle_kernel_price_delta(const oracle_problem *pb, const double *y,
                               int nq, const double *t, const double *S,
                               double *price, double *delta)
{
    const int d = pb->d, n = oracle_num_points(pb);
    double *pts = (double *)malloc(sizeof(double) * (size_t)n * (d + 1));
    oracle_points(pb, pts);
    for (int qi = 0; qi < nq; ++qi) {
        double x[ORACLE_DMAX], u, ut, ux[ORACLE_DMAX], uxx[ORACLE_DMAX * ORACLE_DMAX];
        for (int j = 0; j < d; ++j) x[j] = log(S[(size_t)qi * d + j]);
        oracle_kernel_eval(pb, pts, y, n, t[qi], x, &u, &ut, ux, uxx);
        price[qi] = u;
        for (int j = 0; j < d; ++j) delta[(size_t)qi * d + j] = ux[j] / S[(size_t)qi * d + j];
    }
    free(pts);
}
