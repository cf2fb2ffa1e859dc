/*
 * bsde_oracle.h -- plain, single-threaded FP64 CPU oracle for the Picard +
 * adaptive-control-variate BSDE solver of Labart & Lelong, "A Parallel
 * Algorithm for solving BSDEs" (arXiv:1102.4666).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a slow,
 * obviously correct implementation written straight from the paper.  It
 * shares no source, header, table or helper with the GPU library.
 *
 * What it computes (paper, Section 3 "Presentation of the Algorithm",
 * Algorithm "algodetail" of Section 4.1):
 *   u^0 = 0; for k = 0..K_it-1:
 *     for every grid point (t_i, x_i) and path m = 1..M:
 *       a_m = (T - t_i) [f_{u^k} + (d_t + L^N) u^k](tau, X^N_tau)
 *             + (Phi - u^k(T, .))(X^N_T),        tau = t_i + (T - t_i) U
 *     c_i = mean_m a_m                            (eq. chat)
 *     u_i = sum_l alpha^k_l B_l(t_i, x_i)         (eq. cu)
 *     alpha^{k+1} = argmin ||(u + c) - B alpha||  (eq. alpha)
 * with the option model of Section 5 (log-prices, eq. 4; penalised driver
 * f = -r y + omega (y - Phi)^-, eq. bsde-penal-2) and the correlated
 * Brownian motion of Section 6.2 (Cholesky factor of rho 11' + (1-rho) I).
 *
 * Readings where the paper is silent (each is restated where it is used):
 *  - Euler grid: N equal steps on [t_i, T], h = (T - t_i)/N; coefficients
 *    frozen at the last grid node (phi^N of eq. eqs3).
 *  - One random time tau per path.  X^N_tau is the continuous-time Euler
 *    interpolation inside step j* = floor(U N) (a Brownian bridge from
 *    X_{j*} towards X_{j*+1}), so the step normals do not depend on U.
 *  - Points: a fixed grid for every k (tensor grid in [0,T] x D, or
 *    uniform random spatial points drawn once); time nodes a T/(n_t - 1).
 *  - Domain D_j = [log S0_j - w l_j sqrt(T), log S0_j + w l_j sqrt(T)];
 *    polynomials are centred and normalised to [-1,1]^{d+1} (Section 4,
 *    "Practical determination of the vector alpha").
 *  - Basis: canonical monomials t^{nu_0} prod x_j^{nu_j} of the mapped
 *    variables (Section 4.2), index set {nu : (sum nu_j^q)^{1/q} <= eta}
 *    (eq. hyper_set), derivatives evaluated directly.
 *  - Least squares by Householder QR of B (full column rank required; a
 *    rank-deficient B is an error) in place of LAPACK dgelsy.
 *  - Randomness: Philox4x32-10 (Salmon et al., SC'11), key = 64-bit seed,
 *    counter = (m, i, k, (substream << 24) | block); normals by Box-Muller
 *    (Box & Muller 1958) on u(w) = (w + 1/2) 2^-32.
 *      substream 0, block b: step normals 4b..4b+3, normal q = s d + j
 *      substream 1, block 0: word 0 -> U; blocks >= 1: bridge normals
 *      substream 2: random grid points (counter (b, 0, 0, .))
 */
#ifndef BSDE_ORACLE_H
#define BSDE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_DMAX 16

/* volatility kinds: constant l_j; bump l_j (1 + a e^{-(x_j - log c)^2});
 * Dupire-type of eq. vol_locale, sigma(t, S) = 0.6 (1.2 - e^{-0.1 t}
 * e^{-0.001 (S e^{r t} - s)^2}) e^{-0.05 sqrt t} with s = S0_j (the smile
 * bottom at the forward); for it, l_j only sets the domain width. */
enum { ORACLE_VOL_CONST = 0, ORACLE_VOL_BUMP = 1, ORACLE_VOL_DUPIRE = 2 };
enum {
    ORACLE_PUT_ARITH = 0,  /* (K - mean_j e^{x_j})_+          eq. put_payoff  */
    ORACLE_CALL_ARITH = 1, /* (mean_j e^{x_j} - K)_+          eq. call_payoff */
    ORACLE_PUT_GEOM = 2,   /* (K - exp(mean_j x_j))_+                          */
    ORACLE_CALL_GEOM = 3,  /* (exp(mean_j x_j) - K)_+                          */
    ORACLE_FWD_ARITH = 4,  /* mean_j e^{x_j} - K   (call minus put)            */
    ORACLE_QUAD = 5        /* (sum_j x_j)^2        (test payoff)               */
};
/* points: tensor grid x time nodes; random spatial points x time nodes;
 * or n_x points uniform in [0, T] x D (Algorithm 1's literal draw) */
enum { ORACLE_GRID_TENSOR = 0, ORACLE_GRID_RANDOM = 1, ORACLE_GRID_UNIFORM = 2 };

enum {
    ORACLE_OK = 0,
    ORACLE_EINVAL = 1,
    ORACLE_ERANK = 3
};

typedef struct {
    int d;                          /* number of assets                     */
    int vol_kind;                   /* ORACLE_VOL_*                         */
    double vol_level[ORACLE_DMAX];  /* l_j                                  */
    double bump_a, bump_c;          /* sigma_j = l_j (1 + a e^{-(x_j - log c)^2}) */
    double rho;                     /* uniform correlation                  */
    double r;                       /* interest rate                        */
    double div[ORACLE_DMAX];        /* dividend rates delta_j               */
    int payoff;                     /* ORACLE_* payoff kind                 */
    double K, T;
    double S0[ORACLE_DMAX];
    int grid;                       /* ORACLE_GRID_*                        */
    int n_t;                        /* time nodes (>= 2)                    */
    int n_x;                        /* tensor: per dimension; random: total */
    double width;                   /* domain half-width in l_j sqrt(T)     */
    int eta;                        /* maximal degree                       */
    double q;                       /* hyperbolic q-norm parameter, (0, 1]  */
    int M, N, K_it;
    double omega;                   /* penalisation weight (0 = European)   */
    uint64_t seed;
    int redraw;                     /* random/uniform points: new points    */
                                    /* every Picard iteration (Algorithm 1) */
    double kernel_bw;               /* > 0: the kernel operator of Section  */
                                    /* 3.2 with this bandwidth (mapped z)   */
                                    /* instead of the least-squares one     */
} oracle_problem;

/* --- randomness ------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);
/* count normals of (m, i, k, substream), starting at block first_block. */
void oracle_normals(uint64_t seed, uint32_t m, uint32_t i, uint32_t k,
                    uint32_t sub, uint32_t first_block, int count,
                    double *out);

/* --- setup ------------------------------------------------------------ */
int oracle_num_points(const oracle_problem *pb);
/* index set of d' = dp variates; writes at most cap multi-indices
 * (row-major, dp entries each) and returns the size p of the set. */
int oracle_index_set(int dp, int eta, double q, int *nu, int cap);
int oracle_num_basis(const oracle_problem *pb);
void oracle_domain(const oracle_problem *pb, double *lo, double *hi);
/* points as n rows of (t, x_1..x_d); point i = a * n_spatial + b. */
int oracle_points(const oracle_problem *pb, double *pts);
/* the points used at Picard iteration k: with redraw on a random grid the
 * spatial points are drawn afresh for every k (counter word 2 = k), else
 * the fixed grid of oracle_points (which is iteration 0's). */
int oracle_points_k(const oracle_problem *pb, uint32_t k, double *pts);
/* Cholesky factor (row-major d x d, lower) of rho 11' + (1 - rho) I. */
int oracle_cholesky(int d, double rho, double *L);
/* Least squares argmin ||y - B alpha|| by Householder QR, B row-major n x p. */
int oracle_lstsq(int n, int p, const double *B, const double *y,
                 double *alpha);

/* --- pieces of the path term (exposed for tests) ---------------------- */
double oracle_payoff(const oracle_problem *pb, const double *x);
double oracle_vol(const oracle_problem *pb, int j, double t, double x_j);
/* u, du/dt, grad_x u (d), hessian_x u (d x d) of sum_l alpha_l B_l at (t, x) */
void oracle_eval(const oracle_problem *pb, const int *nu, int p,
                 const double *alpha, double t, const double *x,
                 double *u, double *ut, double *ux, double *uxx);

typedef struct {
    uint32_t jstar;     /* Euler step holding tau                      */
    double U, theta;    /* U and the fraction of step jstar            */
    double tau;
    double xstar[ORACLE_DMAX]; /* X at the last node before tau        */
    double sigstar[ORACLE_DMAX];
    double bstar[ORACLE_DMAX];
    double xtau[ORACLE_DMAX];
    double xT[ORACLE_DMAX];
} oracle_path_out;

void oracle_path(const oracle_problem *pb, double t0, const double *x0,
                 uint32_t i, uint32_t m, uint32_t k, oracle_path_out *out);
double oracle_path_term(const oracle_problem *pb, const int *nu, int p,
                        const double *alpha, double t0, const double *x0,
                        uint32_t i, uint32_t m, uint32_t k);
/* c_i and the sample variance of a_m for points i_begin..i_end-1 at
 * iteration k with coefficients alpha (may be NULL for u = 0). */
void oracle_corrections(const oracle_problem *pb, const double *alpha,
                        uint32_t k, int i_begin, int i_end, double *c,
                        double *var);

/* --- whole algorithm -------------------------------------------------- */
/* Runs iterations k_start..k_end-1 from alpha_start (NULL = u^0 = 0).
 * alpha_hist: (k_end - k_start + 1) x p; c_hist, var_hist, u_hist:
 * (k_end - k_start) x n (each may be NULL). */
int oracle_solve(const oracle_problem *pb, int k_start,
                 const double *alpha_start, int k_end, double *alpha_hist,
                 double *c_hist, double *var_hist, double *u_hist);
/* B_{il} = B_l(t_i, x_i), row-major n x p (the least-squares design matrix). */
void oracle_basis_matrix(const oracle_problem *pb, double *B);
/* the basis matrix of the points of Picard iteration k */
void oracle_basis_matrix_k(const oracle_problem *pb, uint32_t k, double *B);
/* alpha = B^+ y for values y at the grid points (fit of a known function). */
int oracle_fit(const oracle_problem *pb, const double *y, double *alpha);
/* price u(t, log S) and dollar delta e^{-x_j} d_{x_j} u for nq queries. */
void oracle_price_delta(const oracle_problem *pb, const double *alpha,
                        int nq, const double *t, const double *S,
                        double *price, double *delta);

/* --- the kernel operator of Section 3.2 (first version of the method) --- */
/* h(t, x) = sum_i y_i k_i(t, x) / sum_i k_i(t, x), the normalised form of
 * the paper's sum_i u(t_i, x_i) K_t(t - t_i) K_x(x - x_i), with Gaussian
 * kernels k_i = exp(-min(|z - z_i|^2 / (2 b^2), 60)) in the mapped
 * coordinates z of the basis (z_0 = 2t/T - 1, z_j = the map of x_j onto
 * [-1, 1]), b = kernel_bw.  Beyond the clamp a weight is constant (zero
 * derivative).  u, u_t, grad_x u and hess_x u of h at (t, x) over the n
 * points pts with values y. */
void oracle_kernel_eval(const oracle_problem *pb, const double *pts,
                        const double *y, int n, double t, const double *x,
                        double *u, double *ut, double *ux, double *uxx);
/* c_i and variances at iteration k with u^k = h[y] (y NULL: u^k = 0) */
void oracle_kernel_corrections(const oracle_problem *pb, const double *y,
                               uint32_t k, int i_begin, int i_end, double *c,
                               double *var);
/* Picard loop with the kernel operator: y^k = u^k(t_i, x_i) + c^k_i and
 * u^{k+1} = h[y^k].  y_hist: (K_it + 1) x n, row 0 all zero (u^0 = 0),
 * row k + 1 = y^k; c_hist, var_hist, u_hist: K_it x n (each may be NULL). */
int oracle_kernel_solve(const oracle_problem *pb, double *y_hist,
                        double *c_hist, double *var_hist, double *u_hist);
void oracle_kernel_price_delta(const oracle_problem *pb, const double *y,
                               int nq, const double *t, const double *S,
                               double *price, double *delta);

#ifdef __cplusplus
}
#endif
#endif
