"""Independent reference values used to pin the oracle (test code only).

Nothing here shares code with the oracle or the GPU library.  Each function
is a textbook result or a deterministic numerical method:

* Black-Scholes put/call prices and deltas (closed form).
* Geometric-basket put (closed form: the geometric mean of correlated
  log-normals is log-normal).
* Cox-Ross-Rubinstein binomial tree for the American put.
* A finite-difference solver of the 1-D penalised pricing PDE
  d_t u + L u - r u + omega (Phi - u)_+ = 0, which is the PDE of the
  penalised BSDE (eq. bsde-penal-2 of the paper; PDE link eq. edp).
* The exact-expectation version of the projected Picard map of Algorithm
  "algodetail" for constant volatility in d = 1 (no Monte Carlo): the
  expectation of the path term a_m is, by Ito's formula with the frozen
  generator, E[Phi(X_T) + int_t^T f(s, X_s, u^k) ds] - u^k(t, x), so the
  least-squares target y = u^k + E[c^k] is computed by Gauss quadrature.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_banded
from scipy.stats import norm


# --------------------------------------------------------------------------
def bs_put(S, K, r, sigma, tau, q=0.0):
    if tau <= 0:
        return max(K - S, 0.0)
    d1 = (math.log(S / K) + (r - q + 0.5 * sigma ** 2) * tau) / (sigma * math.sqrt(tau))
    d2 = d1 - sigma * math.sqrt(tau)
    return K * math.exp(-r * tau) * norm.cdf(-d2) - S * math.exp(-q * tau) * norm.cdf(-d1)


def bs_put_delta(S, K, r, sigma, tau, q=0.0):
    d1 = (math.log(S / K) + (r - q + 0.5 * sigma ** 2) * tau) / (sigma * math.sqrt(tau))
    return -math.exp(-q * tau) * norm.cdf(-d1)


def bs_call(S, K, r, sigma, tau, q=0.0):
    return bs_put(S, K, r, sigma, tau, q) + S * math.exp(-q * tau) - K * math.exp(-r * tau)


def geometric_basket_put(S0, K, r, sig, rho, T):
    """Put on exp(mean_j log S_j) with uniform correlation rho; returns
    (price, dollar deltas dV/dS0_j)."""
    S0 = np.asarray(S0, float)
    sig = np.asarray(sig, float)
    d = len(S0)
    C = np.full((d, d), rho)
    np.fill_diagonal(C, 1.0)
    m = np.mean(np.log(S0)) + (r - np.mean(sig ** 2) / 2) * T
    v = float(sig @ C @ sig) / d ** 2 * T
    F = math.exp(m + v / 2)
    d1 = (math.log(F / K) + v / 2) / math.sqrt(v)
    d2 = d1 - math.sqrt(v)
    price = math.exp(-r * T) * (K * norm.cdf(-d2) - F * norm.cdf(-d1))
    delta = -math.exp(-r * T) * norm.cdf(-d1) * F / (d * S0)
    return price, delta


def crr_american_put(S, K, r, sigma, T, steps=4000):
    dt = T / steps
    u = math.exp(sigma * math.sqrt(dt))
    dn = 1 / u
    p = (math.exp(r * dt) - dn) / (u - dn)
    disc = math.exp(-r * dt)
    j = np.arange(steps + 1)
    ST = S * u ** (steps - 2 * j)
    V = np.maximum(K - ST, 0.0)
    for n in range(steps - 1, -1, -1):
        j = np.arange(n + 1)
        Sn = S * u ** (n - 2 * j)
        V = disc * (p * V[:-1] + (1 - p) * V[1:])
        V = np.maximum(V, K - Sn)
    return float(V[0])


# --------------------------------------------------------------------------
def penalised_pde_1d(S0, K, r, vol, T, omega, payoff="put", nx=1601,
                     nt=2000, half_width=3.0, source=None, vol_t=None):
    """Fully implicit FD for d_t u + 1/2 s(x)^2 u_xx + (r - s^2/2) u_x - r u
    + omega (Phi - u)_+ + source(t, x) = 0, u(T) = Phi, on x = log S in
    [log S0 - half_width, log S0 + half_width] with Dirichlet data from the
    payoff (put: K e^{-r(T-t)} - S at the left, 0 at the right).  The
    penalty is solved by policy iteration at every time step.  vol(x) is a
    callable of the log-price; vol_t(t, x), if given, a time-dependent one
    (evaluated at the time of each implicit step).  Returns (x grid, list
    of u at t_n, t grid)."""
    x = np.linspace(math.log(S0) - half_width, math.log(S0) + half_width, nx)
    dx = x[1] - x[0]
    dt = T / nt
    s2 = vol(x) ** 2
    if payoff == "put":
        phi = np.maximum(K - np.exp(x), 0.0)
    else:
        phi = np.maximum(np.exp(x) - K, 0.0)
    a = 0.5 * s2 / dx ** 2
    b = (r - 0.5 * s2) / (2 * dx)
    lower = a - b            # coefficient of u_{i-1}
    diag = -2 * a - r        # coefficient of u_i
    upper = a + b            # coefficient of u_{i+1}
    u = phi.copy()
    ts = [T]
    us = [u.copy()]
    for n in range(nt - 1, -1, -1):
        t = n * dt
        if vol_t is not None:
            s2 = vol_t(t, x) ** 2
            a = 0.5 * s2 / dx ** 2
            b = (r - 0.5 * s2) / (2 * dx)
            lower, diag, upper = a - b, -2 * a - r, a + b
        rhs = u.copy()
        if source is not None:
            rhs = rhs + dt * source(t, x)
        active = (phi > u) if omega > 0 else np.zeros(nx, bool)
        for _ in range(50):
            ab = np.zeros((3, nx))
            ab[0, 1:] = -dt * upper[:-1]
            ab[1, :] = 1 - dt * diag + dt * omega * active
            ab[2, :-1] = -dt * lower[1:]
            rr = rhs + dt * omega * active * phi
            # boundaries
            ab[1, 0] = 1.0
            ab[0, 1] = 0.0
            ab[1, -1] = 1.0
            ab[2, -2] = 0.0
            if payoff == "put":
                rr[0] = max(K * math.exp(-r * (T - t)) - math.exp(x[0]), phi[0])
                rr[-1] = 0.0
            else:
                rr[0] = 0.0
                rr[-1] = math.exp(x[-1]) - K * math.exp(-r * (T - t))
            unew = solve_banded((1, 1), ab, rr)
            new_active = (phi > unew) if omega > 0 else active
            if np.array_equal(new_active, active):
                break
            active = new_active
        u = unew
        ts.append(t)
        us.append(u.copy())
    return x, us[::-1], ts[::-1]


def interp_value_delta(x, u, S):
    """Value and dollar delta at price S from an FD solution on log grid."""
    xs = math.log(S)
    val = float(np.interp(xs, x, u))
    du = np.gradient(u, x)
    return val, float(np.interp(xs, x, du)) / S


# --------------------------------------------------------------------------
def monomial_design(pts, T, lo, hi, nu):
    """Design matrix of t^{nu_0} prod x_j^{nu_j} in the mapped variables."""
    z = np.empty_like(pts)
    z[:, 0] = 2 * pts[:, 0] / T - 1
    z[:, 1:] = 2 * (pts[:, 1:] - lo) / (hi - lo) - 1
    B = np.ones((len(pts), len(nu)))
    for l, e in enumerate(nu):
        for v, ev in enumerate(e):
            if ev:
                B[:, l] *= z[:, v] ** ev
    return B


def total_degree_set(dp, eta):
    out = []
    for g in range(eta + 1):
        def rec(prefix, rem, left):
            if left == 1:
                out.append(tuple(prefix + [rem]))
                return
            for v in range(rem, -1, -1):
                rec(prefix + [v], rem - v, left - 1)
        rec([], g, dp)
    return out


def exact_picard_const_vol_1d(S0, K, r, sigma, T, omega, pts, eta, width,
                              K_it, payoff="put", n_leg=24, n_herm=120):
    """Projected Picard iteration with exact expectations for d = 1 and
    constant volatility.  Returns the list of coefficient vectors (monomial
    basis in total-degree order) and of prices u^k(0, log S0)."""
    lo = math.log(S0) - width * sigma * math.sqrt(T)
    hi = math.log(S0) + width * sigma * math.sqrt(T)
    nu = total_degree_set(2, eta)
    B = monomial_design(pts, T, np.array([lo]), np.array([hi]), nu)
    mu = r - 0.5 * sigma ** 2
    gh_x, gh_w = np.polynomial.hermite_e.hermegauss(n_herm)
    gh_w = gh_w / gh_w.sum()
    gl_x, gl_w = np.polynomial.legendre.leggauss(n_leg)

    def phi(xv):
        s = np.exp(xv)
        return np.maximum(K - s, 0) if payoff == "put" else np.maximum(s - K, 0)

    def u_of(alpha, t, xv):
        tt = np.broadcast_to(t, np.shape(xv))
        P = np.stack([tt, xv], axis=-1).reshape(-1, 2)
        return (monomial_design(P, T, np.array([lo]), np.array([hi]), nu)
                @ alpha).reshape(np.shape(xv))

    alpha = np.zeros(len(nu))
    alphas = [alpha.copy()]
    prices = [0.0]
    for _ in range(K_it):
        y = np.empty(len(pts))
        for i, (t0, x0) in enumerate(pts):
            tau = T - t0
            if tau <= 0:
                y[i] = phi(np.array(x0))
                continue
            if payoff == "put":
                term = math.exp(r * tau) * bs_put(math.exp(x0), K, r, sigma, tau)
            else:
                term = math.exp(r * tau) * bs_call(math.exp(x0), K, r, sigma, tau)
            # int_t^T E[f(s, X_s, u^k(s, X_s))] ds by Gauss-Legendre x Hermite
            s = t0 + 0.5 * tau * (gl_x + 1)
            ws = 0.5 * tau * gl_w
            acc = 0.0
            for sv, wv in zip(s, ws):
                xs = x0 + mu * (sv - t0) + sigma * math.sqrt(sv - t0) * gh_x
                uk = u_of(alpha, sv, xs)
                f = -r * uk + omega * np.maximum(phi(xs) - uk, 0.0)
                acc += wv * float(gh_w @ f)
            y[i] = term + acc
        alpha = np.linalg.lstsq(B, y, rcond=None)[0]
        alphas.append(alpha.copy())
        prices.append(float(u_of(alpha, 0.0, np.array(math.log(S0)))))
    return alphas, prices


def exact_picard_const_vol(cfg, pts, K_it, n_leg=16, n_herm=24):
    """Exact-expectation projected Picard iteration in d dimensions for
    constant volatilities, uniform correlation, omega = 0 and the geometric
    put payoff, whose conditional expectation is closed form.  Tensor
    Gauss-Hermite over the correlated Gaussian increment and Gauss-Legendre
    in time make E[int f(u^k)] exact for the polynomial u^k.  Returns the
    prices u^k(0, log S0) for k = 0..K_it.  pts is the (n, d+1) array of
    points, or a function of the iteration k returning the points of that
    iteration (points redrawn every iteration)."""
    pts_of = pts if callable(pts) else (lambda k: pts)
    d = cfg["d"]
    T, r, K = cfg["T"], cfg["r"], cfg["K"]
    sig = np.asarray(cfg["vol_level"], float)
    S0 = np.asarray(cfg["S0"], float)
    assert cfg["payoff"] == "put_geom" and cfg.get("omega", 0.0) == 0.0
    w = cfg.get("width", 4.0)
    lo = np.log(S0) - w * sig * math.sqrt(T)
    hi = np.log(S0) + w * sig * math.sqrt(T)
    nu = total_degree_set(d + 1, cfg["eta"])
    C = np.full((d, d), cfg.get("rho", 0.0))
    np.fill_diagonal(C, 1.0)
    L = np.linalg.cholesky(C)
    mu = r - 0.5 * sig ** 2
    gx, gw = np.polynomial.hermite_e.hermegauss(n_herm)
    gw = gw / gw.sum()
    grids = np.meshgrid(*([gx] * d), indexing="ij")
    Z = np.stack([g.ravel() for g in grids], axis=1)          # (Q, d)
    W = np.ones(len(Z))
    for gwi in np.meshgrid(*([gw] * d), indexing="ij"):
        W = W * gwi.ravel()
    LZ = Z @ L.T * sig                                          # sigma_j (L z)_j
    lx, lw = np.polynomial.legendre.leggauss(n_leg)

    def u_of(alpha, t, X):
        P = np.concatenate([np.full((len(X), 1), t), X], axis=1)
        return monomial_design(P, T, lo, hi, nu) @ alpha

    def geo_put_forward(x0, tau):
        # E[(K - exp(mean X_T))_+] for X_T = x0 + mu tau + sigma L G sqrt(tau)
        m = np.mean(x0) + np.mean(mu) * tau
        v = float(sig @ C @ sig) / d ** 2 * tau
        if v <= 0:
            return max(K - math.exp(m), 0.0)
        F = math.exp(m + v / 2)
        d1 = (math.log(F / K) + v / 2) / math.sqrt(v)
        return K * norm.cdf(-(d1 - math.sqrt(v))) - F * norm.cdf(-d1)

    alpha = np.zeros(len(nu))
    prices = [0.0]
    for k in range(K_it):
        pts = pts_of(k)
        B = monomial_design(pts, T, lo, hi, nu)
        y = np.empty(len(pts))
        for i, row in enumerate(pts):
            t0, x0 = row[0], row[1:]
            tau = T - t0
            acc = geo_put_forward(x0, tau)
            if tau > 0:
                for sv, wv in zip(t0 + 0.5 * tau * (lx + 1), 0.5 * tau * lw):
                    X = x0 + mu * (sv - t0) + math.sqrt(sv - t0) * LZ
                    acc += wv * float(W @ (-r * u_of(alpha, sv, X)))
            y[i] = acc
        alpha = np.linalg.lstsq(B, y, rcond=None)[0]
        prices.append(float(u_of(alpha, 0.0, np.log(S0)[None, :])[0]))
    return prices
