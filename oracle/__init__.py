"""ctypes binding of the FP64 CPU oracle (``bsde_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never does.  The binding
only marshals arguments; every number is computed by the C code, which follows
Algorithm "algodetail" (Section 4.1) of Labart & Lelong, arXiv:1102.4666.

Problems are plain dicts (keys as in ``oracle_problem``; strings for the
enumerations), the same dicts the GPU binding accepts.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
DMAX = 16

VOL_KINDS = {"const": 0, "bump": 1, "dupire": 2}
PAYOFFS = {"put": 0, "call": 1, "put_geom": 2, "call_geom": 3, "fwd": 4,
           "quad": 5}
GRIDS = {"tensor": 0, "random": 1, "uniform": 2}


def build() -> str:
    """Compile the oracle with the host C compiler (plain -O2, one thread)."""
    src = os.path.join(_HERE, "bsde_oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC",
                           "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Problem(C.Structure):
    _fields_ = [
        ("d", C.c_int),
        ("vol_kind", C.c_int),
        ("vol_level", C.c_double * DMAX),
        ("bump_a", C.c_double),
        ("bump_c", C.c_double),
        ("rho", C.c_double),
        ("r", C.c_double),
        ("div", C.c_double * DMAX),
        ("payoff", C.c_int),
        ("K", C.c_double),
        ("T", C.c_double),
        ("S0", C.c_double * DMAX),
        ("grid", C.c_int),
        ("n_t", C.c_int),
        ("n_x", C.c_int),
        ("width", C.c_double),
        ("eta", C.c_int),
        ("q", C.c_double),
        ("M", C.c_int),
        ("N", C.c_int),
        ("K_it", C.c_int),
        ("omega", C.c_double),
        ("seed", C.c_uint64),
        ("redraw", C.c_int),
        ("kernel_bw", C.c_double),
    ]


class PathOut(C.Structure):
    _fields_ = [
        ("jstar", C.c_uint32),
        ("U", C.c_double),
        ("theta", C.c_double),
        ("tau", C.c_double),
        ("xstar", C.c_double * DMAX),
        ("sigstar", C.c_double * DMAX),
        ("bstar", C.c_double * DMAX),
        ("xtau", C.c_double * DMAX),
        ("xT", C.c_double * DMAX),
    ]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_up = C.POINTER(C.c_uint32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Problem)
        L.oracle_philox4x32_10.argtypes = [_up, _up, _up]
        L.oracle_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32,
                                     C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_int, _dp]
        L.oracle_num_points.argtypes = [P]
        L.oracle_index_set.argtypes = [C.c_int, C.c_int, C.c_double, _ip,
                                       C.c_int]
        L.oracle_num_basis.argtypes = [P]
        L.oracle_domain.argtypes = [P, _dp, _dp]
        L.oracle_points.argtypes = [P, _dp]
        L.oracle_points_k.argtypes = [P, C.c_uint32, _dp]
        L.oracle_cholesky.argtypes = [C.c_int, C.c_double, _dp]
        L.oracle_lstsq.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.oracle_payoff.argtypes = [P, _dp]
        L.oracle_payoff.restype = C.c_double
        L.oracle_vol.argtypes = [P, C.c_int, C.c_double, C.c_double]
        L.oracle_vol.restype = C.c_double
        L.oracle_eval.argtypes = [P, _ip, C.c_int, _dp, C.c_double, _dp,
                                  _dp, _dp, _dp, _dp]
        L.oracle_path.argtypes = [P, C.c_double, _dp, C.c_uint32,
                                  C.c_uint32, C.c_uint32, C.POINTER(PathOut)]
        L.oracle_path_term.argtypes = [P, _ip, C.c_int, _dp, C.c_double, _dp,
                                       C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_path_term.restype = C.c_double
        L.oracle_corrections.argtypes = [P, _dp, C.c_uint32, C.c_int,
                                         C.c_int, _dp, _dp]
        L.oracle_solve.argtypes = [P, C.c_int, _dp, C.c_int, _dp, _dp, _dp,
                                   _dp]
        L.oracle_fit.argtypes = [P, _dp, _dp]
        L.oracle_basis_matrix.argtypes = [P, _dp]
        L.oracle_basis_matrix_k.argtypes = [P, C.c_uint32, _dp]
        L.oracle_price_delta.argtypes = [P, _dp, C.c_int, _dp, _dp, _dp,
                                         _dp]
        L.oracle_kernel_eval.argtypes = [P, _dp, _dp, C.c_int, C.c_double,
                                         _dp, _dp, _dp, _dp, _dp]
        L.oracle_kernel_corrections.argtypes = [P, _dp, C.c_uint32, C.c_int,
                                                C.c_int, _dp, _dp]
        L.oracle_kernel_solve.argtypes = [P, _dp, _dp, _dp, _dp]
        L.oracle_kernel_price_delta.argtypes = [P, _dp, C.c_int, _dp, _dp,
                                                _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def make_problem(cfg: dict) -> Problem:
    p = Problem()
    d = int(cfg["d"])
    if not 1 <= d <= DMAX:
        raise ValueError("d out of range")
    p.d = d
    p.vol_kind = VOL_KINDS[cfg.get("vol_kind", "const")]
    lev = np.broadcast_to(np.asarray(cfg["vol_level"], float), (d,))
    div = np.broadcast_to(np.asarray(cfg.get("div", 0.0), float), (d,))
    s0 = np.broadcast_to(np.asarray(cfg["S0"], float), (d,))
    for j in range(d):
        p.vol_level[j] = lev[j]
        p.div[j] = div[j]
        p.S0[j] = s0[j]
    p.bump_a = float(cfg.get("bump_a", 0.0))
    p.bump_c = float(cfg.get("bump_c", 100.0))
    p.rho = float(cfg.get("rho", 0.0))
    p.r = float(cfg["r"])
    p.payoff = PAYOFFS[cfg.get("payoff", "put")]
    p.K = float(cfg["K"])
    p.T = float(cfg["T"])
    p.grid = GRIDS[cfg.get("grid", "tensor")]
    p.n_t = int(cfg["n_t"])
    p.n_x = int(cfg["n_x"])
    p.width = float(cfg.get("width", 4.0))
    p.eta = int(cfg["eta"])
    p.q = float(cfg.get("q", 1.0))
    p.M = int(cfg["M"])
    p.N = int(cfg["N"])
    p.K_it = int(cfg["K_it"])
    p.omega = float(cfg.get("omega", 0.0))
    p.seed = int(cfg.get("seed", 0))
    p.redraw = int(bool(cfg.get("redraw", 0)))
    p.kernel_bw = float(cfg.get("kernel_bw", 0.0))
    return p


def kernel_op(cfg) -> bool:
    """True when cfg asks for the kernel operator of Section 3.2."""
    return float(cfg.get("kernel_bw", 0.0)) > 0.0


# ----------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c.ctypes.data_as(_up), k.ctypes.data_as(_up),
                               out.ctypes.data_as(_up))
    return out


def normals(seed, m, i, k, sub, first_block, count):
    out = np.zeros(count)
    lib().oracle_normals(seed, m, i, k, sub, first_block, count, _d(out))
    return out


def index_set(dp, eta, q=1.0):
    p = lib().oracle_index_set(dp, eta, q, None, 0)
    nu = np.zeros((p, dp), dtype=np.int32)
    lib().oracle_index_set(dp, eta, q, _i(nu), p)
    return nu


def sizes(cfg):
    pb = make_problem(cfg)
    return lib().oracle_num_points(C.byref(pb)), lib().oracle_num_basis(
        C.byref(pb))


def domain(cfg):
    pb = make_problem(cfg)
    lo = np.zeros(pb.d)
    hi = np.zeros(pb.d)
    lib().oracle_domain(C.byref(pb), _d(lo), _d(hi))
    return lo, hi


def points(cfg, k=0):
    """The points of Picard iteration k (the fixed grid unless redraw)."""
    pb = make_problem(cfg)
    n = lib().oracle_num_points(C.byref(pb))
    pts = np.zeros((n, pb.d + 1))
    lib().oracle_points_k(C.byref(pb), k, _d(pts))
    return pts


def cholesky(d, rho):
    L = np.zeros((d, d))
    st = lib().oracle_cholesky(d, rho, _d(L))
    if st:
        raise ValueError("correlation matrix not positive definite")
    return L


def lstsq(B, y):
    B = np.ascontiguousarray(B, float)
    y = np.ascontiguousarray(y, float)
    n, p = B.shape
    a = np.zeros(p)
    st = lib().oracle_lstsq(n, p, _d(B), _d(y), _d(a))
    if st:
        raise np.linalg.LinAlgError("rank deficient (status %d)" % st)
    return a


def payoff(cfg, x):
    pb = make_problem(cfg)
    x = np.ascontiguousarray(x, float)
    return lib().oracle_payoff(C.byref(pb), _d(x))


def vol(cfg, j, t, xj):
    pb = make_problem(cfg)
    return lib().oracle_vol(C.byref(pb), j, t, xj)


def evaluate(cfg, alpha, t, x):
    """u, u_t, grad_x u, hess_x u of the oracle's expansion at (t, x)."""
    pb = make_problem(cfg)
    nu = index_set(pb.d + 1, pb.eta, pb.q)
    a = np.ascontiguousarray(alpha, float)
    x = np.ascontiguousarray(x, float)
    u = np.zeros(1)
    ut = np.zeros(1)
    ux = np.zeros(pb.d)
    uxx = np.zeros((pb.d, pb.d))
    lib().oracle_eval(C.byref(pb), _i(nu), len(nu), _d(a), t, _d(x), _d(u),
                      _d(ut), _d(ux), _d(uxx))
    return u[0], ut[0], ux, uxx


def path(cfg, t0, x0, i, m, k):
    pb = make_problem(cfg)
    x0 = np.ascontiguousarray(np.broadcast_to(np.asarray(x0, float),
                                              (pb.d,)))
    out = PathOut()
    lib().oracle_path(C.byref(pb), t0, _d(x0), i, m, k, C.byref(out))
    d = pb.d
    return {
        "jstar": out.jstar, "U": out.U, "theta": out.theta, "tau": out.tau,
        "xstar": np.array(out.xstar[:d]), "sigstar": np.array(out.sigstar[:d]),
        "bstar": np.array(out.bstar[:d]), "xtau": np.array(out.xtau[:d]),
        "xT": np.array(out.xT[:d]),
    }


def path_term(cfg, alpha, t0, x0, i, m, k):
    pb = make_problem(cfg)
    nu = index_set(pb.d + 1, pb.eta, pb.q)
    x0 = np.ascontiguousarray(np.broadcast_to(np.asarray(x0, float),
                                              (pb.d,)))
    a = None if alpha is None else np.ascontiguousarray(alpha, float)
    return lib().oracle_path_term(C.byref(pb), _i(nu), len(nu),
                                  None if a is None else _d(a), t0, _d(x0), i,
                                  m, k)


def corrections(cfg, alpha, k, i_begin, i_end):
    """c_i, var_i for points i_begin..i_end-1 at iteration k; alpha is the
    coefficient vector of u^k (the point values y^{k-1} with the kernel
    operator), None for u^k = 0."""
    pb = make_problem(cfg)
    cnt = i_end - i_begin
    c = np.zeros(cnt)
    v = np.zeros(cnt)
    a = None if alpha is None else np.ascontiguousarray(alpha, float)
    fn = lib().oracle_kernel_corrections if kernel_op(cfg) else lib().oracle_corrections
    fn(C.byref(pb), None if a is None else _d(a), k, i_begin, i_end, _d(c), _d(v))
    return c, v


def kernel_eval(cfg, y, t, x):
    """u, u_t, grad_x u, hess_x u of the kernel operator applied to the
    values y at the problem's points, at (t, x)."""
    pb = make_problem(cfg)
    pts = np.ascontiguousarray(points(cfg, 0))
    y = np.ascontiguousarray(y, float)
    x = np.ascontiguousarray(np.broadcast_to(np.asarray(x, float), (pb.d,)))
    u, ut = np.zeros(1), np.zeros(1)
    ux, uxx = np.zeros(pb.d), np.zeros((pb.d, pb.d))
    lib().oracle_kernel_eval(C.byref(pb), _d(pts), _d(y), len(pts), t, _d(x),
                             _d(u), _d(ut), _d(ux), _d(uxx))
    return u[0], ut[0], ux, uxx


def solve(cfg, k_start=0, alpha_start=None, k_end=None):
    """Run Picard iterations k_start..k_end-1; returns a dict of histories.
    With the kernel operator (cfg kernel_bw > 0) the whole loop runs from
    u^0 = 0 and "alpha" holds the point values: row 0 zeros, row k + 1 = y^k
    (u^{k+1} is the kernel operator applied to row k + 1)."""
    pb = make_problem(cfg)
    if kernel_op(cfg):
        if k_start != 0 or alpha_start is not None or k_end not in (None, pb.K_it):
            raise ValueError("the kernel operator runs whole solves only")
        n = lib().oracle_num_points(C.byref(pb))
        yh = np.zeros((pb.K_it + 1, n))
        ch = np.zeros((pb.K_it, n))
        vh = np.zeros((pb.K_it, n))
        uh = np.zeros((pb.K_it, n))
        st = lib().oracle_kernel_solve(C.byref(pb), _d(yh), _d(ch), _d(vh), _d(uh))
        if st:
            raise RuntimeError("oracle_kernel_solve failed with status %d" % st)
        return {"alpha": yh, "c": ch, "var": vh, "u": uh, "n": n, "p": n}
    if k_end is None:
        k_end = pb.K_it
    n = lib().oracle_num_points(C.byref(pb))
    p = lib().oracle_num_basis(C.byref(pb))
    nk = k_end - k_start
    ah = np.zeros((nk + 1, p))
    ch = np.zeros((nk, n))
    vh = np.zeros((nk, n))
    uh = np.zeros((nk, n))
    a0 = None if alpha_start is None else np.ascontiguousarray(alpha_start,
                                                               float)
    st = lib().oracle_solve(C.byref(pb), k_start,
                            None if a0 is None else _d(a0), k_end, _d(ah),
                            _d(ch), _d(vh), _d(uh))
    if st:
        raise RuntimeError("oracle_solve failed with status %d" % st)
    return {"alpha": ah, "c": ch, "var": vh, "u": uh, "n": n, "p": p}


def basis_matrix(cfg, k=0):
    pb = make_problem(cfg)
    n = lib().oracle_num_points(C.byref(pb))
    p = lib().oracle_num_basis(C.byref(pb))
    B = np.zeros((n, p))
    lib().oracle_basis_matrix_k(C.byref(pb), k, _d(B))
    return B


def solve_parallel(cfg, workers=8, chunk=64, k_start=0, alpha_start=None,
                   k_end=None, progress=None):
    """The same loop as ``solve`` (the same oracle functions, in the same
    order per point), with the per-point corrections of each iteration
    spread over worker processes.  Results are identical to ``solve``."""
    import multiprocessing as mp
    if kernel_op(cfg):
        raise ValueError("solve_parallel covers the least-squares operator")
    pb = make_problem(cfg)
    if k_end is None:
        k_end = pb.K_it
    B = basis_matrix(cfg)
    n, p = B.shape
    alpha = np.zeros(p) if alpha_start is None else np.array(alpha_start, float)
    have = alpha_start is not None
    ah = [alpha.copy()]
    ch, vh, uh = [], [], []
    ranges = [(i, min(i + chunk, n)) for i in range(0, n, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        redraw = bool(cfg.get("redraw", 0)) and cfg.get("grid") in ("random", "uniform")
        for k in range(k_start, k_end):
            if redraw:
                B = basis_matrix(cfg, k)
            args = [(cfg, alpha if have else None, k, a, b) for a, b in ranges]
            parts = pool.starmap(corrections, args)
            c = np.concatenate([x[0] for x in parts])
            v = np.concatenate([x[1] for x in parts])
            u = _rowdot(B, alpha)
            alpha = lstsq(B, u + c)
            have = True
            ah.append(alpha.copy())
            ch.append(c)
            vh.append(v)
            uh.append(u)
            if progress:
                progress(k)
    return {"alpha": np.array(ah), "c": np.array(ch), "var": np.array(vh),
            "u": np.array(uh), "n": n, "p": p}


def _rowdot(B, alpha):
    # u_i = sum_l alpha_l B_il summed in l order, as in oracle_solve
    u = np.zeros(B.shape[0])
    for l in range(B.shape[1]):
        u = u + alpha[l] * B[:, l]
    return u


def fit(cfg, y):
    pb = make_problem(cfg)
    p = lib().oracle_num_basis(C.byref(pb))
    y = np.ascontiguousarray(y, float)
    a = np.zeros(p)
    st = lib().oracle_fit(C.byref(pb), _d(y), _d(a))
    if st:
        raise np.linalg.LinAlgError("fit failed (status %d)" % st)
    return a


def price_delta(cfg, alpha, t, S):
    """Price and dollar deltas of u = sum alpha_l B_l (the kernel operator
    applied to point values alpha when cfg asks for it) at (t, S)."""
    pb = make_problem(cfg)
    t = np.ascontiguousarray(np.atleast_1d(t), float)
    S = np.ascontiguousarray(np.asarray(S, float).reshape(len(t), pb.d))
    a = np.ascontiguousarray(alpha, float)
    price = np.zeros(len(t))
    delta = np.zeros((len(t), pb.d))
    fn = lib().oracle_kernel_price_delta if kernel_op(cfg) else lib().oracle_price_delta
    fn(C.byref(pb), _d(a), len(t), _d(t), _d(S), _d(price), _d(delta))
    return price, delta
