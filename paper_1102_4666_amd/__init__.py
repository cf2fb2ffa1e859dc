"""Python binding of libbsde.so, the MI355X (gfx950) BSDE solver library.

Argument marshalling only: every step of a solve runs in the library's HIP
kernels (the method of Labart & Lelong, arXiv:1102.4666, Algorithm
"algodetail").  The functions carry the names of the C entry points declared
in ``include/bsde.h``; ``Problem`` wraps a handle for convenience.  Problems
are plain dicts (see ``workloads.py``).

Importing this module does not need a GPU; loading the library does need
``libbsde.so`` (build it with ``python -m paper_1102_4666_amd.build``) and
raises if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsde.so")

VOL_KINDS = {"const": 0, "bump": 1, "dupire": 2}
PAYOFFS = {"put": 0, "call": 1, "put_geom": 2, "call_geom": 3, "fwd": 4,
           "quad": 5}
GRIDS = {"tensor": 0, "random": 1, "uniform": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}

STATUS = {0: "BSDE_OK", 1: "BSDE_EINVAL", 2: "BSDE_ENOMEM", 3: "BSDE_ERANK",
          4: "BSDE_EDEVICE", 5: "BSDE_ESTATE", 6: "BSDE_EUNSUPPORTED",
          7: "BSDE_EBUSY"}

EXPORTS = [
    "bsde_create_problem", "bsde_solve", "bsde_query_price_delta",
    "bsde_problem_sizes", "bsde_get_points", "bsde_get_coefficients",
    "bsde_set_coefficients", "bsde_fit_values", "bsde_get_corrections",
    "bsde_set_tiling", "bsde_autotune", "bsde_last_timings", "bsde_set_timing",
    "bsde_get_tiling", "bsde_autotune_save", "bsde_autotune_load",
    "bsde_solve_batch", "bsde_solve_batch_noalloc",
    "bsde_destroy", "bsde_status_string", "bsde_last_error",
    "bsde_server_create", "bsde_server_submit", "bsde_server_poll",
    "bsde_server_stats", "bsde_server_destroy",
]
BSDE_BATCH_GRAPH = 1


class BsdeError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = "%s failed: %s (%s)" % (where, STATUS.get(status, status),
                                      last_error())
        super().__init__(msg)


class Sigma(C.Structure):
    _fields_ = [("kind", C.c_int), ("level", C.POINTER(C.c_double)),
                ("bump_a", C.c_double), ("bump_c", C.c_double),
                ("rho", C.c_double), ("dividend", C.POINTER(C.c_double))]


class Payoff(C.Structure):
    _fields_ = [("kind", C.c_int), ("K", C.c_double), ("T", C.c_double),
                ("S0", C.POINTER(C.c_double))]


class Grid(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_t", C.c_int), ("n_x", C.c_int),
                ("width", C.c_double), ("eta", C.c_int), ("q", C.c_double),
                ("redraw", C.c_int), ("kernel_bw", C.c_double)]


class Request(C.Structure):
    _fields_ = [("d", C.c_int), ("sigma", Sigma), ("r", C.c_double),
                ("payoff", Payoff), ("grid", Grid), ("M", C.c_int),
                ("N", C.c_int), ("n_picard", C.c_int), ("penalty", C.c_double),
                ("seed", C.c_ulonglong), ("precision", C.c_int),
                ("query_t", C.c_double), ("query_S", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("price", C.c_double),
                ("delta", C.c_double * 10), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double), ("engine_steps", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("requests_per_s", C.c_double),
                ("path_steps_per_s", C.c_double), ("completed", C.c_long),
                ("engine_steps", C.c_long), ("in_flight", C.c_long),
                ("pending", C.c_long), ("reserved_bytes", C.c_size_t)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    """Loads libbsde.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbsde.so is not built; run "
                              "`python -m paper_1102_4666_amd.build`")
        # One HIP runtime per process: PyTorch ships its own copy of the
        # runtime library under the same soname, and whichever is loaded
        # first serves every later user.  Loading torch first binds the
        # library to torch's runtime, so that torch's streams and device
        # memory are valid handles here (and torch still initialises after
        # the library has touched the device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        L.bsde_create_problem.argtypes = [
            C.c_int, C.POINTER(Sigma), C.c_double, C.POINTER(Payoff),
            C.POINTER(Grid), C.c_int, C.c_int, C.c_int, C.c_double,
            C.c_ulonglong, C.c_int, C.POINTER(H)]
        L.bsde_solve.argtypes = [H, C.c_void_p]
        L.bsde_query_price_delta.argtypes = [H, C.c_int, _dp, _dp, _dp, _dp]
        L.bsde_problem_sizes.argtypes = [H, _ip, _ip, _ip]
        L.bsde_get_points.argtypes = [H, _dp]
        L.bsde_get_coefficients.argtypes = [H, C.c_int, _dp, _ip]
        L.bsde_set_coefficients.argtypes = [H, _dp, C.c_int]
        L.bsde_fit_values.argtypes = [H, _dp, C.c_int]
        L.bsde_get_corrections.argtypes = [H, C.c_int, _dp, _dp]
        L.bsde_set_tiling.argtypes = [H, C.c_int, C.c_int]
        L.bsde_last_timings.argtypes = [H, _dp]
        L.bsde_set_timing.argtypes = [H, C.c_int]
        L.bsde_autotune.argtypes = [H, C.c_void_p, _ip, _ip, _dp]
        L.bsde_get_tiling.argtypes = [H, _ip, _ip]
        L.bsde_autotune_save.argtypes = [C.c_char_p, _ip]
        L.bsde_autotune_load.argtypes = [C.c_char_p, _ip]
        L.bsde_solve_batch.argtypes = [C.POINTER(H), C.c_int, C.c_void_p,
                                       C.c_int, _dp]
        L.bsde_solve_batch_noalloc.argtypes = [C.POINTER(H), C.c_int, C.c_void_p]
        L.bsde_server_create.argtypes = [C.c_size_t, C.c_int, C.c_int,
                                         C.POINTER(H)]
        L.bsde_server_submit.argtypes = [H, C.POINTER(Request),
                                         C.POINTER(C.c_ulonglong)]
        L.bsde_server_poll.argtypes = [H, C.c_ulonglong, C.c_int,
                                       C.POINTER(Result)]
        L.bsde_server_stats.argtypes = [H, C.POINTER(ServerStats)]
        L.bsde_server_destroy.argtypes = [H]
        L.bsde_server_destroy.restype = None
        L.bsde_destroy.argtypes = [H]
        L.bsde_destroy.restype = None
        L.bsde_status_string.argtypes = [C.c_int]
        L.bsde_status_string.restype = C.c_char_p
        L.bsde_last_error.argtypes = []
        L.bsde_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("bsde_destroy", "bsde_status_string",
                            "bsde_last_error", "bsde_server_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().bsde_last_error().decode()


def _check(status, where):
    if status != 0:
        raise BsdeError(status, where)


def _arr(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _d(a):
    return a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# --------------------------------------------------------------------------
def _marshal(cfg: dict):
    """The C structs of a problem dict and the arrays they point to."""
    d = int(cfg["d"])
    level = _arr(np.broadcast_to(np.asarray(cfg["vol_level"], float), (d,)))
    div = _arr(np.broadcast_to(np.asarray(cfg.get("div", 0.0), float), (d,)))
    S0 = _arr(np.broadcast_to(np.asarray(cfg["S0"], float), (d,)))
    sig = Sigma(VOL_KINDS[cfg.get("vol_kind", "const")], _d(level),
                float(cfg.get("bump_a", 0.0)), float(cfg.get("bump_c", 100.0)),
                float(cfg.get("rho", 0.0)), _d(div))
    pay = Payoff(PAYOFFS[cfg.get("payoff", "put")], float(cfg["K"]),
                 float(cfg["T"]), _d(S0))
    grid = Grid(GRIDS[cfg.get("grid", "tensor")], int(cfg["n_t"]),
                int(cfg["n_x"]), float(cfg.get("width", 4.0)),
                int(cfg["eta"]), float(cfg.get("q", 1.0)),
                int(bool(cfg.get("redraw", 0))), float(cfg.get("kernel_bw", 0.0)))
    return d, sig, pay, grid, (level, div, S0)


def bsde_create_problem(cfg: dict):
    """Marshals a problem dict into bsde_create_problem; returns the
    handle (a c_void_p)."""
    d, sig, pay, grid, keep = _marshal(cfg)
    h = C.c_void_p()
    st = lib().bsde_create_problem(
        d, C.byref(sig), float(cfg["r"]), C.byref(pay), C.byref(grid),
        int(cfg["M"]), int(cfg["N"]), int(cfg["K_it"]),
        float(cfg.get("omega", 0.0)), int(cfg.get("seed", 0)),
        PRECISIONS[cfg.get("precision", "fp64")], C.byref(h))
    _check(st, "bsde_create_problem")
    return h


def bsde_solve(h, stream=None):
    """stream: a HIP stream handle as int (e.g. torch's
    ``torch.cuda.current_stream().cuda_stream``) or None."""
    _check(lib().bsde_solve(h, C.c_void_p(stream or 0)), "bsde_solve")


def bsde_problem_sizes(h):
    n, p, c = C.c_int(), C.c_int(), C.c_int()
    _check(lib().bsde_problem_sizes(h, C.byref(n), C.byref(p), C.byref(c)),
           "bsde_problem_sizes")
    return n.value, p.value, c.value


def bsde_query_price_delta(h, d, t, S):
    t = _arr(np.atleast_1d(t))
    S = _arr(S, len(t) * d)
    price = np.zeros(len(t))
    delta = np.zeros((len(t), d))
    _check(lib().bsde_query_price_delta(h, len(t), _d(t), _d(S), _d(price),
                                        _d(delta)), "bsde_query_price_delta")
    return price, delta


def bsde_get_points(h, n, d):
    pts = np.zeros((n, d + 1))
    _check(lib().bsde_get_points(h, _d(pts)), "bsde_get_points")
    return pts


def bsde_get_coefficients(h, p, k=-1):
    a = np.zeros(p)
    kd = C.c_int()
    _check(lib().bsde_get_coefficients(h, k, _d(a), C.byref(kd)),
           "bsde_get_coefficients")
    return a, kd.value


def bsde_set_coefficients(h, alpha, k_done):
    a = _arr(alpha)
    _check(lib().bsde_set_coefficients(h, _d(a), int(k_done)),
           "bsde_set_coefficients")


def bsde_fit_values(h, y, k_done):
    y = _arr(y)
    _check(lib().bsde_fit_values(h, _d(y), int(k_done)), "bsde_fit_values")


def bsde_get_corrections(h, n, k):
    c = np.zeros(n)
    v = np.zeros(n)
    _check(lib().bsde_get_corrections(h, int(k), _d(c), _d(v)),
           "bsde_get_corrections")
    return c, v


def bsde_set_tiling(h, groups_per_point, paths_per_lane):
    _check(lib().bsde_set_tiling(h, int(groups_per_point),
                                 int(paths_per_lane)), "bsde_set_tiling")


def bsde_autotune(h, stream=None):
    g, p_, ms = C.c_int(), C.c_int(), C.c_double()
    _check(lib().bsde_autotune(h, C.c_void_p(stream or 0), C.byref(g),
                               C.byref(p_), C.byref(ms)), "bsde_autotune")
    return g.value, p_.value, ms.value


def bsde_get_tiling(h):
    g, p_ = C.c_int(), C.c_int()
    _check(lib().bsde_get_tiling(h, C.byref(g), C.byref(p_)), "bsde_get_tiling")
    return g.value, p_.value


def bsde_autotune_save(path):
    """Write the tilings recorded by bsde_autotune in this process to path;
    returns the number of records."""
    n = C.c_int()
    _check(lib().bsde_autotune_save(os.fsencode(path), C.byref(n)), "bsde_autotune_save")
    return n.value


def bsde_autotune_load(path):
    """Merge the tilings recorded in path for this device's architecture;
    returns the number of records taken."""
    n = C.c_int()
    _check(lib().bsde_autotune_load(os.fsencode(path), C.byref(n)), "bsde_autotune_load")
    return n.value


def bsde_set_timing(h, level):
    _check(lib().bsde_set_timing(h, int(level)), "bsde_set_timing")


def bsde_last_timings(h):
    t = np.zeros(5)
    _check(lib().bsde_last_timings(h, _d(t)), "bsde_last_timings")
    return t


def bsde_solve_batch(handles, stream=None, graph=False):
    """Solves the problems together; returns the GPU time in ms."""
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    ms = C.c_double()
    _check(lib().bsde_solve_batch(arr, len(handles), C.c_void_p(stream or 0),
                                  BSDE_BATCH_GRAPH if graph else 0,
                                  C.byref(ms)), "bsde_solve_batch")
    return ms.value


def solve_batch(problems, stream=None, graph=False):
    """bsde_solve_batch over Problem objects."""
    return bsde_solve_batch([P.h for P in problems], stream, graph)


def bsde_solve_batch_noalloc(handles, stream=None):
    """The batched solve with its tables in the library's fixed workspace
    (no device allocation)."""
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    _check(lib().bsde_solve_batch_noalloc(arr, len(handles), C.c_void_p(stream or 0)),
           "bsde_solve_batch_noalloc")


def solve_batch_noalloc(problems, stream=None):
    """bsde_solve_batch_noalloc over Problem objects."""
    bsde_solve_batch_noalloc([P.h for P in problems], stream)


def bsde_destroy(h):
    if h:
        lib().bsde_destroy(h)


# --------------------------------------------------------------------------
class Problem:
    """Owns one library problem handle."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.d = int(cfg["d"])
        self.h = bsde_create_problem(self.cfg)
        self.n, self.p, self.C = bsde_problem_sizes(self.h)

    def solve(self, stream=None):
        bsde_solve(self.h, stream)
        return self

    def price_delta(self, t=0.0, S=None):
        if S is None:
            S = self.cfg["S0"]
        t = np.atleast_1d(np.asarray(t, float))
        S = np.asarray(S, float).reshape(len(t), self.d)
        return bsde_query_price_delta(self.h, self.d, t, S)

    def points(self):
        return bsde_get_points(self.h, self.n, self.d)

    def coefficients(self, k=-1):
        return bsde_get_coefficients(self.h, self.p, k)[0]

    def set_coefficients(self, alpha, k_done):
        bsde_set_coefficients(self.h, alpha, k_done)

    def fit_values(self, y, k_done=0):
        bsde_fit_values(self.h, y, k_done)

    def corrections(self, k):
        return bsde_get_corrections(self.h, self.n, k)

    def set_tiling(self, groups_per_point, paths_per_lane):
        bsde_set_tiling(self.h, groups_per_point, paths_per_lane)

    def timings(self):
        return bsde_last_timings(self.h)

    def set_timing(self, level):
        """0 = whole solve only, 1 = path kernel per iteration (default),
        2 = every kernel (each level adds event records to the stream)."""
        bsde_set_timing(self.h, level)

    def tiling(self):
        return bsde_get_tiling(self.h)

    def autotune(self, stream=None):
        """(groups per point, paths per lane, path-kernel ms) chosen."""
        return bsde_autotune(self.h, stream)

    def close(self):
        if self.h:
            bsde_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# --------------------------------------------------------------------------
class Server:
    """Continuous-batching request server (bsde_server_*)."""

    def __init__(self, hbm_budget_bytes, max_inflight=64, setup_threads=0):
        self.h = C.c_void_p()
        _check(lib().bsde_server_create(int(hbm_budget_bytes),
                                        int(max_inflight), int(setup_threads),
                                        C.byref(self.h)), "bsde_server_create")

    def submit(self, cfg: dict, query_t=0.0, query_S=None) -> int:
        d, sig, pay, grid, keep = _marshal(cfg)
        qS = None
        if query_S is not None:
            qS = _arr(np.broadcast_to(np.asarray(query_S, float), (d,)))
        req = Request(d, sig, float(cfg["r"]), pay, grid, int(cfg["M"]),
                      int(cfg["N"]), int(cfg["K_it"]),
                      float(cfg.get("omega", 0.0)), int(cfg.get("seed", 0)),
                      PRECISIONS[cfg.get("precision", "fp64")],
                      float(query_t), _d(qS) if qS is not None else None)
        t = C.c_ulonglong()
        _check(lib().bsde_server_submit(self.h, C.byref(req), C.byref(t)),
               "bsde_server_submit")
        return t.value

    def poll(self, ticket: int, wait=True):
        """dict of the result, or None if not finished (wait=False)."""
        r = Result()
        st = lib().bsde_server_poll(self.h, ticket, 1 if wait else 0,
                                    C.byref(r))
        if st == 7:
            return None
        _check(st, "bsde_server_poll")
        return {"status": r.status, "price": r.price,
                "delta": np.array(r.delta[:]), "latency_ms": r.latency_ms,
                "queue_ms": r.queue_ms, "engine_steps": r.engine_steps}

    def stats(self):
        st = ServerStats()
        _check(lib().bsde_server_stats(self.h, C.byref(st)),
               "bsde_server_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            lib().bsde_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
