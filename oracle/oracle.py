"""ctypes binding of the C oracle (mmas_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg. The product library never loads it.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PHER_DENSE = 0
PHER_CANDIDATES = 1

_lib = None


def use_library(path: str):
    """Load the oracle from another build of the same sources (e.g. the
    -march=native build of build.build(native=True)) for the rest of the
    process; call before the first use."""
    global _lib, LIB_PATH
    if _lib is not None and LIB_PATH != path:
        raise RuntimeError("the oracle library is already loaded")
    LIB_PATH = path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_draw_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_draw_word.restype = C.c_uint32
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_float
        L.orc_logf.argtypes = [C.c_float]
        L.orc_logf.restype = C.c_float
        L.orc_logf_n.argtypes = [C.c_int64, p, p]
        L.orc_u01_n.argtypes = [C.c_int64, p, p]
        L.orc_draw_words_n.argtypes = [C.c_int64, C.c_uint64, p, p, p, p, p]
        L.orc_start_node.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_start_node.restype = C.c_uint32
        L.orc_create.argtypes = [C.c_int, p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float,
                                 C.c_double, C.c_uint64, C.c_int, C.c_int]
        L.orc_create.restype = p
        L.orc_destroy.argtypes = [p]
        L.orc_set_deposit.argtypes = [p, C.c_int]
        L.orc_set_deposit.restype = C.c_int
        L.orc_set_select.argtypes = [p, C.c_int]
        L.orc_set_select.restype = C.c_int
        L.orc_set_problem.argtypes = [p, C.c_int]
        L.orc_set_problem.restype = C.c_int
        L.orc_prepare_choice.argtypes = [p]
        L.orc_construct.argtypes = [p, C.c_uint32, C.c_int]
        L.orc_two_opt.argtypes = [p, C.c_int]
        L.orc_update.argtypes = [p]
        L.orc_iterate.argtypes = [p, C.c_uint32, C.c_int]
        L.orc_select_next.argtypes = [p, C.c_int, p, C.c_uint32, C.c_uint32, C.c_uint32, p]
        L.orc_select_next.restype = C.c_int
        L.orc_n.argtypes = [p]
        L.orc_n.restype = C.c_int
        L.orc_cl.argtypes = [p]
        L.orc_cl.restype = C.c_int
        for name in ("orc_get_tours", "orc_get_lengths", "orc_get_pheromone", "orc_set_pheromone",
                     "orc_get_choice", "orc_get_chc", "orc_get_cand", "orc_get_heuristic",
                     "orc_get_limits", "orc_get_iteration_best"):
            getattr(L, name).argtypes = [p, p]
        L.orc_get_fallback.argtypes = [p, p, p]
        L.orc_set_heuristic.argtypes = [p, p]
        L.orc_set_heuristic.restype = C.c_int
        L.orc_get_best.argtypes = [p, p]
        L.orc_restore.argtypes = [p, p, C.c_int64, p]
        L.orc_get_best.restype = C.c_int64
        L.orc_get_nn_tour.argtypes = [p, p]
        L.orc_get_nn_tour.restype = C.c_int64
        L.orc_limits.argtypes = [C.c_float, C.c_int64, C.c_int, C.c_double, p, p]
        L.orc_nearest.argtypes = [C.c_int, p, C.c_int, p]
        L.orc_nn_tour.argtypes = [C.c_int, p, p]
        L.orc_nn_tour.restype = C.c_int64
        L.orc_two_opt_tour.argtypes = [C.c_int, p, p, C.c_int, p]
        L.orc_two_opt_tour.restype = C.c_int64
        L.orc_tour_length.argtypes = [C.c_int, p, p]
        L.orc_tour_length.restype = C.c_int64
        L.orc_bf16_round.argtypes = [C.c_float]
        L.orc_bf16_round.restype = C.c_float
        L.orc_expf.argtypes = [C.c_float]
        L.orc_expf.restype = C.c_float
        L.orc_knn_features.argtypes = [C.c_int, p, p, p, p]
        L.orc_mlp_forward.argtypes = [C.c_int64, p, p, p, p, p, p, C.c_float, C.c_int, p]
        L.orc_mlp_backward.argtypes = [C.c_int64, p, p, p, p, p, p, p, C.c_float, C.c_int, p, p, p, p, p, p]
        L.orc_mlp_backward.restype = C.c_double
        L.orc_adam.argtypes = [C.c_int64, p, p, p, p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float,
                               C.c_float]
        L.orc_install_eta.argtypes = [C.c_int, p, p, p, C.c_int, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def pdec_of(p_best: float, n: int) -> float:
    """p_best^(1/n) through the C library's pow (math.pow)."""
    return math.pow(p_best, 1.0 / n)


# ---- random numbers ----
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw_word(seed, it, ant, step, slot) -> int:
    return int(lib().orc_draw_word(seed, it, ant, step, slot))


def u01(x: int) -> float:
    return float(np.float32(lib().orc_u01(x)))


def logf(u: float) -> np.float32:
    return np.float32(lib().orc_logf(float(np.float32(u))))


def logf_n(u) -> np.ndarray:
    a = np.ascontiguousarray(u, dtype=np.float32)
    out = np.empty_like(a)
    lib().orc_logf_n(a.size, _ptr(a), _ptr(out))
    return out


def u01_n(x) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.empty(a.shape, dtype=np.float32)
    lib().orc_u01_n(a.size, _ptr(a), _ptr(out))
    return out


def draw_words(seed, it, ant, step, slot) -> np.ndarray:
    arrs = np.broadcast_arrays(*(np.asarray(v, dtype=np.uint32) for v in (it, ant, step, slot)))
    it_, ant_, step_, slot_ = (np.ascontiguousarray(a) for a in arrs)
    out = np.empty(it_.shape, dtype=np.uint32)
    lib().orc_draw_words_n(it_.size, seed, _ptr(it_), _ptr(ant_), _ptr(step_), _ptr(slot_), _ptr(out))
    return out


def start_node(seed, it, ant, n) -> int:
    return int(lib().orc_start_node(seed, it, ant, n))


# ---- stand-alone pieces ----
def limits(rho: float, C_len: int, n: int, pdec: float):
    lo = C.c_float()
    hi = C.c_float()
    lib().orc_limits(float(np.float32(rho)), int(C_len), n, pdec, C.byref(lo), C.byref(hi))
    return np.float32(lo.value), np.float32(hi.value)


def nearest(dist: np.ndarray, k: int) -> np.ndarray:
    d = np.ascontiguousarray(dist, dtype=np.int32)
    n = d.shape[0]
    out = np.zeros((n, k), dtype=np.uint16)
    lib().orc_nearest(n, _ptr(d), k, _ptr(out))
    return out


def nn_tour(dist: np.ndarray):
    d = np.ascontiguousarray(dist, dtype=np.int32)
    n = d.shape[0]
    t = np.zeros(n, dtype=np.uint16)
    length = lib().orc_nn_tour(n, _ptr(d), _ptr(t))
    return t, int(length)


def two_opt_tour(dist: np.ndarray, nn: np.ndarray, tour: np.ndarray):
    d = np.ascontiguousarray(dist, dtype=np.int32)
    nnl = np.ascontiguousarray(nn, dtype=np.uint16)
    t = np.array(tour, dtype=np.uint16, copy=True)
    length = lib().orc_two_opt_tour(d.shape[0], _ptr(d), _ptr(nnl), nnl.shape[1], _ptr(t))
    return t, int(length)


def tour_length(dist: np.ndarray, tour: np.ndarray) -> int:
    d = np.ascontiguousarray(dist, dtype=np.int32)
    t = np.ascontiguousarray(tour, dtype=np.uint16)
    return int(lib().orc_tour_length(d.shape[0], _ptr(d), _ptr(t)))


class Colony:
    """One oracle colony (Alg. 1 state for one instance)."""

    def __init__(self, dist, ants, cand_len=32, alpha=1, beta=2, rho=0.02, p_best=0.01,
                 seed=1, pher_mode=PHER_DENSE, ls_nn=0, deposit=0, select="wrs", problem="tsp"):
        self.dist = np.ascontiguousarray(dist, dtype=np.int32)
        self.n = int(self.dist.shape[0])
        self.ants = int(ants)
        self.pher_mode = pher_mode
        self.pdec = pdec_of(p_best, self.n)
        self._h = lib().orc_create(self.n, _ptr(self.dist), self.ants, cand_len, alpha, beta,
                                   float(np.float32(rho)), self.pdec, seed, pher_mode, ls_nn)
        if not self._h:
            raise ValueError("orc_create rejected the arguments")
        err = None
        if lib().orc_set_deposit(self._h, {"iteration": 0, "global": 1}.get(deposit, deposit)) != 0:
            err = "unknown deposit mode"
        elif lib().orc_set_select(self._h, {"wrs": 0, "prwm": 1}.get(select, select)) != 0:
            err = "unknown selection"
        elif lib().orc_set_problem(self._h, {"tsp": 0, "atsp": 1}.get(problem, problem)) != 0:
            err = "unknown problem, or 2-opt on an asymmetric instance"
        if err:
            self.close()
            raise ValueError(err)
        self.cl = int(lib().orc_cl(self._h))

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # per-iteration calls
    def prepare_choice(self):
        lib().orc_prepare_choice(self._h)

    def construct(self, it, nthreads=1):
        lib().orc_construct(self._h, it, nthreads)

    def two_opt(self, nthreads=1):
        lib().orc_two_opt(self._h, nthreads)

    def update(self):
        lib().orc_update(self._h)

    def iterate(self, it, nthreads=1):
        lib().orc_iterate(self._h, it, nthreads)

    def select_next(self, cur, visited, it, ant, step):
        vis = np.ascontiguousarray(visited, dtype=np.uint8)
        fb = C.c_int()
        v = lib().orc_select_next(self._h, cur, _ptr(vis), it, ant, step, C.byref(fb))
        return int(v), bool(fb.value)

    # state
    def _ntau(self):
        return self.n * self.n if self.pher_mode == PHER_DENSE else self.n * self.cl

    def tours(self):
        out = np.zeros((self.ants, self.n), dtype=np.uint16)
        lib().orc_get_tours(self._h, _ptr(out))
        return out

    def lengths(self):
        out = np.zeros(self.ants, dtype=np.int64)
        lib().orc_get_lengths(self._h, _ptr(out))
        return out

    def pheromone(self):
        out = np.zeros(self._ntau(), dtype=np.float32)
        lib().orc_get_pheromone(self._h, _ptr(out))
        return out.reshape(self.n, -1)

    def set_pheromone(self, tau):
        t = np.ascontiguousarray(tau, dtype=np.float32).reshape(-1)
        assert t.size == self._ntau()
        lib().orc_set_pheromone(self._h, _ptr(t))

    def choice(self):
        out = np.zeros(self.n * self.n, dtype=np.float32)
        lib().orc_get_choice(self._h, _ptr(out))
        return out.reshape(self.n, self.n)

    def chc(self):
        out = np.zeros(self.n * self.cl, dtype=np.float32)
        lib().orc_get_chc(self._h, _ptr(out))
        return out.reshape(self.n, self.cl)

    def cand(self):
        out = np.zeros(self.n * self.cl, dtype=np.uint16)
        lib().orc_get_cand(self._h, _ptr(out))
        return out.reshape(self.n, self.cl)

    def heuristic(self):
        out = np.zeros(self.n * self.n, dtype=np.float32)
        lib().orc_get_heuristic(self._h, _ptr(out))
        return out.reshape(self.n, self.n)

    def set_heuristic(self, heur):
        """Dense mode: use `heur` (n x n eta^beta, e.g. install_eta's) from the
        next choice_info on."""
        h = np.ascontiguousarray(heur, dtype=np.float32)
        assert h.shape == (self.n, self.n)
        if lib().orc_set_heuristic(self._h, _ptr(h)) != 0:
            raise ValueError("set_heuristic needs dense trails")

    def fallback(self):
        s = np.zeros(self.ants, dtype=np.int64)
        v = np.zeros(self.ants, dtype=np.int64)
        lib().orc_get_fallback(self._h, _ptr(s), _ptr(v))
        return s, v

    def limits(self):
        out = np.zeros(2, dtype=np.float32)
        lib().orc_get_limits(self._h, _ptr(out))
        return out[0], out[1]

    def best(self):
        t = np.zeros(self.n, dtype=np.uint16)
        length = lib().orc_get_best(self._h, _ptr(t))
        return (t if length >= 0 else None), int(length)

    def nn_tour(self):
        t = np.zeros(self.n, dtype=np.uint16)
        length = lib().orc_get_nn_tour(self._h, _ptr(t))
        return t, int(length)

    def iteration_best(self):
        out = np.zeros(2, dtype=np.int64)
        lib().orc_get_iteration_best(self._h, _ptr(out))
        return int(out[0]), int(out[1])

    def checkpoint(self):
        """The state carried between iterations: trails, limits, global best."""
        t, L = self.best()
        return {"pheromone": self.pheromone(), "limits": np.array(self.limits(), dtype=np.float32),
                "gb_len": L, "gb_tour": t if t is not None else np.zeros(self.n, np.uint16)}

    def restore(self, ck):
        self.set_pheromone(ck["pheromone"])
        lim = np.ascontiguousarray(ck["limits"], dtype=np.float32)
        tour = np.ascontiguousarray(ck["gb_tour"], dtype=np.uint16)
        lib().orc_restore(self._h, _ptr(lim), int(ck["gb_len"]), _ptr(tour))


# ---- learned heuristic ----
HID = 128
IN = 16


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).reshape(a.shape)


def expf(x: float) -> np.float32:
    return np.float32(lib().orc_expf(float(np.float32(x))))


def knn_features(dist, xy):
    d = np.ascontiguousarray(dist, dtype=np.int32)
    n = d.shape[0]
    xyf = np.ascontiguousarray(xy, dtype=np.float32)
    knn = np.zeros((n, 16), dtype=np.uint16)
    feat = np.zeros((n * 16, 8), dtype=np.float32)
    lib().orc_knn_features(n, _ptr(d), _ptr(xyf), _ptr(knn), _ptr(feat))
    return knn, feat


def pad_inputs(feat) -> np.ndarray:
    X = np.zeros((feat.shape[0], IN), dtype=np.float32)
    X[:, :8] = feat
    return X


class MLPParams:
    """W1 [16,128], b1 [128], W2 [128,128], b2 [128], w3 [128], b3 scalar (float32)."""

    def __init__(self, W1, b1, W2, b2, w3, b3):
        self.W1 = np.ascontiguousarray(W1, np.float32)
        self.b1 = np.ascontiguousarray(b1, np.float32)
        self.W2 = np.ascontiguousarray(W2, np.float32)
        self.b2 = np.ascontiguousarray(b2, np.float32)
        self.w3 = np.ascontiguousarray(w3, np.float32)
        self.b3 = np.float32(np.asarray(b3, dtype=np.float32).reshape(-1)[0])

    def arrays(self):
        return self.W1, self.b1, self.W2, self.b2, self.w3


def mlp_forward(X, P: MLPParams, quantize=True):
    X = np.ascontiguousarray(X, np.float32)
    s = np.zeros(X.shape[0], dtype=np.float32)
    lib().orc_mlp_forward(X.shape[0], _ptr(X), *(_ptr(a) for a in P.arrays()), float(P.b3), int(quantize), _ptr(s))
    return s


def mlp_backward(X, f, P: MLPParams, quantize=True):
    X = np.ascontiguousarray(X, np.float32)
    f = np.ascontiguousarray(f, np.float32)
    g = MLPParams(np.zeros_like(P.W1), np.zeros_like(P.b1), np.zeros_like(P.W2), np.zeros_like(P.b2),
                  np.zeros_like(P.w3), 0.0)
    gb3 = C.c_float()
    loss = lib().orc_mlp_backward(X.shape[0], _ptr(X), _ptr(f), *(_ptr(a) for a in P.arrays()), float(P.b3),
                                  int(quantize), *(_ptr(a) for a in g.arrays()), C.byref(gb3))
    g.b3 = np.float32(gb3.value)
    return float(loss), g


def adam(p, g, m, v, lr, b1, b2, eps, t):
    # bias corrections 1 - beta^t from the FP32 betas, raised in float64
    c1 = np.float32(1.0 - math.pow(float(np.float32(b1)), t))
    c2 = np.float32(1.0 - math.pow(float(np.float32(b2)), t))
    for a in (p, g, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    lib().orc_adam(p.size, _ptr(p), _ptr(g), _ptr(m), _ptr(v), float(np.float32(lr)), float(np.float32(b1)),
                   float(np.float32(b2)), float(np.float32(eps)), float(c1), float(c2))


def install_eta(dist, knn, s, beta):
    d = np.ascontiguousarray(dist, dtype=np.int32)
    n = d.shape[0]
    k = np.ascontiguousarray(knn, dtype=np.uint16)
    sc = np.ascontiguousarray(s, dtype=np.float32)
    heur = np.zeros((n, n), dtype=np.float32)
    lib().orc_install_eta(n, _ptr(d), _ptr(k), _ptr(sc), beta, _ptr(heur))
    return heur
