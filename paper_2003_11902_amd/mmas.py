"""Python binding of libmmas (include/mmas.h): argument marshalling only.

Every step of the method runs in the HIP library. PyTorch provides the device
workspace and the stream; nothing here computes any part of the method. If the
library is not built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MMAS_LIBRARY may point at another build of the same library (e.g. a debug
# build); by default the in-tree build is used.
LIB_PATH = os.environ.get("MMAS_LIBRARY") or os.path.join(HERE, "libmmas.so")

# ---- constants mirrored from include/mmas.h --------------------------------
MMAS_OK = 0
MMAS_EINVAL = -1
MMAS_EUNSUPPORTED = -2
MMAS_ENOSPACE = -3
MMAS_EHIP = -4
MMAS_ESTATE = -5

MMAS_TABU_BITMASK = 0
MMAS_TABU_COMPACT = 1
MMAS_TABU_LIST = 2
MMAS_PHER_DENSE = 0
MMAS_PHER_CANDIDATES = 1

MMAS_BUF_DIST = 0
MMAS_BUF_PHEROMONE = 1
MMAS_BUF_CHOICE = 2
MMAS_BUF_CHC = 3
MMAS_BUF_CAND = 4
MMAS_BUF_HEUR = 5
MMAS_BUF_TOURS = 6
MMAS_BUF_LENGTHS = 7
MMAS_BUF_GB_TOUR = 8
MMAS_BUF_NN_TOUR = 9
MMAS_BUF_FALLBACK = 10
MMAS_BUF_STATE = 11
MMAS_BUF_LSNN = 12

TABU = {"bitmask": MMAS_TABU_BITMASK, "compact": MMAS_TABU_COMPACT, "list": MMAS_TABU_LIST}
DEPOSIT = {"iteration": 0, "global": 1}
SELECT = {"wrs": 0, "prwm": 1}
PROBLEM = {"tsp": 0, "atsp": 1}
PHER = {"dense": MMAS_PHER_DENSE, "candidates": MMAS_PHER_CANDIDATES}

EXPORTED = (
    "mmas_workspace_bytes", "mmas_create", "mmas_prepare_choice_info", "mmas_construct",
    "mmas_two_opt", "mmas_update_pheromone", "mmas_best", "mmas_buffer", "mmas_read",
    "mmas_set_pheromone", "mmas_synchronize", "mmas_destroy", "mmas_status_str",
    "mmas_eval_log", "mmas_eval_draws", "mmas_eval_tabu", "mmas_set_selection", "mmas_set_launch",
    "mmas_batch_workspace_bytes", "mmas_batch_create", "mmas_batch_set_launch", "mmas_batch_tune",
    "mmas_batch_capture", "mmas_batch_step", "mmas_batch_iteration", "mmas_batch_context",
    "mmas_batch_destroy", "mmas_mlp_param_count", "mmas_mlp_packed_count", "mmas_mlp_features",
    "mmas_mlp_pack", "mmas_mlp_forward", "mmas_mlp_grad", "mmas_mlp_adam", "mmas_mlp_labels",
    "mmas_set_learned_heuristic", "mmas_last_error", "mmas_set_two_opt_launch", "mmas_batch_set_tabu",
    "mmas_restore", "mmas_set_timing", "mmas_read_timing", "mmas_batch_set_timing", "mmas_batch_read_timing",
    "mmas_mlp_features_noalloc",
)


class mmas_params(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("ants", C.c_int32), ("cand_len", C.c_int32),
        ("alpha", C.c_int32), ("beta", C.c_int32), ("rho", C.c_float),
        ("p_best", C.c_double), ("seed", C.c_uint64), ("tabu", C.c_int32),
        ("pher_mode", C.c_int32), ("ls_nn", C.c_int32), ("deposit", C.c_int32),
        ("problem", C.c_int32),
    ]


class mmas_device_state(C.Structure):
    _fields_ = [
        ("tau_min", C.c_float), ("tau_max", C.c_float), ("delta", C.c_float),
        ("ib_ant", C.c_int32), ("ib_len", C.c_int64), ("gb_len", C.c_int64),
        ("nn_len", C.c_int64), ("flags", C.c_uint32), ("updates", C.c_uint32),
    ]


class MmasError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        detail = ""
        if status == MMAS_EHIP:
            detail = " [" + lib.mmas_last_error().decode(errors="replace") + "]"
        super().__init__(f"{call}: {status_str(status)} ({status}){detail}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; build it with paper_2003_11902_amd/build.py "
            "(or __graft_entry__.build())")
    # torch first: its HIP runtime (libamdhip64.so.7) is then the one the
    # library binds to. Loaded the other way round, torch brings a second HIP
    # and HSA runtime into the process and one of them sees no device.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    p = C.c_void_p
    L.mmas_workspace_bytes.argtypes = [C.POINTER(mmas_params)]
    L.mmas_workspace_bytes.restype = C.c_size_t
    L.mmas_create.argtypes = [p, C.POINTER(mmas_params), p, C.c_size_t, p, C.POINTER(p)]
    L.mmas_create.restype = C.c_int
    for name in ("mmas_prepare_choice_info", "mmas_two_opt", "mmas_update_pheromone", "mmas_synchronize"):
        getattr(L, name).argtypes = [p]
        getattr(L, name).restype = C.c_int
    L.mmas_set_launch.argtypes = [p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.mmas_set_launch.restype = C.c_int
    L.mmas_set_two_opt_launch.argtypes = [p, C.c_int32]
    L.mmas_set_two_opt_launch.restype = C.c_int
    L.mmas_construct.argtypes = [p, C.c_uint32]
    L.mmas_construct.restype = C.c_int
    L.mmas_best.argtypes = [p, p, C.POINTER(C.c_int64)]
    L.mmas_best.restype = C.c_int
    L.mmas_buffer.argtypes = [p, C.c_int, C.POINTER(p), C.POINTER(C.c_size_t)]
    L.mmas_buffer.restype = C.c_int
    L.mmas_read.argtypes = [p, C.c_int, p, C.c_size_t]
    L.mmas_read.restype = C.c_int
    L.mmas_set_pheromone.argtypes = [p, p]
    L.mmas_set_pheromone.restype = C.c_int
    L.mmas_restore.argtypes = [p, p, p, p]
    L.mmas_restore.restype = C.c_int
    L.mmas_set_timing.argtypes = [p, C.c_int32]
    L.mmas_set_timing.restype = C.c_int
    L.mmas_read_timing.argtypes = [p, p, p, C.c_int32]
    L.mmas_read_timing.restype = C.c_int
    L.mmas_destroy.argtypes = [p]
    L.mmas_destroy.restype = None
    L.mmas_eval_log.argtypes = [p, p, C.c_size_t, p]
    L.mmas_eval_log.restype = C.c_int
    L.mmas_eval_draws.argtypes = [C.c_uint64, p, p, p, p, p, C.c_size_t, p]
    L.mmas_eval_draws.restype = C.c_int
    L.mmas_eval_tabu.argtypes = [C.c_int32, C.c_int32, p, C.c_int32, p, p, p, p]
    L.mmas_eval_tabu.restype = C.c_int
    L.mmas_set_selection.argtypes = [p, C.c_int32]
    L.mmas_set_selection.restype = C.c_int
    L.mmas_batch_workspace_bytes.argtypes = [C.c_int32, p, C.POINTER(C.c_size_t)]
    L.mmas_batch_workspace_bytes.restype = C.c_int
    L.mmas_batch_create.argtypes = [C.c_int32, p, p, p, C.c_size_t, p, C.POINTER(p)]
    L.mmas_batch_create.restype = C.c_int
    L.mmas_batch_set_launch.argtypes = [p, C.c_int32, C.c_int32, C.c_int32]
    L.mmas_batch_set_launch.restype = C.c_int
    L.mmas_batch_tune.argtypes = [p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
    L.mmas_batch_set_tabu.argtypes = [p, C.c_int32]
    L.mmas_batch_set_tabu.restype = C.c_int
    L.mmas_batch_tune.restype = C.c_int
    for name in ("mmas_batch_capture", "mmas_batch_step"):
        getattr(L, name).argtypes = [p]
        getattr(L, name).restype = C.c_int
    L.mmas_batch_iteration.argtypes = [p, C.POINTER(C.c_uint32)]
    L.mmas_batch_iteration.restype = C.c_int
    L.mmas_batch_set_timing.argtypes = [p, C.c_int32]
    L.mmas_batch_set_timing.restype = C.c_int
    L.mmas_batch_read_timing.argtypes = [p, p, p, C.c_int32]
    L.mmas_batch_read_timing.restype = C.c_int
    L.mmas_batch_context.argtypes = [p, C.c_int32, C.POINTER(p)]
    L.mmas_batch_context.restype = C.c_int
    L.mmas_batch_destroy.argtypes = [p]
    L.mmas_batch_destroy.restype = None
    L.mmas_mlp_param_count.argtypes = []
    L.mmas_mlp_param_count.restype = C.c_int32
    L.mmas_mlp_packed_count.argtypes = []
    L.mmas_mlp_packed_count.restype = C.c_int32
    L.mmas_mlp_features.argtypes = [p, p, C.c_int32, p, p, p, p, p]
    L.mmas_mlp_features.restype = C.c_int
    L.mmas_mlp_features_noalloc.argtypes = [p, p, C.c_int32, p, p, p, p]
    L.mmas_mlp_features_noalloc.restype = C.c_int
    L.mmas_mlp_pack.argtypes = [p, p, p]
    L.mmas_mlp_pack.restype = C.c_int
    L.mmas_mlp_forward.argtypes = [p, C.c_int64, p, p, p, p]
    L.mmas_mlp_forward.restype = C.c_int
    L.mmas_mlp_grad.argtypes = [p, p, C.c_int64, p, p, p, C.c_int32, p, p]
    L.mmas_mlp_grad.restype = C.c_int
    L.mmas_mlp_adam.argtypes = [p, p, p, p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, p]
    L.mmas_mlp_adam.restype = C.c_int
    L.mmas_mlp_labels.argtypes = [p, C.c_int32, C.c_int32, p, p, p]
    L.mmas_mlp_labels.restype = C.c_int
    L.mmas_set_learned_heuristic.argtypes = [p, p, p]
    L.mmas_set_learned_heuristic.restype = C.c_int
    L.mmas_last_error.argtypes = []
    L.mmas_last_error.restype = C.c_char_p
    L.mmas_status_str.argtypes = [C.c_int]
    L.mmas_status_str.restype = C.c_char_p
    return L


lib = _load()


def status_str(s: int) -> str:
    return lib.mmas_status_str(s).decode()


def _check(status: int, call: str):
    if status != MMAS_OK:
        raise MmasError(status, call)


def mmas_eval_log(u):
    """Device logarithm of a float32 CUDA tensor (new tensor)."""
    import torch

    out = torch.empty_like(u)
    _check(lib.mmas_eval_log(C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()), u.numel(),
                             C.c_void_p(torch.cuda.current_stream().cuda_stream)), "mmas_eval_log")
    return out


def mmas_eval_tabu(tabu, n, marks):
    """The construction's tabu after marking the cities of the int32 CUDA
    tensor `marks` in order: (visited uint8[n], cells uint16, unvisited count
    or -1), as CPU numpy arrays / int."""
    import torch

    t = TABU.get(tabu, tabu)
    dev = marks.device
    words = (n + 31) // 32
    cells = 2 * words if t == MMAS_TABU_BITMASK else (n if t == MMAS_TABU_COMPACT else 2 * n)
    visited = torch.empty(n, dtype=torch.uint8, device=dev)
    state = torch.empty(cells, dtype=torch.int16, device=dev)
    left = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib.mmas_eval_tabu(t, n, C.c_void_p(marks.data_ptr()) if marks.numel() else None, marks.numel(),
                              C.c_void_p(visited.data_ptr()), C.c_void_p(state.data_ptr()),
                              C.c_void_p(left.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "mmas_eval_tabu")
    torch.cuda.synchronize()
    return visited.cpu().numpy(), state.cpu().numpy().view("uint16"), int(left.cpu()[0])


def mmas_eval_draws(seed, it, ant, step, slot):
    """Device Philox draw words for int32/uint32 CUDA tensors of equal length."""
    import torch

    out = torch.empty_like(it)
    _check(lib.mmas_eval_draws(seed, *(C.c_void_p(t.data_ptr()) for t in (it, ant, step, slot)),
                               C.c_void_p(out.data_ptr()), it.numel(),
                               C.c_void_p(torch.cuda.current_stream().cuda_stream)), "mmas_eval_draws")
    return out


def make_params(n, ants, cand_len=32, alpha=1, beta=2, rho=0.02, p_best=0.01, seed=1,
                tabu="bitmask", pher="dense", ls_nn=0, deposit="iteration", problem="tsp") -> mmas_params:
    return mmas_params(n=n, ants=ants, cand_len=cand_len, alpha=alpha, beta=beta, rho=rho,
                       p_best=p_best, seed=seed, tabu=TABU.get(tabu, tabu),
                       pher_mode=PHER.get(pher, pher), ls_nn=ls_nn,
                       deposit=DEPOSIT.get(deposit, deposit), problem=PROBLEM.get(problem, problem))


def mmas_workspace_bytes(params: mmas_params) -> int:
    return int(lib.mmas_workspace_bytes(C.byref(params)))


_DTYPES = {
    MMAS_BUF_DIST: np.int32, MMAS_BUF_PHEROMONE: np.float32, MMAS_BUF_CHOICE: np.float32,
    MMAS_BUF_CHC: np.float32, MMAS_BUF_CAND: np.uint16, MMAS_BUF_HEUR: np.float32,
    MMAS_BUF_TOURS: np.uint16, MMAS_BUF_LENGTHS: np.int64, MMAS_BUF_GB_TOUR: np.uint16,
    MMAS_BUF_NN_TOUR: np.uint16, MMAS_BUF_FALLBACK: np.int64, MMAS_BUF_LSNN: np.uint16,
}


def _adopt(ws, stream):
    """Hands the workspace (allocated on the caller's current stream) to the
    stream the library enqueues on: that stream first waits for the current
    one, and the caching allocator does not reuse the block until the work
    enqueued on it has finished."""
    import torch

    cur = torch.cuda.current_stream(ws.device)
    if stream.cuda_stream != cur.cuda_stream:
        stream.wait_stream(cur)
        ws.record_stream(stream)


class Colony:
    """One context: a distance matrix, its parameters and a torch-owned workspace."""

    def __init__(self, dist, ants, cand_len=32, alpha=1, beta=2, rho=0.02, p_best=0.01, seed=1,
                 tabu="bitmask", pher="dense", ls_nn=0, device=None, stream=None, deposit="iteration",
                 problem="tsp"):
        import torch

        d = np.ascontiguousarray(dist, dtype=np.int32)
        if d.ndim != 2 or d.shape[0] != d.shape[1]:
            raise ValueError("dist must be a square int32 matrix")
        self.n = int(d.shape[0])
        self.params = make_params(self.n, ants, cand_len, alpha, beta, rho, p_best, seed, tabu, pher, ls_nn,
                                  deposit, problem)
        self.ants = int(ants)
        ws_bytes = mmas_workspace_bytes(self.params)
        if ws_bytes == 0:
            raise MmasError(MMAS_EINVAL, "mmas_workspace_bytes")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _adopt(self.ws, self.stream)
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.mmas_create(d.ctypes.data_as(C.c_void_p), C.byref(self.params),
                                 C.c_void_p(self.ws.data_ptr()), ws_bytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
        _check(st, "mmas_create")
        self.cl = min(self.params.cand_len, self.n - 1)

    # -- lifetime --
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.mmas_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the per-iteration calls (Alg. 1) --
    def prepare_choice_info(self):
        _check(lib.mmas_prepare_choice_info(self._ctx), "mmas_prepare_choice_info")

    def construct(self, iteration: int):
        _check(lib.mmas_construct(self._ctx, iteration), "mmas_construct")

    def set_launch(self, ants_per_block=0, table_rows=-1, lanes_per_ant=64, waves_per_ant=0):
        _check(lib.mmas_set_launch(self._ctx, ants_per_block, table_rows, lanes_per_ant, waves_per_ant),
               "mmas_set_launch")

    def two_opt(self):
        _check(lib.mmas_two_opt(self._ctx), "mmas_two_opt")

    def set_two_opt_launch(self, waves_per_ant=0):
        _check(lib.mmas_set_two_opt_launch(self._ctx, waves_per_ant), "mmas_set_two_opt_launch")

    def set_selection(self, select="wrs"):
        _check(lib.mmas_set_selection(self._ctx, SELECT.get(select, select)), "mmas_set_selection")

    def update_pheromone(self):
        _check(lib.mmas_update_pheromone(self._ctx), "mmas_update_pheromone")

    def iterate(self, iteration: int):
        self.prepare_choice_info()
        self.construct(iteration)
        if self.params.ls_nn > 0:
            self.two_opt()
        self.update_pheromone()

    def synchronize(self):
        _check(lib.mmas_synchronize(self._ctx), "mmas_synchronize")

    # -- results --
    def best(self):
        t = np.zeros(self.n, dtype=np.int32)
        length = C.c_int64()
        _check(lib.mmas_best(self._ctx, t.ctypes.data_as(C.c_void_p), C.byref(length)), "mmas_best")
        return (t if length.value >= 0 else None), int(length.value)

    def buffer(self, which: int):
        """(device pointer, bytes) of a workspace view."""
        ptr = C.c_void_p()
        nbytes = C.c_size_t()
        _check(lib.mmas_buffer(self._ctx, which, C.byref(ptr), C.byref(nbytes)), "mmas_buffer")
        return ptr.value, int(nbytes.value)

    def tensor(self, which: int):
        """A torch view (no copy) of a workspace buffer."""
        import torch

        ptr, nbytes = self.buffer(which)
        if nbytes == 0:
            return None
        off = ptr - self.ws.data_ptr()
        # 16-bit city ids travel as int16 tensors (same bits; torch's uint16
        # supports few operations)
        tdt = {np.int32: torch.int32, np.float32: torch.float32, np.uint16: torch.int16,
               np.int64: torch.int64}[_DTYPES[which]]
        return self.ws[off:off + nbytes].view(tdt)

    def read(self, which: int) -> np.ndarray:
        _, nbytes = self.buffer(which)
        if which == MMAS_BUF_STATE:
            st = mmas_device_state()
            _check(lib.mmas_read(self._ctx, which, C.byref(st), nbytes), "mmas_read")
            return st
        out = np.empty(nbytes // np.dtype(_DTYPES[which]).itemsize, dtype=_DTYPES[which])
        _check(lib.mmas_read(self._ctx, which, out.ctypes.data_as(C.c_void_p), nbytes), "mmas_read")
        return out

    def set_learned_heuristic(self, knn, scores):
        """Install eta = (1/d) 2 sigmoid(s) on the kNN edges (torch tensors on the device)."""
        _check(lib.mmas_set_learned_heuristic(self._ctx, _dptr(knn), _dptr(scores)), "mmas_set_learned_heuristic")

    def set_pheromone(self, tau):
        t = np.ascontiguousarray(tau, dtype=np.float32).reshape(-1)
        _, nbytes = self.buffer(MMAS_BUF_PHEROMONE)
        if t.nbytes != nbytes:
            raise ValueError("pheromone has the wrong size")
        _check(lib.mmas_set_pheromone(self._ctx, t.ctypes.data_as(C.c_void_p)), "mmas_set_pheromone")

    # convenience views
    def tours(self):
        return self.read(MMAS_BUF_TOURS).reshape(self.ants, self.n)

    def lengths(self):
        return self.read(MMAS_BUF_LENGTHS)

    def pheromone(self):
        return self.read(MMAS_BUF_PHEROMONE).reshape(self.n, -1)

    def choice(self):
        return self.read(MMAS_BUF_CHOICE).reshape(self.n, self.n)

    def chc(self):
        return self.read(MMAS_BUF_CHC).reshape(self.n, self.cl)

    def cand(self):
        return self.read(MMAS_BUF_CAND).reshape(self.n, self.cl)

    def fallback(self):
        f = self.read(MMAS_BUF_FALLBACK)
        return f[: self.ants], f[self.ants:]

    def state(self):
        return self.read(MMAS_BUF_STATE)

    def limits(self):
        st = self.state()
        return np.float32(st.tau_min), np.float32(st.tau_max)

    def set_timing(self, on=True):
        _check(lib.mmas_set_timing(self._ctx, 1 if on else 0), "mmas_set_timing")

    def read_timing(self, reset=False):
        """{kind: (milliseconds, launches)} for choice, construct, two_opt, update."""
        ms = np.zeros(4, dtype=np.float64)
        calls = np.zeros(4, dtype=np.int64)
        _check(lib.mmas_read_timing(self._ctx, ms.ctypes.data_as(C.c_void_p), calls.ctypes.data_as(C.c_void_p),
                                    1 if reset else 0), "mmas_read_timing")
        return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(("choice", "construct", "two_opt", "update"))}

    def checkpoint(self):
        """Host copies of what mmas_restore takes: trails, state, global-best tour."""
        return {"pheromone": self.pheromone(), "state": self.state(), "gb_tour": self.read(MMAS_BUF_GB_TOUR)}

    def restore(self, ck):
        t = np.ascontiguousarray(ck["pheromone"], dtype=np.float32).reshape(-1)
        g = np.ascontiguousarray(ck["gb_tour"], dtype=np.uint16)
        _, nbytes = self.buffer(MMAS_BUF_PHEROMONE)
        if t.nbytes != nbytes or g.size != self.n:
            raise ValueError("checkpoint does not match this context")
        st = ck["state"]
        _check(lib.mmas_restore(self._ctx, t.ctypes.data_as(C.c_void_p), C.byref(st),
                                g.ctypes.data_as(C.c_void_p)), "mmas_restore")


class _View(Colony):
    """A context owned by a batch: read-only access through the Colony API."""

    def __init__(self, handle, n, ants, params, ws, stream):
        self._ctx = handle
        self.n = n
        self.ants = ants
        self.params = params
        self.ws = ws
        self.stream = stream
        self.cl = min(params.cand_len, n - 1)

    def close(self):  # owned by the batch
        self._ctx = C.c_void_p()


class Batch:
    """Many instances advancing together (mmas_batch_*)."""

    def __init__(self, dists, params_list, device=None, stream=None):
        import torch

        self.count = len(dists)
        self.dists = [np.ascontiguousarray(d, dtype=np.int32) for d in dists]
        arr = (mmas_params * self.count)(*params_list)
        self._params = arr
        nbytes = C.c_size_t()
        _check(lib.mmas_batch_workspace_bytes(self.count, arr, C.byref(nbytes)), "mmas_batch_workspace_bytes")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): the null stream cannot be captured
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        _adopt(self.ws, self.stream)
        ptrs = (C.c_void_p * self.count)(*[d.ctypes.data_as(C.c_void_p) for d in self.dists])
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.mmas_batch_create(self.count, ptrs, arr, C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
                   "mmas_batch_create")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.mmas_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, ants_per_block=4, table_bytes=-1, lanes_per_ant=64):
        _check(lib.mmas_batch_set_launch(self._h, ants_per_block, table_bytes, lanes_per_ant), "mmas_batch_set_launch")

    def tune(self):
        """(ants_per_block, table_bytes, lanes_per_ant, tabu) chosen by the autotuner."""
        apb = C.c_int32()
        tb = C.c_int32()
        lanes = C.c_int32()
        tabu = C.c_int32()
        _check(lib.mmas_batch_tune(self._h, C.byref(apb), C.byref(tb), C.byref(lanes), C.byref(tabu)),
               "mmas_batch_tune")
        return int(apb.value), int(tb.value), int(lanes.value), int(tabu.value)

    def set_tabu(self, tabu):
        _check(lib.mmas_batch_set_tabu(self._h, TABU.get(tabu, tabu)), "mmas_batch_set_tabu")

    def capture(self):
        _check(lib.mmas_batch_capture(self._h), "mmas_batch_capture")

    def step(self):
        _check(lib.mmas_batch_step(self._h), "mmas_batch_step")

    def iteration(self) -> int:
        it = C.c_uint32()
        _check(lib.mmas_batch_iteration(self._h, C.byref(it)), "mmas_batch_iteration")
        return int(it.value)

    def synchronize(self):
        self.stream.synchronize()

    def set_timing(self, on=True):
        _check(lib.mmas_batch_set_timing(self._h, 1 if on else 0), "mmas_batch_set_timing")

    def read_timing(self, reset=False):
        """(milliseconds, launches) of the timed constructions."""
        ms = C.c_double()
        calls = C.c_int64()
        _check(lib.mmas_batch_read_timing(self._h, C.byref(ms), C.byref(calls), 1 if reset else 0),
               "mmas_batch_read_timing")
        return float(ms.value), int(calls.value)

    def instance(self, i) -> Colony:
        h = C.c_void_p()
        _check(lib.mmas_batch_context(self._h, i, C.byref(h)), "mmas_batch_context")
        p = self._params[i]
        return _View(h, int(p.n), int(p.ants), p, self.ws, self.stream)


# ---- learned heuristic: thin wrappers over mmas_mlp_* (torch device tensors) ----

def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _cur_stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def mlp_param_count() -> int:
    return int(lib.mmas_mlp_param_count())


def mlp_packed_count() -> int:
    return int(lib.mmas_mlp_packed_count())


def mmas_mlp_features(dist, xy, with_features=False):
    """(knn [n,16], X [16n,16] bfloat16 bits, feat float32 [16n,8] or None); 16-bit
    arrays are int16 tensors holding the unsigned bits."""
    import torch

    n = int(dist.shape[0])
    dev = dist.device
    knn = torch.empty((n, 16), dtype=torch.int16, device=dev)
    X = torch.empty((16 * n, 16), dtype=torch.int16, device=dev)
    feat = torch.empty((16 * n, 8), dtype=torch.float32, device=dev) if with_features else None
    scratch = torch.empty(8 * n, dtype=torch.uint8, device=dev)
    _check(lib.mmas_mlp_features(_dptr(dist), _dptr(xy), n, _dptr(scratch), _dptr(knn), _dptr(feat), _dptr(X),
                                 _cur_stream()), "mmas_mlp_features")
    return knn, X, feat


def mmas_mlp_features_noalloc(dist, xy, with_features=False):
    """mmas_mlp_features without a scratch argument: the library's static
    per-device scratch serves the feature pass (calls that overlap on one GPU
    race on it)."""
    import torch

    n = int(dist.shape[0])
    dev = dist.device
    knn = torch.empty((n, 16), dtype=torch.int16, device=dev)
    X = torch.empty((16 * n, 16), dtype=torch.int16, device=dev)
    feat = torch.empty((16 * n, 8), dtype=torch.float32, device=dev) if with_features else None
    _check(lib.mmas_mlp_features_noalloc(_dptr(dist), _dptr(xy), n, _dptr(knn), _dptr(feat), _dptr(X),
                                         _cur_stream()), "mmas_mlp_features_noalloc")
    return knn, X, feat


def mmas_mlp_pack(params):
    import torch

    pk = torch.empty(mlp_packed_count(), dtype=torch.int16, device=params.device)
    _check(lib.mmas_mlp_pack(_dptr(params), _dptr(pk), _cur_stream()), "mmas_mlp_pack")
    return pk


def mmas_mlp_forward(X, params, packed):
    import torch

    E = int(X.shape[0])
    s = torch.empty(E, dtype=torch.float32, device=X.device)
    _check(lib.mmas_mlp_forward(_dptr(X), E, _dptr(params), _dptr(packed), _dptr(s), _cur_stream()),
           "mmas_mlp_forward")
    return s


def mmas_mlp_grad(X, target, params, packed, groups=256, partial=None, grad=None):
    """Gradient (param_count floats) and the loss sum (last element)."""
    import torch

    E = int(X.shape[0])
    P = mlp_param_count()
    if partial is None:
        partial = torch.empty(groups * (P + 1), dtype=torch.float32, device=X.device)
    if grad is None:
        grad = torch.empty(P + 1, dtype=torch.float32, device=X.device)
    _check(lib.mmas_mlp_grad(_dptr(X), _dptr(target), E, _dptr(params), _dptr(packed), _dptr(partial), groups,
                             _dptr(grad), _cur_stream()), "mmas_mlp_grad")
    return grad


def mmas_mlp_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib.mmas_mlp_adam(_dptr(params), _dptr(grad), _dptr(m), _dptr(v), lr, beta1, beta2, eps, step,
                             _cur_stream()), "mmas_mlp_adam")


def mmas_mlp_labels(tours, knn):
    import torch

    R, n = int(tours.shape[0]), int(tours.shape[1])
    out = torch.empty((n, 16), dtype=torch.float32, device=tours.device)
    _check(lib.mmas_mlp_labels(_dptr(tours), R, n, _dptr(knn), _dptr(out), _cur_stream()), "mmas_mlp_labels")
    return out
