"""ctypes binding of libdaic (argument marshalling only).

Every step of a run executes in the library's HIP kernels; this module only
converts arguments. It refuses to work without the compiled library: there is
no CPU fallback.

Names follow the C ABI in include/daic.h: a problem is the DAIC tuple
(g, (+), v0, dv1) of the paper's Table 1 on a CSR graph.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdaic.so")

OK, NOT_CONVERGED = 0, 1
SUM, MIN, MAX = 0, 1, 2
G_SRC_SCALE, G_EDGE_SCALE, G_EDGE_ADD, G_COPY, G_DEG_SCALE = 0, 1, 2, 3, 4
F64, F32, F32_KAHAN, U32, I32, NONE = 0, 1, 2, 3, 4, 5
SCHED_ALL, SCHED_TOPK_EXACT, SCHED_TOPK_SAMPLED, SCHED_LEARNED, SCHED_ROUND_ROBIN, SCHED_SWEEP = 0, 1, 2, 3, 4, 5
INF_U32 = 0xFFFFFFFF

_SCHED_NAMES = {"all": SCHED_ALL, "exact": SCHED_TOPK_EXACT, "sampled": SCHED_TOPK_SAMPLED,
                "learned": SCHED_LEARNED, "round_robin": SCHED_ROUND_ROBIN, "sweep": SCHED_SWEEP}
_STATE_NAMES = {"f64": F64, "f32": F32, "f32_kahan": F32_KAHAN, "u32": U32, "i32": I32}

_vp = ctypes.c_void_p


class DaicError(RuntimeError):
    pass


class RunOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("priority_fraction", ctypes.c_double),
                ("sched", ctypes.c_int), ("max_rounds", ctypes.c_uint64),
                ("rounds_per_check", ctypes.c_uint32), ("n_samples", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("hip_stream", _vp), ("model", _vp)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("activations", ctypes.c_uint64),
                ("pushed_edges", ctypes.c_uint64), ("final_residual", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("gteps", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("learned_exact_rounds", ctypes.c_uint64),
                ("learned_fallbacks", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class TrainStats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_uint64), ("positive_fraction", ctypes.c_double),
                ("loss_first", ctypes.c_double), ("loss_final", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("epochs", ctypes.c_uint32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("edges", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DaicError(f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_1710_05785_amd.build` (no CPU fallback exists)")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 with
        # the same soname, so loading torch first makes libdaic bind to that
        # runtime and share device memory and streams with it.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        L.daic_last_error.restype = ctypes.c_char_p
        L.daic_graph_create.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp, ctypes.c_int,
                                        ctypes.POINTER(_vp)]
        L.daic_graph_create_device.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp,
                                               ctypes.c_int, _vp, ctypes.POINTER(_vp)]
        L.daic_graph_destroy.argtypes = [_vp]
        L.daic_graph_destroy.restype = None
        L.daic_problem_create.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp,
                                          ctypes.c_int, ctypes.POINTER(_vp)]
        L.daic_problem_set_init.argtypes = [_vp, _vp, _vp]
        L.daic_run.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.POINTER(Stats)]
        L.daic_problem_get.argtypes = [_vp, _vp, _vp]
        L.daic_problem_destroy.argtypes = [_vp]
        L.daic_problem_destroy.restype = None
        L.daic_problem_set_init_device.argtypes = [_vp, _vp, _vp, _vp]
        L.daic_profile.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.c_uint32,
                                   ctypes.POINTER(KernelTime), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(Stats)]
        L.daic_batch_create.argtypes = [ctypes.c_uint32, ctypes.POINTER(_vp), _vp, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(_vp)]
        L.daic_batch_set_init.argtypes = [_vp, ctypes.c_uint32, _vp, _vp]
        L.daic_batch_tune.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
        L.daic_batch_run.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.POINTER(Stats), _vp]
        L.daic_batch_get.argtypes = [_vp, ctypes.c_uint32, _vp]
        L.daic_batch_destroy.argtypes = [_vp]
        L.daic_batch_destroy.restype = None
        L.daic_sched_model_create.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]
        L.daic_sched_model_get.argtypes = [_vp, _vp, _vp, _vp]
        L.daic_sched_model_set_features.argtypes = [_vp, _vp, _vp]
        L.daic_sched_destroy.argtypes = [_vp]
        L.daic_sched_destroy.restype = None
        L.daic_mlp_forward.argtypes = [_vp, _vp, ctypes.c_uint64, _vp]
        L.daic_sched_score.argtypes = [_vp, _vp, _vp]
        _u64p = ctypes.POINTER(ctypes.c_uint64)
        L.daic_tile_table.argtypes = [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp, _vp, _u64p, _u64p, _u64p]
        L.daic_mlp_grad.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, _vp,
                                    ctypes.POINTER(ctypes.c_double)]
        L.daic_trace_record.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.POINTER(_vp)]
        L.daic_trace_get.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
        L.daic_trace_destroy.argtypes = [_vp]
        L.daic_trace_destroy.restype = None
        L.daic_trace_samples.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
        L.daic_trace_create.argtypes = [_vp, _vp, ctypes.c_uint64, ctypes.POINTER(_vp)]
        L.daic_sched_step.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, ctypes.c_float, _vp,
                                      ctypes.POINTER(ctypes.c_double)]
        L.daic_sched_save.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]
        L.daic_sched_load.argtypes = [_vp, ctypes.c_size_t, ctypes.POINTER(_vp)]
        L.daic_sched_train.argtypes = [ctypes.POINTER(_vp), ctypes.c_uint32,
                                       ctypes.POINTER(TrainOpts), _vp, ctypes.POINTER(TrainStats)]
        L.daic_run_progress.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.c_uint64, _vp, _vp,
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(Stats)]
        L.daic_select_frontier.argtypes = [_vp, ctypes.POINTER(RunOpts), ctypes.c_uint64, _vp,
                                           ctypes.POINTER(ctypes.c_double)]
        L.daic_problem_set_const.argtypes = [_vp, _vp]
        L.daic_problem_check_init.argtypes = [_vp, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
        L.daic_problem_save.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]
        L.daic_problem_load.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.daic_batch_get_state.argtypes = [_vp, ctypes.c_uint32, _vp, _vp, _vp]
        L.daic_batch_save.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]
        L.daic_batch_load.argtypes = [_vp, _vp, ctypes.c_size_t]
        _lib = L
    return _lib


def _save(fn, h, what) -> bytes:
    n = ctypes.c_size_t(0)
    check(fn(h, None, ctypes.byref(n)), what)
    buf = ctypes.create_string_buffer(n.value)
    check(fn(h, buf, ctypes.byref(n)), what)
    return buf.raw[:n.value]


def _load(fn, h, data: bytes, what):
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    check(fn(h, buf, len(data)), what)


def check(rc: int, what: str) -> int:
    if rc < 0:
        msg = lib().daic_last_error().decode(errors="replace")
        raise DaicError(f"{what} failed ({rc}): {msg}")
    return rc


def _addr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Graph:
    """A CSR graph on the device (daic_graph)."""

    def __init__(self, row_ptr, col, w=None, *, _handle=None, _keep=()):
        self._h = None
        self._keep = _keep
        if _handle is not None:
            self._h = _handle
            return
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        col = np.ascontiguousarray(col, dtype=np.uint32)
        n = row_ptr.shape[0] - 1
        m = col.shape[0]
        wt = NONE
        if w is not None:
            w = np.ascontiguousarray(w)
            wt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32,
                  np.dtype(np.uint32): U32}[w.dtype]
        h = _vp()
        check(lib().daic_graph_create(n, m, _addr(row_ptr), _addr(col), _addr(w), wt,
                                      ctypes.byref(h)), "daic_graph_create")
        self._h = h
        self.n, self.m = n, m

    @classmethod
    def from_device(cls, row_ptr, col, w=None, stream=None):
        """Borrow torch device tensors (uint64/int64 row_ptr, int32 col)."""
        n = row_ptr.shape[0] - 1
        m = col.shape[0]
        wt = NONE
        if w is not None:
            import torch

            wt = {torch.float64: F64, torch.float32: F32, torch.int32: U32}[w.dtype]
        h = _vp()
        check(lib().daic_graph_create_device(n, m, _addr(row_ptr), _addr(col), _addr(w), wt,
                                             _stream_handle(stream), ctypes.byref(h)),
              "daic_graph_create_device")
        g = cls(None, None, _handle=h, _keep=(row_ptr, col, w))
        g.n, g.m = n, m
        return g

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None:
            lib().daic_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class RunResult:
    status: int
    stats: dict

    @property
    def converged(self):
        return self.status == OK


class Problem:
    """A DAIC problem (daic_problem) on a Graph."""

    def __init__(self, graph: Graph, op: int, g: int, alpha: float = 0.0, alpha_pv=None,
                 state="f64"):
        self.graph = graph
        self.op = op
        self.state = _STATE_NAMES[state] if isinstance(state, str) else state
        self.n = graph.n
        apv = None if alpha_pv is None else np.ascontiguousarray(alpha_pv, dtype=np.float64)
        h = _vp()
        check(lib().daic_problem_create(graph.handle, op, g, float(alpha), _addr(apv), self.state,
                                        ctypes.byref(h)), "daic_problem_create")
        self._h = h

    def _host_dtype(self):
        return {F64: np.float64, F32: np.float64, F32_KAHAN: np.float64, U32: np.uint32,
                I32: np.int32}[self.state]

    def set_init(self, v0, dv1):
        dt = self._host_dtype()
        v0 = np.ascontiguousarray(v0, dtype=dt)
        dv1 = np.ascontiguousarray(dv1, dtype=dt)
        if v0.shape != (self.n,) or dv1.shape != (self.n,):
            raise ValueError("v0 and dv1 must have n entries")
        check(lib().daic_problem_set_init(self._h, _addr(v0), _addr(dv1)), "daic_problem_set_init")

    def sched_score(self, model):
        """Selection multiplier of every vertex under the learned rule at
        round 0 (test hook of the scoring kernel)."""
        out = np.empty(self.n, dtype=np.float32)
        check(lib().daic_sched_score(self._h, model.handle, _addr(out)), "daic_sched_score")
        return out

    def set_init_device(self, v0, dv1, stream=None):
        """(v0, dv1) from device tensors in the state's element type."""
        if v0.numel() != self.n or dv1.numel() != self.n:
            raise ValueError("v0 and dv1 must have n entries")
        check(lib().daic_problem_set_init_device(self._h, _addr(v0), _addr(dv1),
                                                 _stream_handle(stream)),
              "daic_problem_set_init_device")

    def profile(self, **kw):
        """Run with per-kernel event timing; returns (RunResult, [kernel dicts])."""
        o = self.make_opts(**kw)
        st = Stats()
        arr = (KernelTime * 32)()
        cnt = ctypes.c_uint32(0)
        rc = check(lib().daic_profile(self._h, ctypes.byref(o), 32, arr, ctypes.byref(cnt),
                                      ctypes.byref(st)), "daic_profile")
        ks = [{"name": arr[i].name.decode(), "launches": arr[i].launches,
               "total_ms": arr[i].total_ms, "alg_bytes": arr[i].alg_bytes,
               "edges": arr[i].edges} for i in range(cnt.value)]
        return RunResult(rc, st.as_dict()), ks

    @staticmethod
    def make_opts(eps=0.0, q=1.0, sched="all", max_rounds=0, rounds_per_check=8, n_samples=4096,
                  seed=0, stream=None, model=None):
        o = RunOpts()
        o.eps = eps
        o.priority_fraction = q
        o.sched = _SCHED_NAMES[sched] if isinstance(sched, str) else sched
        o.max_rounds = max_rounds
        o.rounds_per_check = rounds_per_check
        o.n_samples = n_samples
        o.seed = seed
        o.hip_stream = _stream_handle(stream)
        o.model = None if model is None else model.handle
        return o

    def run(self, **kw) -> RunResult:
        o = self.make_opts(**kw)
        st = Stats()
        rc = check(lib().daic_run(self._h, ctypes.byref(o), ctypes.byref(st)), "daic_run")
        return RunResult(rc, st.as_dict())

    def get(self, with_dv=False):
        dt = self._host_dtype()
        v = np.empty(self.n, dtype=dt)
        dv = np.empty(self.n, dtype=dt) if with_dv else None
        check(lib().daic_problem_get(self._h, _addr(v), _addr(dv)), "daic_problem_get")
        return (v, dv) if with_dv else v

    def run_progress(self, max_points=100000, **kw):
        """Run one round at a time; returns (RunResult, updates[], progress[])."""
        o = self.make_opts(**kw)
        st = Stats()
        up = np.zeros(max_points, dtype=np.uint64)
        pr = np.zeros(max_points, dtype=np.float64)
        pts = ctypes.c_uint64(0)
        rc = check(lib().daic_run_progress(self._h, ctypes.byref(o), max_points, _addr(up), _addr(pr),
                                           ctypes.byref(pts), ctypes.byref(st)), "daic_run_progress")
        k = pts.value
        return RunResult(rc, st.as_dict()), up[:k], pr[:k]

    def set_const(self, c):
        """The constant c of the update function (Eq. decompose), for the
        fourth-condition check."""
        dt = np.float64 if self.state in (F64, F32, F32_KAHAN) else self._host_dtype()
        c = np.ascontiguousarray(c, dtype=dt)
        if c.shape != (self.n,):
            raise ValueError("c must have n entries")
        check(lib().daic_problem_set_const(self._h, _addr(c)), "daic_problem_set_const")

    def check_init(self, tol=0.0):
        """Checks v (+) dv = f(v) on the device; returns the mismatch count
        (0), raising DaicError when some vertex fails."""
        bad = ctypes.c_uint64(0)
        rc = lib().daic_problem_check_init(self._h, float(tol), ctypes.byref(bad))
        if rc < 0:
            msg = lib().daic_last_error().decode(errors="replace")
            raise DaicError(f"daic_problem_check_init failed ({rc}, {bad.value} mismatches): {msg}")
        return bad.value

    def save_state(self) -> bytes:
        """The state snapshot of daic_problem_save."""
        return _save(lib().daic_problem_save, self._h, "daic_problem_save")

    def load_state(self, data: bytes):
        _load(lib().daic_problem_load, self._h, data, "daic_problem_load")

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.save_state())

    def load(self, path):
        with open(path, "rb") as f:
            self.load_state(f.read())

    def select_frontier(self, round_no=0, **kw):
        o = self.make_opts(**kw)
        sel = np.zeros(self.n, dtype=np.uint8)
        tau = ctypes.c_double(0)
        check(lib().daic_select_frontier(self._h, ctypes.byref(o), round_no, _addr(sel),
                                         ctypes.byref(tau)), "daic_select_frontier")
        return sel.astype(bool), tau.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().daic_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many graphs x many right-hand sides solved together (daic_batch):
    personalized PageRank (g=G_DEG_SCALE) or weighted sums such as
    multi-label Adsorption (g=G_EDGE_SCALE, graphs with weights). rhs: one
    count (<= 64) or one per graph."""

    def __init__(self, graphs, rhs, alpha: float, state="f32", g=None):
        self.graphs = list(graphs)
        G = len(self.graphs)
        self.rhs = [int(rhs)] * G if np.isscalar(rhs) else [int(r) for r in rhs]
        self.n = [g.n for g in self.graphs]
        handles = (_vp * G)(*[g.handle for g in self.graphs])
        r = np.ascontiguousarray(self.rhs, dtype=np.uint32)
        st = _STATE_NAMES[state] if isinstance(state, str) else state
        h = _vp()
        gk = G_DEG_SCALE if g is None else g
        check(lib().daic_batch_create(G, handles, _addr(r), SUM, gk, float(alpha), st,
                                      ctypes.byref(h)), "daic_batch_create")
        self._h = h

    def set_init(self, g: int, v0, dv1):
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        dv1 = np.ascontiguousarray(dv1, dtype=np.float64)
        shape = (self.n[g], self.rhs[g])
        if v0.shape != shape or dv1.shape != shape:
            raise ValueError(f"expected arrays of shape {shape}")
        check(lib().daic_batch_set_init(self._h, g, _addr(v0), _addr(dv1)), "daic_batch_set_init")

    def tune(self) -> str:
        buf = ctypes.create_string_buffer(256)
        check(lib().daic_batch_tune(self._h, buf, 256), "daic_batch_tune")
        return buf.value.decode()

    def run(self, eps=1e-6, rounds_per_check=8, max_rounds=0, stream=None, sched="all", q=1.0):
        """sched "all" (synchronous dense rounds) or "sweep" (blocks of
        ceil(q n_g) vertices of every graph in turn, asynchronous order)."""
        o = Problem.make_opts(eps=eps, q=q, sched=sched, rounds_per_check=rounds_per_check,
                              max_rounds=max_rounds, stream=stream)
        st = Stats()
        inst = np.zeros(sum(self.rhs), dtype=np.float64)
        rc = check(lib().daic_batch_run(self._h, ctypes.byref(o), ctypes.byref(st), _addr(inst)),
                   "daic_batch_run")
        return RunResult(rc, st.as_dict()), inst

    def get(self, g: int):
        out = np.empty((self.n[g], self.rhs[g]), dtype=np.float64)
        check(lib().daic_batch_get(self._h, g, _addr(out)), "daic_batch_get")
        return out

    def get_state(self, g: int):
        """(v, dv, finish states) of graph g's instances."""
        v = np.empty((self.n[g], self.rhs[g]), dtype=np.float64)
        dv = np.empty((self.n[g], self.rhs[g]), dtype=np.float64)
        done = np.empty(self.rhs[g], dtype=np.uint8)
        check(lib().daic_batch_get_state(self._h, g, _addr(v), _addr(dv), _addr(done)),
              "daic_batch_get_state")
        return v, dv, done

    def save_state(self) -> bytes:
        return _save(lib().daic_batch_save, self._h, "daic_batch_save")

    def load_state(self, data: bytes):
        _load(lib().daic_batch_load, self._h, data, "daic_batch_load")

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.save_state())

    def load(self, path):
        with open(path, "rb") as f:
            self.load_state(f.read())

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().daic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


N_PARAMS = 4481
_PARAM_SHAPES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)),
                 ("b3", (1,))]


def pack_params(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float32).reshape(-1) for k, _ in _PARAM_SHAPES])


def unpack_params(flat) -> dict:
    out, o = {}, 0
    for k, shp in _PARAM_SHAPES:
        c = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + c]).reshape(shp)
        o += c
    return out


class SchedModel:
    """The learned scheduler's network (daic_sched_model)."""

    def __init__(self, params=None, seed=0, *, _handle=None):
        if _handle is not None:
            self._h = _handle
            return
        flat = None if params is None else np.ascontiguousarray(
            pack_params(params) if isinstance(params, dict) else params, dtype=np.float32)
        h = _vp()
        check(lib().daic_sched_model_create(_addr(flat), seed, ctypes.byref(h)),
              "daic_sched_model_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self):
        flat = np.empty(N_PARAMS, dtype=np.float32)
        mean = np.empty(3, dtype=np.float32)
        std = np.empty(3, dtype=np.float32)
        check(lib().daic_sched_model_get(self._h, _addr(flat), _addr(mean), _addr(std)),
              "daic_sched_model_get")
        return unpack_params(flat), mean, std

    def set_features(self, mean, std):
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        check(lib().daic_sched_model_set_features(self._h, _addr(mean), _addr(std)),
              "daic_sched_model_set_features")

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty(x.shape[0], dtype=np.float32)
        check(lib().daic_mlp_forward(self._h, _addr(x), x.shape[0], _addr(out)), "daic_mlp_forward")
        return out

    def grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = ctypes.c_double(0)
        check(lib().daic_mlp_grad(self._h, _addr(x), _addr(y), x.shape[0], _addr(g),
                                  ctypes.byref(loss)), "daic_mlp_grad")
        return unpack_params(g), loss.value

    def step(self, x, y, lr):
        """One Adam step on standardized samples; returns (gradient dict, loss)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = ctypes.c_double(0)
        check(lib().daic_sched_step(self._h, _addr(x), _addr(y), x.shape[0], float(lr), _addr(g),
                                    ctypes.byref(loss)), "daic_sched_step")
        return unpack_params(g), loss.value

    def save(self) -> bytes:
        n = ctypes.c_size_t(0)
        check(lib().daic_sched_save(self._h, None, ctypes.byref(n)), "daic_sched_save")
        buf = ctypes.create_string_buffer(n.value)
        check(lib().daic_sched_save(self._h, buf, ctypes.byref(n)), "daic_sched_save")
        return buf.raw[:n.value]

    @classmethod
    def load(cls, data: bytes) -> "SchedModel":
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        h = _vp()
        check(lib().daic_sched_load(buf, len(data), ctypes.byref(h)), "daic_sched_load")
        return cls(_handle=h)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().daic_sched_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trace:
    """Training samples captured from an exact top-k run (daic_trace)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def record(cls, problem: "Problem", samples_per_round=4096, horizon=4, **run_kw):
        run_kw.setdefault("sched", "exact")
        o = Problem.make_opts(**run_kw)
        h = _vp()
        check(lib().daic_trace_record(problem._h, ctypes.byref(o), samples_per_round, horizon,
                                      ctypes.byref(h)), "daic_trace_record")
        return cls(h)

    @classmethod
    def from_samples(cls, x, y):
        """A trace of caller samples (x [n, 3] raw features, y [n] in {0, 1})."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        h = _vp()
        check(lib().daic_trace_create(_addr(x), _addr(y), y.shape[0], ctypes.byref(h)),
              "daic_trace_create")
        return cls(h)

    @property
    def handle(self):
        return self._h

    def samples(self):
        """(vertex, round) of every sample of a recorded trace."""
        n = ctypes.c_uint64(0)
        check(lib().daic_trace_samples(self._h, None, None, ctypes.byref(n)), "daic_trace_samples")
        vid = np.empty(n.value, dtype=np.uint32)
        rnd = np.empty(n.value, dtype=np.uint32)
        check(lib().daic_trace_samples(self._h, _addr(vid), _addr(rnd), ctypes.byref(n)),
              "daic_trace_samples")
        return vid, rnd

    def get(self):
        n = ctypes.c_uint64(0)
        check(lib().daic_trace_get(self._h, None, None, ctypes.byref(n)), "daic_trace_get")
        x = np.empty((n.value, 3), dtype=np.float32)
        y = np.empty(n.value, dtype=np.float32)
        check(lib().daic_trace_get(self._h, _addr(x), _addr(y), ctypes.byref(n)), "daic_trace_get")
        return x, y

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().daic_trace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sched_train(traces, model: SchedModel, epochs=10, batch=65536, lr=1e-3, seed=0) -> dict:
    """Train the scheduler network on the device from captured traces."""
    arr = (_vp * len(traces))(*[t.handle for t in traces])
    o = TrainOpts(epochs, batch, lr, seed)
    st = TrainStats()
    check(lib().daic_sched_train(arr, len(traces), ctypes.byref(o), model.handle, ctypes.byref(st)),
          "daic_sched_train")
    return {k: getattr(st, k) for k, _ in TrainStats._fields_}


def tile_table(pstart, lb, max_edges=0, group_parts=0, share_div=0) -> dict:
    """Host-only tile table of a partitioned in-edge order (daic_tile_table)."""
    ps = np.ascontiguousarray(pstart, dtype=np.uint32)
    n_part = ps.size - 1
    cnt = [ctypes.c_uint64(0) for _ in range(3)]
    args = (_addr(ps), n_part, lb, max_edges, group_parts, share_div)
    rc = lib().daic_tile_table(*args, 0, None, None, None, None, *[ctypes.byref(c) for c in cnt])
    if rc != 0 and cnt[0].value == 0:
        check(rc, "daic_tile_table")
    nt = cnt[0].value
    tp, te, ts, order = (np.zeros(nt + 1, dtype=np.uint32) for _ in range(4))
    check(lib().daic_tile_table(*args, nt + 1, _addr(tp), _addr(te), _addr(ts), _addr(order),
                                *[ctypes.byref(c) for c in cnt]), "daic_tile_table")
    return {"tile_part": tp[:nt], "tile_e": te, "tile_slot": ts[:nt], "order": order[:nt],
            "n_split": cnt[1].value, "n_slots": cnt[2].value}


def select_frontier_noalloc(op, state, v, dv, sel_out, tau_out=None, round_no=0, **kw):
    """daic_select_frontier_noalloc on torch device tensors: the selection of
    one round from (v, dv) written into sel_out (uint8, n) and tau_out
    (float64, 1, optional); enqueued on kw["stream"] (default stream)."""
    o = Problem.make_opts(**kw)
    st = _STATE_NAMES[state] if isinstance(state, str) else state
    L = lib()
    if not hasattr(L.daic_select_frontier_noalloc, "_typed"):
        L.daic_select_frontier_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _vp, _vp,
                                                   ctypes.POINTER(RunOpts), ctypes.c_uint64, _vp, _vp]
        L.daic_select_frontier_noalloc._typed = True
    n = v.numel()
    if dv.numel() != n or sel_out.numel() != n:
        raise ValueError("v, dv and sel_out must have n entries")
    check(L.daic_select_frontier_noalloc(op, st, n, _addr(v), _addr(dv), ctypes.byref(o), round_no,
                                         _addr(sel_out), _addr(tau_out)),
          "daic_select_frontier_noalloc")
