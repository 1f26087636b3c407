"""Python binding of libqqa (include/qqa.h): argument marshalling only.

Every stage of the solver runs in the HIP library; this module converts Python values
and torch device tensors into the C ABI's plain pointers and sizes.  torch provides
device memory and streams.  The library must be built (``__graft_entry__.build()``):
importing the binding without it raises, there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loaded first so that libqqa binds to the HIP runtime torch already uses

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqqa.so")

QQA_OK, QQA_PENDING = 0, 1
QQA_E_ARG, QQA_E_GRAPH, QQA_E_NOMEM, QQA_E_ADMISSION = -1, -2, -3, -4
QQA_E_DEVICE, QQA_E_UNKNOWN_REQ, QQA_E_CANCELLED = -5, -6, -7
QQA_MIS, QQA_MAXCUT, QQA_MAXCLIQUE, QQA_COLORING = 0, 1, 2, 3
QQA_STEP_ADAMW, QQA_STEP_LANGEVIN = 0, 1
QQA_ENGINE_AUTO, QQA_ENGINE_STREAM, QQA_ENGINE_PERSISTENT, QQA_ENGINE_LDS_BLOCK, QQA_ENGINE_BATCH = -1, 0, 1, 2, 3
QQA_ENGINE_SLICED, QQA_ENGINE_COMPACT, QQA_ENGINE_BATCH_RESIDENT = 4, 5, 6
ENGINES = {"auto": -1, "stream": 0, "persistent": 1, "lds_block": 2, "batch": 3, "sliced": 4, "compact": 5,
           "batch_resident": 6}

PROBLEMS = {"mis": QQA_MIS, "maxcut": QQA_MAXCUT, "maxclique": QQA_MAXCLIQUE, "coloring": QQA_COLORING,
            QQA_MIS: QQA_MIS, QQA_MAXCUT: QQA_MAXCUT, QQA_MAXCLIQUE: QQA_MAXCLIQUE, QQA_COLORING: QQA_COLORING}


class QQAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qqa error {code}: {msg}")
        self.code = code


class qqa_schedule(C.Structure):
    _fields_ = [("gamma_min", C.c_float), ("gamma_max", C.c_float), ("lr", C.c_float),
                ("weight_decay", C.c_float), ("temperature", C.c_float), ("comm_alpha", C.c_float),
                ("entropy_alpha", C.c_int32), ("beta1", C.c_float), ("beta2", C.c_float),
                ("adam_eps", C.c_float), ("penalty_lambda", C.c_int32), ("rule", C.c_int32)]


class qqa_graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("weight", C.c_void_p), ("dense", C.c_void_p)]


class qqa_result(C.Structure):
    _fields_ = [("best_replica", C.c_int32), ("feasible", C.c_int32), ("best_objective", C.c_int64),
                ("best_size_or_cut", C.c_int64), ("best_violations", C.c_int64),
                ("replica_objective", C.c_void_p), ("replica_size_or_cut", C.c_void_p),
                ("replica_violations", C.c_void_p), ("best_x", C.c_void_p), ("queue_ms", C.c_double),
                ("device_ms", C.c_double), ("step_loop_ms", C.c_double), ("latency_ms", C.c_double),
                ("engine", C.c_int32), ("kernel_us", C.c_double), ("first_update_ms", C.c_double)]


class qqa_serve_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("shed", C.c_int64), ("completed", C.c_int64),
                ("rate_updates_per_s", C.c_double), ("deadline_ms", C.c_double),
                ("device_bytes_held", C.c_size_t), ("device_bytes_cached", C.c_size_t)]


class qqa_dev_graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("weight", C.c_void_p), ("dense", C.c_void_p)]


_lib = None


def lib():
    """The loaded libqqa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64, i64, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_size_t
        sig = {
            "qqa_schedule_default": (None, [vp, i32, i32]),
            "qqa_replica_stride": (i32, [i32]),
            "qqa_create": (C.c_int, [vp, C.c_int, sz, vp]),
            "qqa_destroy": (None, [vp]),
            "qqa_last_error": (C.c_char_p, [vp]),
            "qqa_graph_validate": (C.c_int, [vp, i32, vp, sz]),
            "qqa_graph_upload": (C.c_int, [vp, vp, i32, vp]),
            "qqa_graph_release": (C.c_int, [vp, i64]),
            "qqa_solve": (C.c_int, [vp, vp, i32, vp, i32, i32, u64, vp]),
            "qqa_solve_resident": (C.c_int, [vp, i64, i32, vp, i32, i32, u64, vp]),
            "qqa_solve_batch": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp]),
            "qqa_poll": (C.c_int, [vp, i64, vp, i32]),
            "qqa_cancel": (C.c_int, [vp, i64]),
            "qqa_serve_start": (C.c_int, [vp, i32]),
            "qqa_serve_submit": (C.c_int, [vp, vp, i32, vp, i32, i32, u64, vp]),
            "qqa_serve_stop": (C.c_int, [vp]),
            "qqa_serve_set_deadline": (C.c_int, [vp, C.c_double]),
            "qqa_serve_get_stats": (C.c_int, [vp, vp]),
            "qqa_dev_last_error": (C.c_char_p, []),
            "qqa_dev_philox": (C.c_int, [u64, i32, i32, u32, u32, vp, vp]),
            "qqa_dev_noise": (C.c_int, [u64, i32, i32, u32, vp, vp]),
            "qqa_dev_init": (C.c_int, [u64, i32, i32, vp, vp, vp, vp]),
            "qqa_dev_step": (C.c_int, [vp, i32, vp, i32, i32, i32, u64, vp, vp, vp, vp, i32, vp]),
            "qqa_set_replica_layout": (C.c_int, [vp, i32, i32]),
            "qqa_set_engine": (C.c_int, [vp, i32]),
            "qqa_dev_run": (C.c_int, [vp, i32, vp, i32, i32, i32, i32, u64, vp, vp, vp, vp, i32, i32, vp]),
            "qqa_autotune": (C.c_int, [vp, i64, i32, i32, vp]),
            "qqa_autotune_batch": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp]),
            "qqa_dev_eval": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
            "qqa_dev_eval_noalloc": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
            "qqa_dev_dense_coupling": (C.c_int, [vp, vp, vp, i32, i32, i32, vp]),
            "qqa_dev_replica_sums": (C.c_int, [vp, i32, i32, vp, vp]),
            "qqa_solve_coloring": (C.c_int, [vp, vp, i32, vp, i32, i32, u64, vp]),
            "qqa_solve_coloring_resident": (C.c_int, [vp, i64, i32, vp, i32, i32, u64, vp]),
            "qqa_dev_color_step": (C.c_int, [vp, i32, vp, i32, i32, i32, u64, vp, vp, vp, vp, i32, vp]),
            "qqa_dev_color_eval": (C.c_int, [vp, i32, i32, vp, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t)


_DTYPES = {"f32": (torch.float32,), "i64": (torch.int64, torch.uint64), "u64": (torch.int64, torch.uint64),
           "i32": (torch.int32,), "u32": (torch.int32, torch.uint32), "u8": (torch.uint8,)}


def _dev(t, kind: str, count: int, name: str):
    """Pointer to a device tensor the qqa_dev_* kernels read or write: it must be a contiguous
    CUDA tensor of the element type `kind` holding at least `count` elements.  Anything else
    is refused here, before a kernel could access memory outside it."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: a CUDA tensor is required, got {type(t).__name__}")
    if t.dtype not in _DTYPES[kind]:
        raise ValueError(f"{name}: dtype {t.dtype} where {kind} is required")
    if t.numel() < count:
        raise ValueError(f"{name}: {t.numel()} elements, at least {count} required")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor is on {t.device}, the kernels need device memory")
    return _ptr(t)


def _state(t, rows: int, S: int, name: str):
    return _dev(t, "f32", rows * qqa_replica_stride(S), name)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_check(rc: int):
    if rc < 0:
        raise QQAError(rc, lib().qqa_dev_last_error().decode())
    return rc


# ---- schedule ---------------------------------------------------------------------------

def qqa_schedule_default(problem, n: int) -> qqa_schedule:
    s = qqa_schedule()
    lib().qqa_schedule_default(C.byref(s), PROBLEMS[problem], n)
    return s


def schedule(problem, n: int, **overrides) -> qqa_schedule:
    """Default schedule with named fields replaced."""
    s = qqa_schedule_default(problem, n)
    for k, v in overrides.items():
        if k == "rule" and isinstance(v, str):
            v = {"adamw": QQA_STEP_ADAMW, "langevin": QQA_STEP_LANGEVIN}[v]
        setattr(s, k, v)
    return s


def qqa_replica_stride(S: int) -> int:
    return lib().qqa_replica_stride(S)


# ---- device-level stages ---------------------------------------------------------------------

class DevGraph:
    """Device copy of a CSR graph dict (qqa_inputs format) as int32 CSR + float32 weights,
    or of a dense matrix; `.struct` is the qqa_dev_graph the library reads."""

    def __init__(self, g: dict | None = None, dense: np.ndarray | None = None, device="cuda"):
        if dense is not None:
            self.dense = torch.as_tensor(np.ascontiguousarray(dense, np.float32), device=device)
            self.n = int(dense.shape[0])
            self.row_ptr = self.col = self.weight = None
            self.struct = qqa_dev_graph(self.n, 0, None, None, None, _ptr(self.dense))
            return
        self.n = int(g["n"])
        self.row_ptr = torch.as_tensor(np.asarray(g["row_ptr"], np.int32), device=device)
        self.col = torch.as_tensor(np.asarray(g["col"], np.int32), device=device)
        w = g.get("weight")
        self.weight = None if w is None else torch.as_tensor(np.asarray(w, np.float32), device=device)
        self.dense = None
        self.struct = qqa_dev_graph(self.n, int(self.col.numel()), _ptr(self.row_ptr), _ptr(self.col),
                                    _ptr(self.weight), None)


def qqa_dev_philox(seed, n, nquads, k, stream_id, out, stream=None):
    out_p = _dev(out, "u32", 4 * max(n, 0) * max(nquads, 0), "out")
    return _dev_check(lib().qqa_dev_philox(seed, n, nquads, k, stream_id, out_p, _stream(stream)))


def qqa_dev_noise(seed, n, S, k, xi, stream=None):
    return _dev_check(lib().qqa_dev_noise(seed, n, S, k, _state(xi, n, S, "xi"), _stream(stream)))


def qqa_dev_init(seed, n, S, P, m=None, v=None, stream=None):
    return _dev_check(lib().qqa_dev_init(seed, n, S, _state(P, n, S, "P"), _state(m, n, S, "m"), _state(v, n, S, "v"),
                                         _stream(stream)))


def qqa_dev_step(g: DevGraph, problem, sched: qqa_schedule | None, S, t, K, seed, P_in, P_out, m, v,
                 lanes_per_row=0, stream=None):
    n = g.n
    return _dev_check(lib().qqa_dev_step(C.byref(g.struct), PROBLEMS[problem], None if sched is None else C.byref(sched),
                                         S, t, K, seed, _state(P_in, n, S, "P_in"), _state(P_out, n, S, "P_out"),
                                         _state(m, n, S, "m"), _state(v, n, S, "v"), lanes_per_row, _stream(stream)))


def qqa_dev_run(g: DevGraph, problem, sched: qqa_schedule | None, S, t0, t1, K, seed, P0, P1, m, v,
                engine="auto", lanes_per_row=0, stream=None):
    e = ENGINES[engine] if isinstance(engine, str) else engine
    n = g.n
    return _dev_check(lib().qqa_dev_run(C.byref(g.struct), PROBLEMS[problem], None if sched is None else C.byref(sched),
                                        S, t0, t1, K, seed, _state(P0, n, S, "P0"), _state(P1, n, S, "P1"),
                                        _state(m, n, S, "m"), _state(v, n, S, "v"), e, lanes_per_row, _stream(stream)))


def qqa_dev_replica_sums(P, n, S, T, stream=None):
    """T (device uint64/int64 tensor of stride entries) = per-replica sums of P in 2^-32 units."""
    return _dev_check(lib().qqa_dev_replica_sums(_state(P, n, S, "P"), n, S, _dev(T, "u64", qqa_replica_stride(S), "T"),
                                                 _stream(stream)))


def qqa_dev_dense_coupling(W, P, C, n, S, problem, stream=None):
    return _dev_check(lib().qqa_dev_dense_coupling(_dev(W, "f32", n * n, "W"), _state(P, n, S, "P"), _state(C, n, S, "C"),
                                                   n, S, PROBLEMS[problem], _stream(stream)))


def qqa_dev_color_step(g: DevGraph, colors, sched: qqa_schedule | None, S, t, K, seed, V_in, V_out, m, v,
                       lanes_per_row=0, stream=None):
    rows = g.n * max(colors, 0)
    return _dev_check(lib().qqa_dev_color_step(C.byref(g.struct), colors, None if sched is None else C.byref(sched),
                                               S, t, K, seed, _state(V_in, rows, S, "V_in"), _state(V_out, rows, S, "V_out"),
                                               _state(m, rows, S, "m"), _state(v, rows, S, "v"),
                                               lanes_per_row, _stream(stream)))


def qqa_dev_color_eval(g: DevGraph, colors, S, V, X, conflicts, best, stream=None):
    stride = qqa_replica_stride(S)
    return _dev_check(lib().qqa_dev_color_eval(C.byref(g.struct), colors, S, _state(V, g.n * max(colors, 0), S, "V"),
                                               _dev(X, "u8", g.n * stride, "X"), _dev(conflicts, "i64", S, "conflicts"),
                                               _dev(best, "i32", 1, "best"), _stream(stream)))


def _eval_args(g, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best, stream):
    return (C.byref(g.struct), PROBLEMS[problem], penalty_lambda, S, _state(P, g.n, S, "P"),
            _dev(size_or_cut, "i64", S, "size_or_cut"), _dev(viol, "i64", S, "viol"), _dev(obj, "i64", S, "obj"),
            _dev(best, "i32", 1, "best"), _stream(stream))


def qqa_dev_eval(g: DevGraph, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best, stream=None):
    return _dev_check(lib().qqa_dev_eval(*_eval_args(g, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best,
                                                     stream)))


def qqa_dev_eval_noalloc(g: DevGraph, problem, penalty_lambda, S, P, size_or_cut, viol, obj, best, stream=None):
    """qqa_dev_eval on the library's fixed device scratch (no allocation)."""
    return _dev_check(lib().qqa_dev_eval_noalloc(*_eval_args(g, problem, penalty_lambda, S, P, size_or_cut, viol, obj,
                                                             best, stream)))


# ---- request-level API ------------------------------------------------------------------------

def host_graph(g: dict | None = None, dense: np.ndarray | None = None):
    """qqa_graph over host arrays; returns (struct, keepalive)."""
    if dense is not None:
        d = np.ascontiguousarray(dense, np.float32)
        return qqa_graph(d.shape[0], 0, None, None, None, _ptr(d)), (d,)
    rp = np.ascontiguousarray(g["row_ptr"], np.int64)
    col = np.ascontiguousarray(g["col"], np.int32)
    w = g.get("weight")
    w = None if w is None else np.ascontiguousarray(w, np.float32)
    return qqa_graph(int(g["n"]), int(col.size), _ptr(rp), _ptr(col), _ptr(w), None), (rp, col, w)


def qqa_graph_validate(g: dict | None = None, problem="mis", dense: np.ndarray | None = None):
    """(return code, message) of the library's host-side graph check."""
    st, keep = host_graph(g, dense)
    buf = C.create_string_buffer(256)
    rc = lib().qqa_graph_validate(C.byref(st), PROBLEMS[problem], buf, 256)
    return rc, buf.value.decode()


class Result(dict):
    pass


class Context:
    """One qqa_ctx (device context with its own stream unless one is given)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        self._c = C.c_void_p()
        s = None if stream is None else _stream(stream)
        rc = lib().qqa_create(C.byref(self._c), device, hbm_budget, s)
        if rc != QQA_OK:
            raise QQAError(rc, "qqa_create failed")
        self._pending = {}

    def _check(self, rc):
        if rc < 0:
            raise QQAError(rc, lib().qqa_last_error(self._c).decode())
        return rc

    def close(self):
        if self._c:
            lib().qqa_destroy(self._c)
            self._c = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, g: dict | None = None, problem="mis", dense: np.ndarray | None = None) -> int:
        st, keep = host_graph(g, dense)
        gid = C.c_int64()
        self._check(lib().qqa_graph_upload(self._c, C.byref(st), PROBLEMS[problem], C.byref(gid)))
        return gid.value

    def set_engine(self, policy):
        self._check(lib().qqa_set_engine(self._c, ENGINES[policy] if isinstance(policy, str) else policy))

    def set_replica_layout(self, S: int, lanes_per_row: int):
        self._check(lib().qqa_set_replica_layout(self._c, S, lanes_per_row))

    def autotune(self, gid: int, problem, S: int) -> int:
        out = C.c_int32()
        self._check(lib().qqa_autotune(self._c, gid, PROBLEMS[problem], S, C.byref(out)))
        return out.value

    def autotune_batch(self, gids, problems, S, steps, sched=None) -> tuple[bool, list[int]]:
        """Tune replica layouts, and the resident-or-slot choice, on shortened copies of this
        batch; returns whether the resident engine was kept and each instance's lanes per row."""
        cnt = len(gids)
        g = np.asarray(gids, np.int64)
        pr = np.asarray([PROBLEMS[p] for p in problems], np.int32)
        Ss = np.asarray(S, np.int32)
        ks = np.asarray(steps, np.int32)
        if not (len(pr) == len(Ss) == len(ks) == cnt) or (sched is not None and len(sched) != cnt):
            raise ValueError("batch arrays must have one entry per instance")
        sch = None if sched is None else (qqa_schedule * cnt)(*sched)
        out = C.c_int32()
        lanes = np.zeros(cnt, np.int32)
        self._check(lib().qqa_autotune_batch(self._c, cnt, _ptr(g), _ptr(pr), sch, _ptr(Ss), _ptr(ks), _ptr(lanes),
                                             C.byref(out)))
        return bool(out.value), [int(x) for x in lanes]

    def release(self, gid: int):
        self._check(lib().qqa_graph_release(self._c, gid))

    def _track(self, rid, n, S):
        self._pending[rid] = (n, S)
        return rid

    def solve(self, g: dict | None, problem, S, steps, seed, sched=None, dense=None) -> int:
        st, keep = host_graph(g, dense)
        rid = C.c_int64()
        self._check(lib().qqa_solve(self._c, C.byref(st), PROBLEMS[problem],
                                    None if sched is None else C.byref(sched), S, steps, seed, C.byref(rid)))
        return self._track(rid.value, st.n, S)

    def solve_coloring(self, g: dict, colors: int, S, steps, seed, sched=None) -> int:
        st, keep = host_graph(g)
        rid = C.c_int64()
        self._check(lib().qqa_solve_coloring(self._c, C.byref(st), colors, None if sched is None else C.byref(sched),
                                             S, steps, seed, C.byref(rid)))
        return self._track(rid.value, int(g["n"]), S)

    def solve_coloring_resident(self, gid: int, n: int, colors: int, S, steps, seed, sched=None) -> int:
        rid = C.c_int64()
        self._check(lib().qqa_solve_coloring_resident(self._c, gid, colors, None if sched is None else C.byref(sched),
                                                      S, steps, seed, C.byref(rid)))
        return self._track(rid.value, n, S)

    def solve_resident(self, gid: int, n: int, problem, S, steps, seed, sched=None) -> int:
        rid = C.c_int64()
        self._check(lib().qqa_solve_resident(self._c, gid, PROBLEMS[problem], None if sched is None else C.byref(sched),
                                             S, steps, seed, C.byref(rid)))
        return self._track(rid.value, n, S)

    def solve_batch(self, gids, ns, problems, S, steps, seeds, sched=None) -> list[int]:
        cnt = len(gids)
        g = np.asarray(gids, np.int64)
        pr = np.asarray([PROBLEMS[p] for p in problems], np.int32)
        Ss = np.asarray(S, np.int32)
        ks = np.asarray(steps, np.int32)
        sd = np.asarray(seeds, np.uint64)
        out = np.zeros(cnt, np.int64)
        sch = None
        if sched is not None:
            sch = (qqa_schedule * cnt)(*sched)
        self._check(lib().qqa_solve_batch(self._c, cnt, _ptr(g), _ptr(pr), sch, _ptr(Ss), _ptr(ks), _ptr(sd),
                                          _ptr(out)))
        return [self._track(int(r), int(n), int(s)) for r, n, s in zip(out, ns, Ss)]

    def serve_start(self, max_slots: int = 256):
        self._check(lib().qqa_serve_start(self._c, max_slots))

    def serve_submit(self, g: dict | None, problem, S, steps, seed, sched=None, dense=None) -> int:
        st, keep = host_graph(g, dense)
        rid = C.c_int64()
        self._check(lib().qqa_serve_submit(self._c, C.byref(st), PROBLEMS[problem],
                                           None if sched is None else C.byref(sched), S, steps, seed, C.byref(rid)))
        return self._track(rid.value, st.n, S)

    def serve_set_deadline(self, deadline_ms: float):
        self._check(lib().qqa_serve_set_deadline(self._c, float(deadline_ms)))

    def serve_stats(self) -> dict:
        st = qqa_serve_stats()
        self._check(lib().qqa_serve_get_stats(self._c, C.byref(st)))
        return {f: getattr(st, f) for f, _ in qqa_serve_stats._fields_}

    def serve_stop(self):
        self._check(lib().qqa_serve_stop(self._c))

    def cancel(self, rid: int):
        self._check(lib().qqa_cancel(self._c, rid))

    def poll(self, rid: int, timeout_us: int = -1, want_x: bool = True) -> Result | None:
        """Result dict when done, None while pending; raises on errors."""
        n, S = self._pending[rid]
        objs = np.zeros(S, np.int64)
        size = np.zeros(S, np.int64)
        viol = np.zeros(S, np.int64)
        x = np.zeros(n, np.uint8) if want_x else None
        res = qqa_result()
        res.replica_objective = objs.ctypes.data
        res.replica_size_or_cut = size.ctypes.data
        res.replica_violations = viol.ctypes.data
        res.best_x = None if x is None else x.ctypes.data
        rc = lib().qqa_poll(self._c, rid, C.byref(res), timeout_us)
        if rc == QQA_PENDING:
            return None
        self._pending.pop(rid, None)
        self._check(rc)
        return Result(best_replica=res.best_replica, feasible=bool(res.feasible), best_objective=res.best_objective,
                      best_size_or_cut=res.best_size_or_cut, best_violations=res.best_violations, obj=objs,
                      size_or_cut=size, viol=viol, best_x=x, queue_ms=res.queue_ms, device_ms=res.device_ms,
                      step_loop_ms=res.step_loop_ms, latency_ms=res.latency_ms, kernel_us=res.kernel_us,
                      first_update_ms=res.first_update_ms,
                      engine={v: k for k, v in ENGINES.items()}.get(res.engine, res.engine))
