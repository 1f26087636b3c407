"""FP64 CPU oracle for the PQQA replica update -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It wraps ``qqa_oracle.c`` (plain single-threaded double-precision C, built
with gcc) through ctypes; it shares no code with the solver library.

Every function here is a thin marshalling layer: the arithmetic lives in the C file,
whose header lists what pins each function.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qqa_oracle.c")
_LIB = os.path.join(_HERE, "libqqa_oracle.so")

MIS, MAXCUT, MAXCLIQUE = 0, 1, 2
ADAMW, LANGEVIN = 0, 1
STREAM_INIT, STREAM_NOISE = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("gamma_min", C.c_double), ("gamma_max", C.c_double), ("lr", C.c_double),
                ("weight_decay", C.c_double), ("temperature", C.c_double),
                ("comm_alpha", C.c_double), ("entropy_alpha", C.c_int32), ("rule", C.c_int32),
                ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("lam", C.c_double), ("problem", C.c_int32), ("pad_", C.c_int32)]


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("dense", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("weight", C.c_void_p), ("W", C.c_void_p)]


@dataclasses.dataclass
class Params:
    """Solver hyper-parameters.  Defaults: gamma from -2 to 0.1, alpha-entropy alpha = 4,
    AdamW with weight decay 0.01, temperature 1e-3 (Implementation paragraph and the
    appendix sections on the schedule and optimiser); lr, comm_alpha and the Adam
    moments are choices the paper leaves open."""
    problem: int = MIS
    gamma_min: float = -2.0
    gamma_max: float = 0.1
    lr: float = 0.1
    weight_decay: float = 0.01
    temperature: float = 1e-3
    comm_alpha: float = 0.1
    entropy_alpha: int = 4
    rule: int = ADAMW
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    lam: float = 2.0

    def as_float32(self) -> "Params":
        """Copy with every real parameter rounded to binary32, i.e. the values a
        single-precision solver actually sees."""
        d = dataclasses.asdict(self)
        for k, v in d.items():
            if isinstance(v, float):
                d[k] = float(np.float32(v))
        return Params(**d)

    def _c(self) -> _Params:
        return _Params(self.gamma_min, self.gamma_max, self.lr, self.weight_decay,
                       self.temperature, self.comm_alpha, self.entropy_alpha, self.rule,
                       self.beta1, self.beta2, self.adam_eps, self.lam, self.problem, 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i32, u32, u64, i64, d = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox4x32_10_inverse.argtypes = [vp, vp, vp]
        L.orc_u01.argtypes = [u32]
        L.orc_u01.restype = d
        L.orc_normals4.argtypes = [vp, vp]
        L.orc_philox_grid.argtypes = [u64, i32, i32, u32, u32, vp]
        L.orc_noise.argtypes = [u64, i32, i32, u32, vp]
        L.orc_init.argtypes = [u64, i32, i32, vp]
        L.orc_gamma.argtypes = [vp, i32, i32]
        L.orc_gamma.restype = d
        L.orc_energy.argtypes = [vp, vp, i32, vp, d]
        L.orc_energy.restype = d
        L.orc_grad.argtypes = [vp, vp, i32, vp, d, vp, vp, vp, vp]
        L.orc_step.argtypes = [vp, vp, i32, i32, i32, u64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_run.argtypes = [vp, vp, i32, i32, i32, i32, u64, vp, vp, vp]
        L.orc_eval.argtypes = [i32, i64, vp, i32, vp, vp, vp, vp, vp]
        L.orc_eval.restype = C.c_int
        L.orc_cat_sigma.argtypes = [i32, i32, i32, vp, vp, vp]
        L.orc_cat_entropy.argtypes = [i32, i32, i32, C.c_int, vp, i32]
        L.orc_cat_entropy.restype = d
        L.orc_cat_energy.argtypes = [vp, vp, i32, i32, vp, d]
        L.orc_cat_energy.restype = d
        L.orc_cat_grad.argtypes = [vp, vp, i32, i32, vp, d, vp, vp]
        L.orc_cat_step.argtypes = [vp, vp, i32, i32, i32, i32, u64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_cat_run.argtypes = [vp, vp, i32, i32, i32, i32, i32, u64, vp, vp, vp]
        L.orc_cat_eval.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _GraphRef:
    """Keeps the numpy arrays behind an orc_graph alive while C uses them."""

    def __init__(self, g: dict | None = None, W: np.ndarray | None = None):
        if W is not None:
            self.W = np.ascontiguousarray(W, dtype=np.float64)
            self.s = _Graph(self.W.shape[0], 1, None, None, None, _p(self.W))
        else:
            self.rp = np.ascontiguousarray(g["row_ptr"], dtype=np.int64)
            self.col = np.ascontiguousarray(g["col"], dtype=np.int32)
            w = g.get("weight")
            self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
            self.s = _Graph(g["n"], 0, _p(self.rp), _p(self.col), _p(self.w), None)

    @property
    def n(self) -> int:
        return self.s.n

    def ptr(self):
        return C.byref(self.s)


def graph(g: dict | None = None, W: np.ndarray | None = None) -> _GraphRef:
    """Oracle view of a CSR graph dict (qqa_inputs format) or of a dense matrix W."""
    return _GraphRef(g, W)


def _as_graph(g) -> _GraphRef:
    if isinstance(g, _GraphRef):
        return g
    if isinstance(g, np.ndarray):
        return _GraphRef(W=g)
    return _GraphRef(g)


# ---- random numbers ----------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def philox_inverse(out, key) -> np.ndarray:
    o = np.ascontiguousarray(out, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    c = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10_inverse(_p(o), _p(k), _p(c))
    return c


def philox_grid(seed: int, n: int, nquads: int, k: int, stream: int) -> np.ndarray:
    out = np.zeros((n, nquads, 4), np.uint32)
    lib().orc_philox_grid(seed, n, nquads, k, stream, _p(out))
    return out


def u01(r: int) -> float:
    return lib().orc_u01(int(r))


def normals4(r) -> np.ndarray:
    rr = np.ascontiguousarray(r, dtype=np.uint32)
    xi = np.zeros(4)
    lib().orc_normals4(_p(rr), _p(xi))
    return xi


def noise(seed: int, n: int, S: int, k: int) -> np.ndarray:
    xi = np.zeros((n, S))
    lib().orc_noise(seed, n, S, k, _p(xi))
    return xi


def init(seed: int, n: int, S: int) -> np.ndarray:
    P = np.zeros((n, S))
    lib().orc_init(seed, n, S, _p(P))
    return P


# ---- the method ---------------------------------------------------------------------------

def gamma(params: Params, t: int, K: int) -> float:
    pr = params._c()
    return lib().orc_gamma(C.byref(pr), t, K)


def energy(params: Params, g, P: np.ndarray, gamma_value: float) -> float:
    G = _as_graph(g)
    pr = params._c()
    P = np.ascontiguousarray(P, dtype=np.float64)
    return lib().orc_energy(C.byref(pr), G.ptr(), P.shape[1], _p(P), gamma_value)


def grad(params: Params, g, P: np.ndarray, gamma_value: float):
    """Returns (gf, ge, gc, sigma)."""
    G = _as_graph(g)
    pr = params._c()
    P = np.ascontiguousarray(P, dtype=np.float64)
    n, S = P.shape
    gf, ge, gc = np.zeros((n, S)), np.zeros((n, S)), np.zeros((n, S))
    sigma = np.zeros(n)
    lib().orc_grad(C.byref(pr), G.ptr(), S, _p(P), gamma_value, _p(gf), _p(ge), _p(gc), _p(sigma))
    return gf, ge, gc, sigma


def step(params: Params, g, t: int, K: int, seed: int, P, m, v) -> dict:
    """One update from state (P, m, v) (any float dtype; promoted exactly to float64).
    Returns P, m, v after the update plus the diagnostics pre_clamp, g, gabs, sigma."""
    G = _as_graph(g)
    pr = params._c()
    P_in = np.array(P, dtype=np.float64, order="C")
    n, S = P_in.shape
    m2 = np.array(m, dtype=np.float64, order="C")
    v2 = np.array(v, dtype=np.float64, order="C")
    out = {k: np.zeros((n, S)) for k in ("P", "pre_clamp", "g", "gabs")}
    out["sigma"] = np.zeros(n)
    lib().orc_step(C.byref(pr), G.ptr(), S, t, K, seed, _p(P_in), _p(out["P"]), _p(m2), _p(v2),
                   _p(out["pre_clamp"]), _p(out["g"]), _p(out["gabs"]), _p(out["sigma"]))
    out["m"], out["v"] = m2, v2
    return out


def run(params: Params, g, t0: int, t1: int, K: int, seed: int, P, m, v):
    """Updates t0..t1-1 applied to copies of (P, m, v); returns the new (P, m, v)."""
    G = _as_graph(g)
    pr = params._c()
    P2 = np.array(P, dtype=np.float64, order="C")
    m2 = np.array(m, dtype=np.float64, order="C")
    v2 = np.array(v, dtype=np.float64, order="C")
    lib().orc_run(C.byref(pr), G.ptr(), P2.shape[1], t0, t1, K, seed, _p(P2), _p(m2), _p(v2))
    return P2, m2, v2


def evaluate(problem: int, lam: int, g, P) -> dict:
    """Round x = [p > 1/2] and evaluate exactly; returns per-replica int64 arrays and best."""
    G = _as_graph(g)
    P = np.ascontiguousarray(P, dtype=np.float64)
    S = P.shape[1]
    a, b, o = np.zeros(S, np.int64), np.zeros(S, np.int64), np.zeros(S, np.int64)
    best = np.zeros(1, np.int32)
    rc = lib().orc_eval(problem, int(lam), G.ptr(), S, _p(P), _p(a), _p(b), _p(o), _p(best))
    if rc != 0:
        raise ValueError("weight not on the 2^-16 grid")
    return {"size_or_cut": a, "viol": b, "obj": o, "best": int(best[0])}


def solve(params: Params, g, S: int, K: int, seed: int) -> dict:
    """Whole run: U(0,1) init, K updates, rounding and exact evaluation."""
    G = _as_graph(g)
    P = init(seed, G.n, S)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    P, m, v = run(params, G, 0, K, K, seed, P, m, v)
    res = evaluate(params.problem, int(round(params.lam)), G, P)
    res["P"] = P
    return res


# ---- categorical K-state variant (graph coloring) -------------------------------------------
# V has shape (n, K, S): V[i, k, s] is the clamped weight of colour k for variable i in replica s.

def _v3(V):
    return np.ascontiguousarray(V, dtype=np.float64)


def cat_sigma(V):
    """(sigma, Z): Clamp-normalised probabilities and the row sums Z (n, S)."""
    V = _v3(V)
    n, K, S = V.shape
    sg = np.zeros_like(V)
    Z = np.zeros((n, S))
    lib().orc_cat_sigma(n, K, S, _p(V), _p(sg), _p(Z))
    return sg, Z


def cat_entropy(sigma, alpha: int = 4) -> np.ndarray:
    """s_K per replica."""
    sg = _v3(sigma)
    n, K, S = sg.shape
    return np.array([lib().orc_cat_entropy(n, K, S, alpha, _p(sg), s) for s in range(S)])


def cat_energy(params: Params, g, V, gamma_value: float) -> float:
    G = _as_graph(g)
    pr = params._c()
    V = _v3(V)
    return lib().orc_cat_energy(C.byref(pr), G.ptr(), V.shape[1], V.shape[2], _p(V), gamma_value)


def cat_grad(params: Params, g, V, gamma_value: float):
    """(dR/dV, gabs)."""
    G = _as_graph(g)
    pr = params._c()
    V = _v3(V)
    gV, ga = np.zeros_like(V), np.zeros_like(V)
    lib().orc_cat_grad(C.byref(pr), G.ptr(), V.shape[1], V.shape[2], _p(V), gamma_value, _p(gV), _p(ga))
    return gV, ga


def cat_step(params: Params, g, t: int, Kt: int, seed: int, V, m, v) -> dict:
    G = _as_graph(g)
    pr = params._c()
    V_in = _v3(V)
    n, K, S = V_in.shape
    m2, v2 = _v3(m).copy(), _v3(v).copy()
    out = {k: np.zeros_like(V_in) for k in ("V", "pre_clamp", "g", "gabs")}
    lib().orc_cat_step(C.byref(pr), G.ptr(), K, S, t, Kt, seed, _p(V_in), _p(out["V"]), _p(m2), _p(v2),
                       _p(out["pre_clamp"]), _p(out["g"]), _p(out["gabs"]))
    out["m"], out["v"] = m2, v2
    return out


def cat_init(seed: int, n: int, K: int, S: int) -> np.ndarray:
    """U(0,1) start with Philox row index i*K + k."""
    return init(seed, n * K, S).reshape(n, K, S)


def cat_run(params: Params, g, t0: int, t1: int, Kt: int, seed: int, V, m, v):
    G = _as_graph(g)
    pr = params._c()
    V2, m2, v2 = _v3(V).copy(), _v3(m).copy(), _v3(v).copy()
    n, K, S = V2.shape
    lib().orc_cat_run(C.byref(pr), G.ptr(), K, S, t0, t1, Kt, seed, _p(V2), _p(m2), _p(v2))
    return V2, m2, v2


def cat_eval(g, V) -> dict:
    """colors (n, S) = argmax_k V (first maximum), conflicts (S,), best replica."""
    G = _as_graph(g)
    V = _v3(V)
    n, K, S = V.shape
    colors = np.zeros((n, S), np.int32)
    conf = np.zeros(S, np.int64)
    best = np.zeros(1, np.int32)
    lib().orc_cat_eval(G.ptr(), K, S, _p(V), _p(colors), _p(conf), _p(best))
    return {"colors": colors, "conflicts": conf, "best": int(best[0])}


def cat_solve(params: Params, g, K: int, S: int, steps: int, seed: int) -> dict:
    G = _as_graph(g)
    V = cat_init(seed, G.n, K, S)
    z = np.zeros_like(V)
    V, _, _ = cat_run(params, G, 0, steps, steps, seed, V, z, z)
    res = cat_eval(G, V)
    res["V"] = V
    return res
