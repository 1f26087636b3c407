"""Seeded synthetic inputs for the QQA solver: graphs, weights, solver states, request streams.

This module is shared by the tests, the benchmark and the oracle's test harness.  It
holds none of the method's arithmetic: it only draws instances (graph structure,
coupling weights, starting states, arrival times) from fixed random models, each
seeded so that every caller sees the same bytes.

Graph models (the paper's benchmark families, regenerated synthetically because the
datasets themselves are not available):
  * random d-regular graphs (pairing model), the family of the MIS scaling study;
  * Erdos-Renyi G(n, p), the family of the ER-[700-800] / ER-[9000-11000] MIS sets;
  * Barabasi-Albert preferential attachment with m edges per new node, the BA max-cut
    family;
  * complete graphs with Gaussian couplings quantised to a 2^-16 grid (dense max-cut);
  * Model RB constraint-satisfaction instances with a planted solution, as the
    compatibility graphs whose cliques are consistent partial assignments (max clique);
  * queens graphs (graph coloring).

A graph is returned as a dict ``{"n", "row_ptr" (int64, n+1), "col" (int32, nnz),
"weight" (float32, nnz, or None)}`` holding a symmetric CSR without self-loops or
duplicate entries, columns sorted within each row.
"""

from __future__ import annotations

import math

import numpy as np

WEIGHT_QUANTUM = 2.0 ** -16
"""Max-cut weights are integer multiples of this quantum, so discrete objectives are exact."""


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed))


def csr_from_edges(n: int, edges: np.ndarray, weights: np.ndarray | None = None) -> dict:
    """Symmetric CSR from an array of undirected edges (i, j), i != j, no duplicates."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if edges.size:
        if np.any(edges[:, 0] == edges[:, 1]):
            raise ValueError("self-loop in edge list")
        lo = np.minimum(edges[:, 0], edges[:, 1])
        hi = np.maximum(edges[:, 0], edges[:, 1])
        key = lo * n + hi
        if np.unique(key).size != key.size:
            raise ValueError("duplicate edge in edge list")
    src = np.concatenate([edges[:, 0], edges[:, 1]])
    dst = np.concatenate([edges[:, 1], edges[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    g = {"n": int(n), "row_ptr": row_ptr, "col": dst.astype(np.int32), "weight": None}
    if weights is not None:
        w = np.asarray(weights, dtype=np.float32).reshape(-1)
        g["weight"] = np.concatenate([w, w])[order].astype(np.float32)
    return g


def edge_list(g: dict) -> np.ndarray:
    """Undirected edges (i < j) of a CSR graph, one row per edge."""
    n = g["n"]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(g["row_ptr"]))
    cols = g["col"].astype(np.int64)
    keep = rows < cols
    return np.stack([rows[keep], cols[keep]], axis=1)


def random_regular(n: int, d: int, seed) -> dict:
    """Random simple d-regular graph: pairing (configuration) model, resampled until simple.

    Exactly uniform over simple d-regular graphs; practical for small d (the acceptance
    probability is about exp(-(d*d-1)/4))."""
    if (n * d) % 2 or d >= n:
        raise ValueError("need n*d even and d < n")
    rng = _rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    for _ in range(100000):
        perm = rng.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        return csr_from_edges(n, np.stack([lo, hi], axis=1))
    raise RuntimeError("pairing model did not produce a simple graph")


def random_regular_swapped(n: int, d: int, seed) -> dict:
    """Random simple d-regular graph for large d: one pairing (configuration model), then
    each self-loop or repeated edge is removed by a double-edge swap with a uniformly chosen
    other edge, (u, v), (x, y) -> (u, x), (v, y), taken only when both new edges are new and
    not loops.  Degrees stay exactly d; the distribution is close to uniform (the swaps act
    on O(d^2) of the n d / 2 edges), which is what the large random-regular MIS instances
    need."""
    if (n * d) % 2 or d >= n:
        raise ValueError("need n*d even and d < n")
    rng = _rng(seed)
    stubs = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), d))
    lo = np.minimum(stubs[0::2], stubs[1::2])
    hi = np.maximum(stubs[0::2], stubs[1::2])
    key = lo * n + hi
    order = np.argsort(key, kind="stable")
    dup = np.zeros(key.size, bool)
    dup[order[1:]] = key[order[1:]] == key[order[:-1]]
    bad_mask = (lo == hi) | dup
    bad = np.nonzero(bad_mask)[0].tolist()
    if bad:
        present = set(np.unique(key[~bad_mask]).tolist())
        pending = set(bad)
        for e in bad:
            u, v = int(lo[e]), int(hi[e])
            for _ in range(10000):
                f = int(rng.integers(key.size))
                if f in pending:
                    continue
                x, y = int(lo[f]), int(hi[f])
                if rng.random() < 0.5:
                    x, y = y, x
                k1 = min(u, x) * n + max(u, x)
                k2 = min(v, y) * n + max(v, y)
                if u == x or v == y or k1 == k2 or k1 in present or k2 in present:
                    continue
                present.discard(int(key[f]))
                present.update((k1, k2))
                lo[e], hi[e], key[e] = min(u, x), max(u, x), k1
                lo[f], hi[f], key[f] = min(v, y), max(v, y), k2
                break
            else:
                raise RuntimeError("no valid swap found")
            pending.discard(e)
    return csr_from_edges(n, np.stack([lo, hi], axis=1))


def erdos_renyi(n: int, mean_degree: float, seed) -> dict:
    """G(n, p) with p = mean_degree / (n - 1).

    The edge count is drawn from Binomial(n(n-1)/2, p) and that many distinct pairs are
    then drawn uniformly, which is the same distribution as independent edge coins."""
    rng = _rng(seed)
    pairs = n * (n - 1) // 2
    p = 0.0 if n < 2 else min(1.0, float(mean_degree) / (n - 1))
    m = int(rng.binomial(pairs, p)) if pairs else 0
    if m == 0:
        return csr_from_edges(n, np.zeros((0, 2), np.int64))
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        want = int((m - keys.size) * 1.1) + 16
        i = rng.integers(0, n, size=want)
        j = rng.integers(0, n, size=want)
        ok = i != j
        lo, hi = np.minimum(i[ok], j[ok]), np.maximum(i[ok], j[ok])
        keys = np.unique(np.concatenate([keys, lo * n + hi]))
    keys = rng.choice(keys, size=m, replace=False)
    return csr_from_edges(n, np.stack([keys // n, keys % n], axis=1))


def barabasi_albert(n: int, m: int, seed) -> dict:
    """Preferential attachment: start from the complete graph on m+1 nodes, then each new
    node joins m distinct existing nodes chosen with probability proportional to degree."""
    if n <= m:
        raise ValueError("need n > m")
    rng = _rng(seed)
    edges = [(i, j) for i in range(m + 1) for j in range(i + 1, m + 1)]
    # every node appears in `ends` once per incident edge: a uniform draw from it is a
    # degree-proportional draw over nodes
    ends = [v for e in edges for v in e]
    draws = rng.random(size=4 * m * n + 64)
    pos = 0
    for v in range(m + 1, n):
        chosen: list[int] = []
        while len(chosen) < m:
            if pos >= draws.size:
                draws = rng.random(size=4 * m * n + 64)
                pos = 0
            u = ends[int(draws[pos] * len(ends))]
            pos += 1
            if u not in chosen:
                chosen.append(u)
        for u in chosen:
            edges.append((u, v))
            ends.append(u)
            ends.append(v)
    return csr_from_edges(n, np.asarray(edges, dtype=np.int64))


def pm1_weights(g: dict, seed) -> dict:
    """Copy of `g` with iid uniform +-1 weights per undirected edge (mirrored)."""
    e = edge_list(g)
    rng = _rng(seed)
    w = np.where(rng.random(e.shape[0]) < 0.5, -1.0, 1.0).astype(np.float32)
    return csr_from_edges(g["n"], e, w)


def dense_gaussian(n: int, seed, clip: float = 8.0) -> np.ndarray:
    """Symmetric n x n float32 coupling matrix with N(0,1) entries rounded to the 2^-16
    grid and clipped to |w| < clip, zero diagonal (the complete-graph max-cut instance)."""
    rng = _rng(seed)
    z = rng.standard_normal((n, n))
    q = np.clip(np.rint(z / WEIGHT_QUANTUM), -(clip / WEIGHT_QUANTUM - 1), clip / WEIGHT_QUANTUM - 1)
    w = np.triu(q, 1)
    w = (w + w.T) * WEIGHT_QUANTUM
    return w.astype(np.float32)


def synthetic_state(n: int, S: int, seed, p_zero: float = 0.1, p_one: float = 0.1):
    """A solver state (P, m, v) as float32 n x S arrays, for single-step comparisons.

    P mixes interior U(0,1) values with exact 0 and 1 (clamped replicas); m is centred
    Gaussian; v is positive, of the size of a squared gradient."""
    rng = _rng(seed)
    P = rng.random((n, S)).astype(np.float32)
    r = rng.random((n, S))
    P[r < p_zero] = 0.0
    P[(r >= p_zero) & (r < p_zero + p_one)] = 1.0
    m = (0.5 * rng.standard_normal((n, S))).astype(np.float32)
    v = (np.square(rng.standard_normal((n, S))) + 0.01).astype(np.float32)
    return P, m, v


def instance_batch(count: int, seed, n_range=(200, 5000), deg_range=(3.0, 20.0)) -> list[dict]:
    """`count` independent ER instances with n ~ U{n_range} and mean degree ~ U[deg_range]."""
    root = np.random.SeedSequence(seed)
    out = []
    for k, child in enumerate(root.spawn(count)):
        r = np.random.default_rng(child)
        n = int(r.integers(n_range[0], n_range[1] + 1))
        d = float(r.uniform(deg_range[0], deg_range[1]))
        out.append(erdos_renyi(n, d, int(child.generate_state(1)[0])))
    return out


def poisson_requests(rate: float, duration: float, seed, n_range=(1e3, 1e5),
                     replicas=(32, 128), steps_range=(1000, 3000)) -> list[dict]:
    """Request stream: Poisson arrivals at `rate`/s for `duration` s.  Each request is an
    MIS or +-1 max-cut instance (1/2 each) on an ER (mean degree ~ U[3,20]) or BA (m=4)
    graph (1/2 each), n log-uniform in n_range, S uniform over `replicas`, steps
    ~ U{steps_range}.  Graphs are described, not built: `build_request_graph` builds one."""
    rng = _rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(round(10 ** rng.uniform(math.log10(n_range[0]), math.log10(n_range[1]))))
        out.append({
            "arrival": t,
            "problem": "mis" if rng.random() < 0.5 else "maxcut",
            "family": "er" if rng.random() < 0.5 else "ba",
            "n": n,
            "mean_degree": float(rng.uniform(3.0, 20.0)),
            "S": int(replicas[int(rng.integers(0, len(replicas)))]),
            "steps": int(rng.integers(steps_range[0], steps_range[1] + 1)),
            "graph_seed": int(rng.integers(0, 2 ** 31)),
            "solver_seed": int(rng.integers(0, 2 ** 31)),
        })
    return out


def build_request_graph(req: dict) -> dict:
    if req["family"] == "er":
        g = erdos_renyi(req["n"], req["mean_degree"], req["graph_seed"])
    else:
        g = barabasi_albert(req["n"], 4, req["graph_seed"])
    if req["problem"] == "maxcut":
        g = pm1_weights(g, req["graph_seed"] + 1)
    return g


# --- small graphs with textbook optima (for exact pins) ------------------------------

def rb_model(n_vars: int, domain: int, r: float, p: float, seed) -> dict:
    """Model RB (Xu and Li, 2000) with a planted solution (the forced-satisfiable variant of
    Xu, Boussemart, Hemery and Lecoutre, 2007), returned as its compatibility graph.

    n_vars variables share a domain of `domain` values; m = round(r n ln n) binary
    constraints each pick two distinct variables at random (with repetition across
    constraints) and forbid round(p domain^2) value pairs chosen uniformly without
    replacement, never the pair of a planted assignment drawn first.  Graph: one node per
    (variable, value), node id variable * domain + value; an edge joins two nodes of
    different variables unless some constraint on that variable pair forbids their
    values.  A clique holds at most one node per variable, and the planted assignment is
    a clique of size n_vars, so the clique number is exactly n_vars."""
    rng = _rng(seed)
    d = int(domain)
    N = n_vars * d
    planted = rng.integers(0, d, n_vars)
    adj = np.ones((N, N), dtype=bool)
    for x in range(n_vars):
        adj[x * d:(x + 1) * d, x * d:(x + 1) * d] = False  # one value per variable
    m = int(round(r * n_vars * math.log(n_vars)))
    t = int(round(p * d * d))
    for _ in range(m):
        x, y = rng.choice(n_vars, 2, replace=False)
        allowed = np.ones(d * d, dtype=bool)
        allowed[planted[x] * d + planted[y]] = False  # the planted pair stays compatible
        pairs = rng.choice(np.nonzero(allowed)[0], t, replace=False)
        a, b = pairs // d, pairs % d
        adj[x * d + a, y * d + b] = False
        adj[y * d + b, x * d + a] = False
    iu, ju = np.nonzero(np.triu(adj, 1))
    g = csr_from_edges(N, np.stack([iu, ju], axis=1))
    g["planted_clique"] = np.arange(n_vars, dtype=np.int64) * d + planted
    return g


def queens(rows: int, cols: int | None = None) -> dict:
    """Queens graph of a rows x cols board (the coloring benchmark family): one node per
    square, node id r * cols + c, adjacent when the squares share a row, a column or a
    diagonal, i.e. a queen on one attacks the other."""
    cols = rows if cols is None else cols
    edges = []
    for a in range(rows * cols):
        ra, ca = divmod(a, cols)
        for b in range(a + 1, rows * cols):
            rb, cb = divmod(b, cols)
            if ra == rb or ca == cb or abs(ra - rb) == abs(ca - cb):
                edges.append((a, b))
    return csr_from_edges(rows * cols, np.array(edges, dtype=np.int64).reshape(-1, 2))


def cycle(n: int) -> dict:
    return csr_from_edges(n, np.array([(i, (i + 1) % n) for i in range(n)], dtype=np.int64))


def complete(n: int) -> dict:
    return csr_from_edges(n, np.array([(i, j) for i in range(n) for j in range(i + 1, n)],
                                      dtype=np.int64).reshape(-1, 2))


def complete_bipartite(a: int, b: int) -> dict:
    return csr_from_edges(a + b, np.array([(i, a + j) for i in range(a) for j in range(b)],
                                          dtype=np.int64).reshape(-1, 2))


def petersen() -> dict:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return csr_from_edges(10, np.array(outer + spokes + inner, dtype=np.int64))


def dense_to_csr(W: np.ndarray) -> dict:
    """CSR view of a dense symmetric coupling matrix (nonzero off-diagonal entries)."""
    n = W.shape[0]
    iu, ju = np.nonzero(np.triu(W, 1))
    return csr_from_edges(n, np.stack([iu, ju], axis=1), W[iu, ju])
