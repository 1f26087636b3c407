"""GPU parity of each stage of the path against the FP64 oracle, through the C ABI.

Bars: Philox integers, initial state, rounding and every discrete objective are
bit-exact; one update agrees with the oracle (run from the same float32 state, promoted
exactly to float64) within the per-step tolerance below."""

import numpy as np
import pytest

import qqa_inputs as qi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# ---- per-step tolerance contract ---------------------------------------------------------
# P in [0,1]: |dP| <= 1e-5 (absolute, i.e. relative to the range of P).  The clamp is
# 1-Lipschitz, so it needs no exemption.  m, v: |d| <= 1e-5 * max(|ref|, scale), with
# scale (1-b1) G for m and (1-b2) G^2 for v, where G is the oracle's sum of the magnitudes
# of every term of the gradient before cancellation (each neighbour's contribution to gf,
# |ge|, and alpha_c (|p| + |mu|) / sigma for the STD term): a float32 gradient carries an
# absolute error of a few ulp of G.
# An element is exempt (and counted) only where float32 cannot determine the result from
# the inputs to that accuracy: the update's derivative with respect to the gradient times
# that error bound exceeds half the tolerance while the update stays within that bound of
# [0,1] (AdamW's normalisation of a gradient that cancels to ~0 with no moment history
# flips a full step).  Exempt elements must still lie within the conditioned bound.
TOL_P = 1e-5
TOL_REL = 1e-5
ULPS = 2e-7          # float32 gradient error bound, relative to G (a few ulp)
MAX_EXEMPT_FRAC = 1e-4


def step_sensitivity(ref, m_in, v_in, t, sched, adam):
    """|d P_new / d g| of the update rule at the oracle's gradient."""
    g = ref["g"]
    if not adam:
        return np.full_like(g, float(np.float32(sched.lr)))
    k = t + 1
    b1, b2 = float(np.float32(sched.beta1)), float(np.float32(sched.beta2))
    eps, lr = float(np.float32(sched.adam_eps)), float(np.float32(sched.lr))
    c1, c2 = 1.0 / (1.0 - b1 ** k), 1.0 / (1.0 - b2 ** k)
    m1 = b1 * m_in + (1 - b1) * g
    v1 = b2 * v_in + (1 - b2) * g * g
    sq = np.sqrt(c2 * v1)
    den = sq + eps
    dsq = np.where(sq > 0, c2 * (1 - b2) * g / np.maximum(sq, 1e-300), 0.0)
    return lr * np.abs(c1 * (1 - b1) / den - c1 * m1 * dsq / (den * den))


def qqa():
    import paper_2409_02135_amd as q
    q.lib()
    return q


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def padded(a: np.ndarray, stride: int) -> np.ndarray:
    out = np.zeros((a.shape[0], stride), np.float32)
    out[:, :a.shape[1]] = a
    return out


def run_gpu_step(q, g, problem, sched, S, t, K, seed, P, m, v, lanes_per_row=0):
    stride = q.qqa_replica_stride(S)
    d = dev()
    G = q.DevGraph(dense=g["dense"]) if "dense" in g else q.DevGraph(g)
    Pi = torch.as_tensor(padded(P, stride), device=d)
    Po = torch.full_like(Pi, -7.0)
    mt = torch.as_tensor(padded(m, stride), device=d)
    vt = torch.as_tensor(padded(v, stride), device=d)
    q.qqa_dev_step(G, problem, sched, S, t, K, seed, Pi, Po, mt, vt, lanes_per_row)
    torch.cuda.synchronize()
    return Po.cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy()


def oracle_params(orc, q, sched, problem):
    return orc.Params(problem={"mis": 0, "maxcut": 1, "maxclique": 2}[problem], gamma_min=sched.gamma_min,
                      gamma_max=sched.gamma_max,
                      lr=sched.lr, weight_decay=sched.weight_decay, temperature=sched.temperature,
                      comm_alpha=sched.comm_alpha, entropy_alpha=sched.entropy_alpha, rule=sched.rule,
                      beta1=sched.beta1, beta2=sched.beta2, adam_eps=sched.adam_eps,
                      lam=float(sched.penalty_lambda)).as_float32()


def check_step(label, gpu, ref, S, adam, beta1, beta2, sens=None, comm_alpha=0.1):
    Pg, mg, vg = (x[:, :S].astype(np.float64) for x in gpu)
    assert np.all(gpu[0][:, S:] == 0.0), f"{label}: padding replicas not zero"
    assert np.all(np.isfinite(Pg)) and Pg.min() >= 0 and Pg.max() <= 1, f"{label}: P out of box"
    g, gabs, sig = ref["g"], ref["gabs"], ref["sigma"][:, None]
    dg = ULPS * gabs
    exempt = np.zeros(g.shape, bool)
    if sens is not None:
        # an update that leaves [0,1] by more than its own error bound clamps exactly
        b = sens * dg
        pre = ref["pre_clamp"]
        exempt |= (b > TOL_P / 2) & (pre > -b) & (pre < 1.0 + b)
    n_ex = int(exempt.sum())
    ok = ~exempt
    dP_all = np.abs(Pg - ref["P"])
    dP = dP_all[ok]
    stats = {"exempt": n_ex, "of": int(exempt.size), "max_dP": float(dP.max()) if dP.size else 0.0}
    if n_ex:
        bound = TOL_P + 10 * (sens if sens is not None else 1.0) * dg
        stats["exempt_max_dP"] = float(dP_all[exempt].max())
        assert np.all(dP_all[exempt] <= np.minimum(bound, 1.0)[exempt]), f"{label}: exempt outside bound {stats}"
    if adam:
        sm = np.maximum(np.abs(ref["m"]), (1 - beta1) * gabs)[ok]
        sv = np.maximum(np.abs(ref["v"]), (1 - beta2) * gabs * gabs)[ok]
        rm = np.abs(mg - ref["m"])[ok] / sm
        rv = np.abs(vg - ref["v"])[ok] / sv
        stats.update(max_rel_m=float(rm.max()) if rm.size else 0.0, max_rel_v=float(rv.max()) if rv.size else 0.0)
    print(label, stats)
    assert n_ex <= max(8, MAX_EXEMPT_FRAC * exempt.size), f"{label}: {stats}"
    assert stats["max_dP"] <= TOL_P, f"{label}: {stats}"
    if adam:
        assert stats["max_rel_m"] <= TOL_REL and stats["max_rel_v"] <= TOL_REL, f"{label}: {stats}"
    return stats


def compare_step(label, q, orc, g, problem, sched, S, t, K, seed, P, m, v, lanes_per_row=0):
    """Run one update on the GPU and in the oracle from the same float32 state; check it."""
    gpu = run_gpu_step(q, g, problem, sched, S, t, K, seed, P, m, v, lanes_per_row)
    og = orc.graph(W=g["dense"]) if "dense" in g else g
    ref = orc.step(oracle_params(orc, q, sched, problem), og, t, K, seed, P, m, v)
    adam = sched.rule == 0
    sens = step_sensitivity(ref, m.astype(np.float64), v.astype(np.float64), t, sched, adam)
    return check_step(label, gpu, ref, S, adam, sched.beta1, sched.beta2, sens, float(np.float32(sched.comm_alpha)))


# ---- Philox / noise / init -------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,nq,k,sid", [(0, 1, 1, 0, 0), (1234567890123, 257, 64, 7, 1),
                                               (2 ** 64 - 1, 100, 3, 2 ** 32 - 1, 1), (42, 5000, 8, 3000, 0)])
def test_philox_bit_exact(orc, seed, n, nq, k, sid):
    q = qqa()
    out = torch.zeros(n * nq * 4, dtype=torch.int32, device=dev())
    q.qqa_dev_philox(seed, n, nq, k, sid, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(n, nq, 4)
    assert np.array_equal(got, orc.philox_grid(seed, n, nq, k, sid))


@pytest.mark.parametrize("S", [1, 7, 16, 256, 1000])
def test_noise_matches_oracle(orc, S):
    q = qqa()
    n = 300
    stride = q.qqa_replica_stride(S)
    xi = torch.full((n, stride), 9.0, device=dev())
    q.qqa_dev_noise(77, n, S, 12, xi)
    torch.cuda.synchronize()
    got = xi.cpu().numpy()
    ref = orc.noise(77, n, S, 12)
    assert np.max(np.abs(got[:, :S] - ref)) < 2e-5
    assert np.all(got[:, S:] == 0)


@pytest.mark.parametrize("S", [1, 5, 16, 32, 128, 256, 1028])
def test_init_bit_exact(orc, S):
    q = qqa()
    n = 1001
    stride = q.qqa_replica_stride(S)
    P = torch.full((n, stride), -1.0, device=dev())
    m = torch.full_like(P, 3.0)
    v = torch.full_like(P, 3.0)
    q.qqa_dev_init(2024, n, S, P, m, v)
    torch.cuda.synchronize()
    got = P.cpu().numpy()
    assert np.array_equal(got[:, :S].astype(np.float64), orc.init(2024, n, S))
    assert np.all(got[:, S:] == 0) and not m.any().item() and not v.any().item()


# ---- one update --------------------------------------------------------------------------------

GRAPHS = {
    "er1000": lambda: qi.erdos_renyi(1000, 5.0, 1),
    "rrg256": lambda: qi.random_regular(256, 3, 0),
    "ba1500_pm1": lambda: qi.pm1_weights(qi.barabasi_albert(1500, 4, 2), 3),
    "er777_dense_deg": lambda: qi.erdos_renyi(777, 40.0, 4),
}


@pytest.mark.parametrize("gname,problem", [("er1000", "mis"), ("rrg256", "mis"), ("ba1500_pm1", "maxcut"),
                                            ("er777_dense_deg", "mis"), ("er1000", "maxcut")])
@pytest.mark.parametrize("S", [16, 100, 256])
@pytest.mark.parametrize("rule", ["adamw", "langevin"])
def test_step_parity_synthetic_state(orc, gname, problem, S, rule):
    q = qqa()
    g = GRAPHS[gname]()
    sched = q.schedule(problem, g["n"], rule=rule, comm_alpha=0.2)
    P, m, v = qi.synthetic_state(g["n"], S, seed=S + len(gname))
    if rule == "langevin":
        m = np.zeros_like(P)
        v = np.zeros_like(P)
    K, seed = 500, 99
    for t in (0, 7, K - 1):
        compare_step(f"{gname}/{problem}/S{S}/{rule}/t{t}", q, orc, g, problem, sched, S, t, K, seed, P, m, v)


@pytest.mark.parametrize("S", [1, 3, 7, 32, 520])
def test_step_parity_ragged_replica_counts(orc, S):
    q = qqa()
    g = qi.erdos_renyi(333, 6.0, 8)
    sched = q.schedule("mis", g["n"])
    P, m, v = qi.synthetic_state(g["n"], S, seed=S)
    compare_step(f"S{S}", q, orc, g, "mis", sched, S, 3, 10, 5, P, m, v)


@pytest.mark.parametrize("problem,gname", [("mis", "er1000"), ("maxcut", "ba1500_pm1")])
def test_step_parity_on_oracle_trajectory(orc, problem, gname):
    """States the method actually visits: the oracle's own trajectory (float64, rounded to
    float32) at early, middle and late points of the schedule."""
    q = qqa()
    g = GRAPHS[gname]()
    S, K, seed = 64, 300, 3
    sched = q.schedule(problem, g["n"])
    pr = oracle_params(orc, q, sched, problem)
    P = orc.init(seed, g["n"], S)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    t_prev = 0
    for t in (0, 40, 150, 299):
        P, m, v = orc.run(pr, g, t_prev, t, K, seed, P, m, v)
        t_prev = t
        P32, m32, v32 = (x.astype(np.float32) for x in (P, m, v))
        compare_step(f"traj/{problem}/t{t}", q, orc, g, problem, sched, S, t, K, seed, P32, m32, v32)


def test_step_edge_cases(orc):
    q = qqa()
    # no edges at all, a single variable, all replicas equal (sigma = 0)
    for g in (qi.complete_bipartite(0, 50), qi.complete_bipartite(0, 1)):
        n = g["n"]
        sched = q.schedule("mis", n)
        P = np.full((n, 8), 0.25, np.float32)
        z = np.zeros_like(P)
        compare_step(f"edge n={n}", q, orc, g, "mis", sched, 8, 0, 5, 1, P, z, z)


def test_step_is_deterministic():
    q = qqa()
    g = qi.pm1_weights(qi.barabasi_albert(3000, 4, 1), 1)
    sched = q.schedule("maxcut", g["n"])
    P, m, v = qi.synthetic_state(g["n"], 128, seed=1)
    a = run_gpu_step(q, g, "maxcut", sched, 128, 11, 100, 8, P, m, v)
    b = run_gpu_step(q, g, "maxcut", sched, 128, 11, 100, 8, P, m, v)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---- rounding + exact evaluation -----------------------------------------------------------------

def run_gpu_eval(q, g, problem, lam, P, dense=None):
    d = dev()
    S = P.shape[1]
    stride = q.qqa_replica_stride(S)
    G = q.DevGraph(dense=dense) if dense is not None else q.DevGraph(g)
    Pt = torch.as_tensor(padded(P.astype(np.float32), stride), device=d)
    a = torch.zeros(S, dtype=torch.int64, device=d)
    b = torch.zeros_like(a)
    o = torch.zeros_like(a)
    best = torch.zeros(1, dtype=torch.int32, device=d)
    q.qqa_dev_eval(G, problem, lam, S, Pt, a, b, o, best)
    torch.cuda.synchronize()
    return {"size_or_cut": a.cpu().numpy(), "viol": b.cpu().numpy(), "obj": o.cpu().numpy(),
            "best": int(best.item())}


@pytest.mark.parametrize("gname,problem", [("er1000", "mis"), ("ba1500_pm1", "maxcut"), ("rrg256", "mis"),
                                            ("er777_dense_deg", "mis")])
@pytest.mark.parametrize("S", [1, 13, 64, 256])
def test_eval_bit_exact(orc, gname, problem, S):
    q = qqa()
    g = GRAPHS[gname]()
    rng = np.random.default_rng(S)
    # values near the threshold included: 0.5 rounds to 0, the next float up to 1
    P = rng.choice(np.array([0.0, 1.0, 0.5, np.nextafter(np.float32(0.5), np.float32(1)), 0.3, 0.7], np.float32),
                   size=(g["n"], S), p=[0.3, 0.3, 0.1, 0.1, 0.1, 0.1]).astype(np.float32)
    got = run_gpu_eval(q, g, problem, 2, P)
    ref = orc.evaluate(0 if problem == "mis" else 1, 2, g, P)
    for k in ("size_or_cut", "viol", "obj"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["best"] == ref["best"]


def test_eval_dense_bit_exact(orc):
    q = qqa()
    W = qi.dense_gaussian(300, 5)
    P = (np.random.default_rng(0).random((300, 40)) > 0.5).astype(np.float32)
    got = run_gpu_eval(q, None, "maxcut", 0, P, dense=W)
    ref = orc.evaluate(1, 0, orc.graph(W=W), P)
    for k in ("size_or_cut", "viol", "obj"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["best"] == ref["best"]


# ---- full-size shapes, sampled -------------------------------------------------------------------------

@pytest.mark.parametrize("shape", ["er20000_S256_mis", "ba100000_S128_maxcut"])
def test_full_size_step_and_eval(orc, shape):
    """The sparse benchmark shapes at full size in the launch configuration the solver uses:
    one update from a synthetic state (the oracle runs the whole step) and the exact
    evaluation of the same synthetic state on both sides."""
    q = qqa()
    if shape.startswith("er"):
        g, problem, S = qi.erdos_renyi(20000, 5.0, 0), "mis", 256
    else:
        g, problem, S = qi.pm1_weights(qi.barabasi_albert(100000, 4, 0), 1), "maxcut", 128
    sched = q.schedule(problem, g["n"])
    P, m, v = qi.synthetic_state(g["n"], S, seed=5)
    K = 3000
    compare_step(shape, q, orc, g, problem, sched, S, 1234, K, 17, P, m, v)
    got = run_gpu_eval(q, g, problem, 2, P)
    ref_e = orc.evaluate(0 if problem == "mis" else 1, 2, g, P)
    for k in ("size_or_cut", "viol", "obj"):
        assert np.array_equal(got[k], ref_e[k]), k
    assert got["best"] == ref_e["best"]


@pytest.mark.parametrize("S", [4, 16, 128, 256, 600])
def test_step_parity_split_hub_rows(orc, S):
    """Rows above the split threshold (a 3000-neighbour hub, and mid-size hubs) take the
    chunked partial-sum path."""
    n = 3001
    er = qi.edge_list(qi.erdos_renyi(n, 4.0, 9))
    hub = np.stack([np.zeros(n - 1, np.int64), np.arange(1, n, dtype=np.int64)], axis=1)
    mid = np.stack([np.full(200, 7, np.int64), np.arange(1000, 1200, dtype=np.int64)], axis=1)
    e = np.concatenate([hub, mid, er])
    e = np.stack([e.min(1), e.max(1)], 1)
    e = np.unique(e, axis=0)
    e = e[e[:, 0] != e[:, 1]]
    for problem in ("mis", "maxcut"):
        g = qi.csr_from_edges(n, e, np.where(np.arange(len(e)) % 3 == 0, -1.0, 1.0).astype(np.float32)
                              if problem == "maxcut" else None)
        q = qqa()
        sched = q.schedule(problem, n)
        P, m, v = qi.synthetic_state(n, S, seed=S)
        compare_step(f"hub/{problem}/S{S}", q, orc, g, problem, sched, S, 5, 50, 3, P, m, v)


@pytest.mark.parametrize("S", [1, 3, 4, 8, 16, 32, 100, 128, 256, 1024])
@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_step_parity_every_replica_layout(orc, S, lanes):
    """Every (lanes per row, quads per lane) layout the autotuner may pick, including the
    edge-split layouts (more lanes than quads: lane slices share the row's edges)."""
    q = qqa()
    nq = (S + 3) // 4
    if nq < lanes // 2 and (nq & (nq - 1)):
        pytest.skip("layout wider than the row (edge split needs a power-of-two quad count)")
    qpl = 1
    while lanes * qpl < nq:
        qpl *= 2
    if qpl > (16 if lanes == 64 else 8):
        pytest.skip("more quads per lane than the kernels are built for")
    g = qi.pm1_weights(qi.barabasi_albert(700, 4, 3), 4)
    sched = q.schedule("maxcut", g["n"])
    P, m, v = qi.synthetic_state(g["n"], S, seed=lanes)
    compare_step(f"layout{lanes}/S{S}", q, orc, g, "maxcut", sched, S, 2, 20, 8, P, m, v, lanes)
