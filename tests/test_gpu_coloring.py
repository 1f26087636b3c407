"""Graph coloring (the categorical K-state variant) through the C ABI: one update against the
oracle from the same float32 state (several graphs, colour counts, replica counts and every
replica layout, and states on the oracle's own trajectory; shapes served by the single-launch
update and by the two-launch one), the colouring and its conflict count bit-exact against the
oracle on the same state, whole solves whose reported cost is exact for the returned
colouring, the single-launch update bitwise equal to the two-launch one over whole solves,
ten-seed quality against stored oracle results, and the argument checks."""

import json
import os

import numpy as np
import pytest

import qqa_inputs as qi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_stats.json")


def qqa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_02135_amd as q
    q.lib()
    return q


def rows(a, stride):
    """(n, K, S) -> (n*K, stride) float32, padding replicas 0"""
    n, K, S = a.shape
    out = np.zeros((n * K, stride), np.float32)
    out[:, :S] = a.reshape(n * K, S)
    return out


def run_gpu(q, g, colors, sched, S, t, K, seed, V, m, v, lanes=0):
    stride = q.qqa_replica_stride(S)
    d = torch.device("cuda")
    G = q.DevGraph(g)
    Vi = torch.as_tensor(rows(V, stride), device=d)
    Vo = torch.full_like(Vi, -7.0)
    mt = torch.as_tensor(rows(m, stride), device=d)
    vt = torch.as_tensor(rows(v, stride), device=d)
    q.qqa_dev_color_step(G, colors, sched, S, t, K, seed, Vi, Vo, mt, vt, lanes)
    torch.cuda.synchronize()
    return Vo.cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy()


def compare(label, q, orc, g, colors, S, t, K, seed, V, m, v, lanes=0):
    from test_gpu_parity import check_step, oracle_params, step_sensitivity
    sched = q.schedule("mis", g["n"])  # the schedule defaults do not depend on the problem here
    gpu = run_gpu(q, g, colors, sched, S, t, K, seed, V, m, v, lanes)
    ref = orc.cat_step(oracle_params(orc, q, sched, "mis"), g, t, K, seed, V, m, v)
    flat = {k: ref[k].reshape(-1, S) for k in ("m", "v", "pre_clamp", "g", "gabs")}
    flat["P"] = ref["V"].reshape(-1, S)
    flat["sigma"] = np.zeros(flat["P"].shape[0])
    m64, v64 = m.reshape(-1, S).astype(np.float64), v.reshape(-1, S).astype(np.float64)
    sens = step_sensitivity(flat, m64, v64, t, sched, True)
    return check_step(label, gpu, flat, S, True, sched.beta1, sched.beta2, sens)


def state(n, colors, S, seed):
    P, m, v = qi.synthetic_state(n * colors, S, seed=seed)
    return P.reshape(n, colors, S), m.reshape(n, colors, S), v.reshape(n, colors, S)


GRAPHS = {
    "queen5": lambda: qi.queens(5),
    "queen8": lambda: qi.queens(8),
    "er500": lambda: qi.erdos_renyi(500, 6.0, 1),
    "rrg200": lambda: qi.random_regular(200, 3, 2),
}


# colours 2..8 take the register-resident update kernel, more colours the three-pass one
@pytest.mark.parametrize("gname,colors,S", [("queen5", 5, 16), ("queen8", 9, 64), ("er500", 4, 32), ("er500", 3, 1),
                                            ("rrg200", 3, 256), ("queen8", 2, 100), ("queen8", 8, 40),
                                            ("queen8", 17, 40), ("er500", 31, 8)])
def test_step_parity(orc, gname, colors, S):
    q = qqa()
    g = GRAPHS[gname]()
    V, m, v = state(g["n"], colors, S, colors + S)
    for t in (0, 9, 99):
        compare(f"color {gname}/K{colors}/S{S}/t{t}", q, orc, g, colors, S, t, 100, 5, V, m, v)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_step_parity_every_layout(orc, lanes):
    q = qqa()
    g = qi.queens(6)
    V, m, v = state(g["n"], 7, 32, lanes)
    compare(f"color layout{lanes}", q, orc, g, 7, 32, 3, 50, 2, V, m, v, lanes)


def test_step_parity_on_oracle_trajectory(orc):
    from test_gpu_parity import oracle_params
    q = qqa()
    g = qi.queens(6)
    colors, S, K, seed = 7, 32, 300, 4
    sched = q.schedule("mis", g["n"])
    pr = oracle_params(orc, q, sched, "mis")
    V = orc.cat_init(seed, g["n"], colors, S)
    m = np.zeros_like(V)
    v = np.zeros_like(V)
    t_prev = 0
    for t in (1, 40, 150, 299):
        V, m, v = orc.cat_run(pr, g, t_prev, t, K, seed, V, m, v)
        t_prev = t
        compare(f"color traj t{t}", q, orc, g, colors, S, t, K, seed, *(x.astype(np.float32) for x in (V, m, v)))


@pytest.mark.parametrize("colors,S", [(5, 16), (3, 7), (11, 64)])
def test_eval_bit_exact(orc, colors, S):
    q = qqa()
    g = qi.queens(5) if colors <= 5 else qi.queens(8)
    rng = np.random.default_rng(colors)
    n = g["n"]
    V = rng.integers(0, 4, (n, colors, S)).astype(np.float32) / 3.0  # many exact ties
    stride = q.qqa_replica_stride(S)
    d = torch.device("cuda")
    X = torch.zeros((n, stride), dtype=torch.uint8, device=d)
    conf = torch.zeros(S, dtype=torch.int64, device=d)
    best = torch.zeros(1, dtype=torch.int32, device=d)
    q.qqa_dev_color_eval(q.DevGraph(g), colors, S, torch.as_tensor(rows(V, stride), device=d), X, conf, best)
    torch.cuda.synchronize()
    ref = orc.cat_eval(g, V.astype(np.float64))
    assert np.array_equal(X.cpu().numpy()[:, :S].astype(np.int32), ref["colors"])
    assert np.array_equal(conf.cpu().numpy(), ref["conflicts"])
    assert int(best.cpu()[0]) == ref["best"]


def conflicts_of(g, x):
    r = np.repeat(np.arange(g["n"]), np.diff(g["row_ptr"]))
    keep = r < g["col"]
    return int(np.sum(x[r[keep]] == x[g["col"][keep]]))


def test_solve_consistent_and_repeatable():
    q = qqa()
    g = qi.queens(6)
    ctx = q.Context(0)
    a = ctx.poll(ctx.solve_coloring(g, 7, 32, 600, 3))
    gid = ctx.upload(g, "coloring")
    b = ctx.poll(ctx.solve_coloring_resident(gid, g["n"], 7, 32, 600, 3))
    ctx.release(gid)
    ctx.close()
    assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    assert np.array_equal(a["obj"], a["size_or_cut"]) and np.array_equal(a["obj"], a["viol"])
    assert a["best_x"].max() < 7
    assert a["best_objective"] == conflicts_of(g, a["best_x"].astype(np.int64))
    assert a["best_replica"] == int(np.argmin(a["obj"]))
    assert a["engine"] == "stream"


def test_ten_seed_quality_within_oracle_spread():
    q = qqa()
    wl = json.load(open(GOLD))["workloads"].get("queen7_colors7_S32_K1000")
    if wl is None:
        pytest.skip("no stored oracle statistics for the coloring workload")
    _, board, colors, _, _, S, K = wl["recipe"]
    g = qi.queens(board)
    ctx = q.Context(0)
    gid = ctx.upload(g, "coloring")
    res = [ctx.poll(ctx.solve_coloring_resident(gid, g["n"], colors, S, K, s)) for s in range(10)]
    ctx.release(gid)
    ctx.close()
    ref_best = np.array([wl["seeds"][str(s)]["best_objective"] for s in range(10)], np.float64)
    ref_mean = np.array([wl["seeds"][str(s)]["mean_objective"] for s in range(10)], np.float64)
    best = np.array([r["best_objective"] for r in res], np.float64)
    mean = np.array([r["obj"].mean() for r in res], np.float64)
    for r in res:
        assert r["best_objective"] == conflicts_of(g, r["best_x"].astype(np.int64))
    assert ref_best.min() <= best.mean() <= ref_best.max(), (best, ref_best)
    assert ref_mean.min() <= mean.mean() <= ref_mean.max(), (mean, ref_mean)


def test_full_size_single_launch_update(orc):
    """The coloring benchmark shape (ER n = 10^5, mean degree 10, 8 colours, S = 32), which the
    single-launch update serves: one update from a synthetic state against the oracle."""
    q = qqa()
    g = qi.erdos_renyi(100000, 10.0, 0)
    V, m, v = state(g["n"], 8, 32, 13)
    compare("er1e5 K8 S32", q, orc, g, 8, 32, 456, 1000, 3, V, m, v)


def test_argument_checks():
    q = qqa()
    g = qi.queens(4)
    ctx = q.Context(0)
    for bad in (1, 256):
        with pytest.raises(q.QQAError) as e:
            ctx.solve_coloring(g, bad, 8, 10, 0)
        assert e.value.code == q.QQA_E_ARG
    with pytest.raises(q.QQAError) as e:
        ctx.solve(g, "coloring", 8, 10, 0)
    assert e.value.code == q.QQA_E_ARG
    gid = ctx.upload(g, "coloring")
    with pytest.raises(q.QQAError) as e:
        ctx.solve_batch([gid], [g["n"]], ["coloring"], [8], [10], [0])
    assert e.value.code == q.QQA_E_ARG
    ctx.release(gid)
    ctx.close()


@pytest.mark.parametrize("gname,colors,S", [("er2000", 8, 32), ("queen6", 4, 16), ("er2000", 3, 64), ("queen6", 5, 8),
                                            ("er2000", 2, 4), ("queen6", 7, 1), ("er2000d12", 8, 32)])
def test_single_launch_update_matches_two_launches_bitwise(gname, colors, S):
    """Shapes whose colours x replica quads fit a wavefront run gradient and update in one
    launch under the automatic policy; the streaming policy keeps two launches.  Mean degree
    7 takes 8-neighbour load batches, queens 6 x 6 and mean degree 12 take 16."""
    q = qqa()
    g = {"er2000": lambda: qi.erdos_renyi(2000, 7.0, 3), "er2000d12": lambda: qi.erdos_renyi(2000, 12.0, 4),
         "queen6": lambda: qi.queens(6)}[gname]()
    ctx = q.Context(0)
    gid = ctx.upload(g, "coloring")
    ctx.set_engine("auto")
    a = ctx.poll(ctx.solve_coloring_resident(gid, g["n"], colors, S, 300, 5))
    ctx.set_engine("stream")
    b = ctx.poll(ctx.solve_coloring_resident(gid, g["n"], colors, S, 300, 5))
    ctx.release(gid)
    ctx.close()
    assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    assert a["best_objective"] == conflicts_of(g, a["best_x"].astype(np.int64))
