"""Max clique (appendix energy with the per-replica sum 1^T p): the fixed-point replica sums
bit-exact against an integer reference, one update against the oracle (sparse, split rows,
dense), one update from states on the oracle's own trajectory, whole solves whose reported
objectives are exact for the returned solution, ten-seed quality against stored oracle
results, and the forms that refuse max clique."""

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


def adjacency(g):
    n = g["n"]
    A = np.zeros((n, n), np.int8)
    rows = np.repeat(np.arange(n), np.diff(g["row_ptr"]))
    A[rows, g["col"]] = 1
    return A


def clique_objective(A, x, lam=2):
    """l(x) from its definition: -|x| + lambda * #(selected pairs that are not adjacent)."""
    sel = np.nonzero(x)[0]
    sub = A[np.ix_(sel, sel)]
    k = len(sel)
    nonadj = (k * (k - 1) - int(sub.sum())) // 2
    return -k + lam * nonadj, nonadj


@pytest.mark.parametrize("n,S", [(1, 1), (7, 3), (100, 33), (20000, 256), (600, 4096)])
def test_replica_sums_bit_exact(n, S):
    q = qqa()
    stride = q.qqa_replica_stride(S)
    rng = np.random.default_rng(n + S)
    P = np.zeros((n, stride), np.float32)
    P[:, :S] = rng.random((n, S), dtype=np.float32)
    P[: n // 5, : S // 2] = 1.0  # exact ones and tiny values too
    P[n // 5: n // 4, :S] = rng.random((n // 4 - n // 5, S), dtype=np.float32) * 1e-6
    ref = np.rint(P.astype(np.float64) * 2.0 ** 32).astype(np.uint64).sum(axis=0)
    T = torch.full((stride,), 12345, dtype=torch.int64, device="cuda")
    q.qqa_dev_replica_sums(torch.as_tensor(P, device="cuda"), n, S, T)
    torch.cuda.synchronize()
    got = T.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref)


GRAPHS = {
    "er300": lambda: qi.erdos_renyi(300, 6.0, 1),
    "rb20x12": lambda: qi.rb_model(20, 12, 2.6, 0.25, 0),   # degrees 160-212: split rows
    "er5000": lambda: qi.erdos_renyi(5000, 5.0, 2),
}


@pytest.mark.parametrize("gname,S", [("er300", 64), ("rb20x12", 32), ("er5000", 256), ("rb20x12", 100)])
def test_step_parity(orc, gname, S):
    from test_gpu_parity import compare_step
    q = qqa()
    g = GRAPHS[gname]()
    sched = q.schedule("maxclique", g["n"])
    P, m, v = qi.synthetic_state(g["n"], S, seed=S)
    for t in (0, 7, 99):
        compare_step(f"clique {gname}/S{S}/t{t}", q, orc, g, "maxclique", sched, S, t, 100, 3, P, m, v)


def test_dense_step_parity(orc):
    from test_gpu_parity import compare_step
    q = qqa()
    g = qi.rb_model(16, 10, 2.6, 0.25, 3)
    W = adjacency(g).astype(np.float32)
    sched = q.schedule("maxclique", g["n"])
    P, m, v = qi.synthetic_state(g["n"], 64, seed=4)
    compare_step("clique dense", q, orc, {"dense": W, "n": g["n"]}, "maxclique", sched, 64, 5, 100, 2, P, m, v)


def test_step_parity_on_oracle_trajectory(orc):
    from test_gpu_parity import compare_step, oracle_params
    q = qqa()
    g = qi.rb_model(20, 12, 2.6, 0.25, 0)
    S, K, seed = 32, 300, 3
    sched = q.schedule("maxclique", g["n"])
    pr = oracle_params(orc, q, sched, "maxclique")
    P = orc.init(seed, g["n"], S)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    t_prev = 0
    for t in (0, 40, 150, 299):
        P, m, v = orc.run(pr, g, t_prev, t, K, seed, P, m, v)
        t_prev = t
        P32, m32, v32 = (x.astype(np.float32) for x in (P, m, v))
        compare_step(f"clique traj t{t}", q, orc, g, "maxclique", sched, S, t, K, seed, P32, m32, v32)


def test_solve_consistent_and_repeatable():
    q = qqa()
    g = qi.rb_model(20, 12, 2.6, 0.25, 5)
    A = adjacency(g)
    ctx = q.Context(0)
    gid = ctx.upload(g, "maxclique")
    a = ctx.poll(ctx.solve_resident(gid, g["n"], "maxclique", 64, 500, 4))
    b = ctx.poll(ctx.solve_resident(gid, g["n"], "maxclique", 64, 500, 4))
    ctx.release(gid)
    ctx.close()
    assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    assert np.array_equal(a["obj"], -a["size_or_cut"] + 2 * a["viol"])
    obj, nonadj = clique_objective(A, a["best_x"].astype(bool))
    assert a["best_objective"] == obj and a["best_violations"] == nonadj
    assert a["engine"] == "stream"
    assert a["feasible"] and a["best_size_or_cut"] >= 15  # planted clique: 20


def _clique_states(g, S, seed):
    """Rounding-threshold values (exactly 1/2 rounds to 0, the next float up to 1), planted
    cliques (feasible replicas), and duplicated replicas (tied objectives, which the lowest
    index breaks)."""
    rng = np.random.default_rng(seed)
    n = g["n"]
    half_up = np.nextafter(np.float32(0.5), np.float32(1))
    vals = np.array([0.0, 1.0, 0.5, half_up, 0.2, 0.9], np.float32)
    P = rng.choice(vals, size=(n, S), p=[0.55, 0.15, 0.1, 0.1, 0.05, 0.05]).astype(np.float32)
    A = adjacency(g)
    for s in range(0, S, 3):  # a greedy clique from a random start: no violations
        P[:, s] = 0.0
        order = rng.permutation(n)
        chosen = []
        for i in order[: min(n, 64)]:
            if all(A[i, j] for j in chosen):
                chosen.append(i)
        P[chosen, s] = rng.choice(np.array([1.0, half_up], np.float32), size=len(chosen))
        if s + 1 < S:
            P[:, s + 1] = P[:, s]  # the same rounded solution: tied (violations, objective)
    return P


@pytest.mark.parametrize("gname", ["er300", "rb20x12"])
@pytest.mark.parametrize("S", [1, 13, 64, 1000])
def test_eval_bit_exact_against_oracle(orc, gname, S):
    """Rounding and exact evaluation of max clique (selected pairs that are not adjacent,
    l = -size + lambda * violations, the lexicographic best replica) against the oracle's,
    every replica compared."""
    q = qqa()
    g = {"er300": lambda: qi.erdos_renyi(300, 60.0, 11), "rb20x12": lambda: qi.rb_model(20, 12, 2.6, 0.25, 0)}[gname]()
    stride = q.qqa_replica_stride(S)
    P = _clique_states(g, S, seed=S)
    Pp = np.zeros((g["n"], stride), np.float32)
    Pp[:, :S] = P
    d = torch.device("cuda")
    out = [torch.full((S,), -99, dtype=torch.int64, device=d) for _ in range(3)]
    best = torch.full((1,), -5, dtype=torch.int32, device=d)
    q.qqa_dev_eval(q.DevGraph(g), "maxclique", 2, S, torch.as_tensor(Pp, device=d), *out, best)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in out]
    ref = orc.evaluate(2, 2, g, P)
    for k, a in zip(("size_or_cut", "viol", "obj"), got):
        assert np.array_equal(a, ref[k]), k
    assert int(best.item()) == ref["best"]
    assert ref["viol"].min() == 0  # feasible replicas exist, so the best is a clique
    if S > 1:
        # the duplicated replicas tie, and the lower index is the one reported
        b = ref["best"]
        assert not (b % 3 == 1 and ref["obj"][b - 1] == ref["obj"][b] and ref["viol"][b - 1] == ref["viol"][b])


def test_ten_seed_quality_within_oracle_spread():
    q = qqa()
    wl = json.load(open(GOLD))["workloads"].get("rb20x12_maxclique_S32_K1000")
    if wl is None:
        pytest.skip("no stored oracle statistics for the max-clique workload")
    n_vars, d, r, p, gseed = wl["recipe"][1:6]
    g = qi.rb_model(n_vars, d, r, p, gseed)
    ctx = q.Context(0)
    gid = ctx.upload(g, "maxclique")
    res = [ctx.poll(ctx.solve_resident(gid, g["n"], "maxclique", 32, 1000, s)) for s in range(10)]
    ctx.release(gid)
    ctx.close()
    ref_best = np.array([wl["seeds"][str(s)]["best_objective"] for s in range(10)], np.float64)
    ref_mean = np.array([wl["seeds"][str(s)]["mean_objective"] for s in range(10)], np.float64)
    best = np.array([r["best_objective"] for r in res], np.float64)
    mean = np.array([r["obj"].mean() for r in res], np.float64)
    assert ref_best.min() <= best.mean() <= ref_best.max(), (best, ref_best)
    assert ref_mean.min() <= mean.mean() <= ref_mean.max(), (mean, ref_mean)


def test_forms_that_refuse_max_clique():
    q = qqa()
    g = qi.rb_model(10, 6, 2.6, 0.25, 1)
    ctx = q.Context(0)
    gid = ctx.upload(g, "maxclique")
    with pytest.raises(q.QQAError) as e:
        ctx.solve_batch([gid], [g["n"]], ["maxclique"], [8], [10], [0])
    assert e.value.code == q.QQA_E_ARG
    ctx.release(gid)
    ctx.close()
