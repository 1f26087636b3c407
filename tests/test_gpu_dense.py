"""The dense coupling path (FP32 matrix-core product + the fused update): the product
against a float64 reference of the same float32 inputs, one update against the oracle,
and whole solves whose reported objectives are exact for the returned solution."""

import json
import os

import numpy as np
import pytest

import qqa_inputs as qi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def qqa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_02135_amd as q
    q.lib()
    return q


@pytest.mark.parametrize("n,S", [(64, 16), (100, 100), (257, 33), (1024, 256), (4096, 256)])
@pytest.mark.parametrize("problem", ["maxcut", "mis"])
def test_dense_coupling_product(n, S, problem):
    q = qqa()
    d = torch.device("cuda")
    W = qi.dense_gaussian(n, n) if problem == "maxcut" else (qi.dense_gaussian(n, n) > 0.8).astype(np.float32)
    stride = q.qqa_replica_stride(S)
    P, _, _ = qi.synthetic_state(n, S, seed=n)
    Pp = np.zeros((n, stride), np.float32)
    Pp[:, :S] = P
    Ct = torch.full((n, stride), 7.0, device=d)
    q.qqa_dev_dense_coupling(torch.as_tensor(W, device=d), torch.as_tensor(Pp, device=d), Ct, n, S, problem)
    torch.cuda.synchronize()
    C = Ct.cpu().numpy()[:, :S].astype(np.float64)
    B = (2.0 * P - 1.0) if problem == "maxcut" else P.astype(np.float64)
    ref = W.astype(np.float64) @ B
    scale = np.abs(W.astype(np.float64)) @ np.abs(B)  # sum of the magnitudes of the terms
    # FP32 accumulation of n products: every element within the worst-case bound n u sum|terms|
    # (u = 2^-24); the typical error grows like sqrt(n) u, so the median must stay below it
    # (a dropped term or a misplaced operand moves most elements far above that)
    u = 2.0 ** -24
    rel = np.abs(C - ref) / (scale + 1e-30)
    assert np.all(rel <= n * u), rel.max()
    assert np.median(rel) <= np.sqrt(n) * u, np.median(rel)


@pytest.mark.parametrize("n,S", [(300, 64), (700, 100), (2048, 256)])
def test_dense_step_parity(orc, n, S):
    from test_gpu_parity import compare_step  # same tolerance contract as the sparse path
    q = qqa()
    W = qi.dense_gaussian(n, 3)
    sched = q.schedule("maxcut", n)
    P, m, v = qi.synthetic_state(n, S, seed=S)
    g = {"dense": W, "n": n}
    compare_step(f"dense{n}/S{S}", q, orc, g, "maxcut", sched, S, 5, 100, 2, P, m, v)


def test_dense_step_parity_on_oracle_trajectory(orc):
    """States the method visits: the oracle's own dense trajectory at early, middle and late
    points of the schedule, one GPU update from each."""
    from test_gpu_parity import compare_step, oracle_params
    q = qqa()
    n, S, K, seed = 256, 64, 300, 3
    W = qi.dense_gaussian(n, 5)
    g = {"dense": W, "n": n}
    sched = q.schedule("maxcut", n)
    pr = oracle_params(orc, q, sched, "maxcut")
    og = orc.graph(W=W)
    P = orc.init(seed, n, S)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    t_prev = 0
    for t in (0, 40, 150, 299):
        P, m, v = orc.run(pr, og, t_prev, t, K, seed, P, m, v)
        t_prev = t
        P32, m32, v32 = (x.astype(np.float32) for x in (P, m, v))
        compare_step(f"dense traj t{t}", q, orc, g, "maxcut", sched, S, t, K, seed, P32, m32, v32)


def objective_dense(W, x):
    q = np.rint(W.astype(np.float64) * 65536).astype(np.int64)
    diff = x[:, None] != x[None, :]
    return -int(np.sum(np.triu(q, 1)[diff[: len(x), : len(x)]]))


def test_dense_solve_consistent_and_repeatable():
    q = qqa()
    W = qi.dense_gaussian(512, 8)
    ctx = q.Context(0)
    gid = ctx.upload(None, "maxcut", dense=W)
    a = ctx.poll(ctx.solve_resident(gid, 512, "maxcut", 64, 300, 4))
    b = ctx.poll(ctx.solve_resident(gid, 512, "maxcut", 64, 300, 4))
    ctx.release(gid)
    ctx.close()
    assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    assert a["best_objective"] == objective_dense(W, a["best_x"].astype(bool))
    assert a["feasible"] and a["engine"] == "stream"


def test_dense_ten_seed_quality_within_oracle_spread():
    q = qqa()
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_stats.json")))
    wl = gold["workloads"].get("dense256_gauss_maxcut_S32_K500")
    if wl is None:
        pytest.skip("no stored oracle statistics for the dense workload")
    W = qi.dense_gaussian(256, 0)
    ctx = q.Context(0)
    gid = ctx.upload(None, "maxcut", dense=W)
    res = [ctx.poll(ctx.solve_resident(gid, 256, "maxcut", 32, 500, s)) for s in range(10)]
    ctx.release(gid)
    ctx.close()
    ref_best = np.array([wl["seeds"][str(s)]["best_objective"] for s in range(10)], np.float64)
    ref_mean = np.array([wl["seeds"][str(s)]["mean_objective"] for s in range(10)], np.float64)
    best = np.array([r["best_objective"] for r in res], np.float64)
    mean = np.array([r["obj"].mean() for r in res], np.float64)
    # small enough for the one-workgroup engine, which has no dense product: must stream
    assert all(r["engine"] == "stream" for r in res)
    assert all(r["best_objective"] == objective_dense(W, r["best_x"].astype(bool)) for r in res)
    assert ref_best.min() <= best.mean() <= ref_best.max(), (best, ref_best)
    assert ref_mean.min() <= mean.mean() <= ref_mean.max(), (mean, ref_mean)
