"""Kernels with the default schedule's facts fixed at compile time (problem, AdamW, entropy
power 4) and the generic kernels give the same bits: every engine that has both runs here
with default and non-default schedules (Langevin, entropy power 2 and 6) and is compared with
the streaming engine, which is always generic."""

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


SCHEDULES = [{}, {"rule": "langevin"}, {"entropy_alpha": 2}, {"entropy_alpha": 6}]


def _solve(ctx, engine, gid, n, problem, S, K, seed, sched):
    ctx.set_engine(engine)
    r = ctx.poll(ctx.solve_resident(gid, n, problem, S, K, seed, sched))
    return r


@pytest.mark.parametrize("over", SCHEDULES, ids=["default", "langevin", "alpha2", "alpha6"])
def test_lds_block_facts_and_generic_equal_streaming(over):
    q = qqa()
    ctx = q.Context(0)
    cases = [(qi.random_regular(256, 3, 0), "mis", 16), (qi.pm1_weights(qi.erdos_renyi(300, 6.0, 1), 2), "maxcut", 32)]
    for g, problem, S in cases:
        gid = ctx.upload(g, problem)
        sched = q.schedule(problem, g["n"], **over)
        a = _solve(ctx, "auto", gid, g["n"], problem, S, 300, 5, sched)
        b = _solve(ctx, "stream", gid, g["n"], problem, S, 300, 5, sched)
        ctx.release(gid)
        assert a["engine"] == "lds_block" and b["engine"] == "stream"
        assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"]), (problem, over)
    ctx.close()


@pytest.mark.parametrize("over", SCHEDULES, ids=["default", "langevin", "alpha2", "alpha6"])
def test_resident_batch_facts_and_generic_equal_slots(over):
    # a batch whose instances share the default schedule runs the fixed-facts resident and
    # slot kernels; a mixed batch (every other instance on the other schedule) the generic ones
    q = qqa()
    ctx = q.Context(0)
    gs = qi.instance_batch(24, 3, n_range=(200, 1500), deg_range=(3.0, 12.0))
    gids = [ctx.upload(g, "mis") for g in gs]
    ns = [g["n"] for g in gs]
    for mixed in (False, True):
        sch = [q.schedule("mis", n, **(over if (not mixed or i % 2 == 0) else {})) for i, n in enumerate(ns)]
        res = {}
        for engine in ("auto", "stream"):
            ctx.set_engine(engine)
            ids = ctx.solve_batch(gids, ns, ["mis"] * len(gs), [32] * len(gs), [200] * len(gs), list(range(len(gs))), sch)
            res[engine] = [ctx.poll(i) for i in ids]
        assert res["auto"][0]["engine"] == "batch_resident" and res["stream"][0]["engine"] != "batch_resident"
        for a, b in zip(res["auto"], res["stream"]):
            assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"]), (mixed, over)
    for gid in gids:
        ctx.release(gid)
    ctx.close()


@pytest.mark.parametrize("over", SCHEDULES, ids=["default", "langevin", "alpha2", "alpha6"])
def test_sliced_slice_major_facts_and_generic_equal_row_major(over):
    # a context's sliced solve keeps its state slice-major and runs the fixed-facts kernel for
    # the default schedule (the generic slice-major kernel otherwise); the per-stage path runs
    # the generic row-major kernel on the same seed and schedule: same bits
    q = qqa()
    for g, problem, S in [(qi.erdos_renyi(20000, 5.0, 0), "mis", 256),
                          (qi.pm1_weights(qi.barabasi_albert(20000, 4, 5), 3), "maxcut", 128)]:
        n, K, seed = g["n"], 60, 3
        sched = q.schedule(problem, n, **over)
        ctx = q.Context(0)
        gid = ctx.upload(g, problem)
        r = _solve(ctx, "sliced", gid, n, problem, S, K, seed, sched)
        ctx.release(gid)
        ctx.close()
        assert r["engine"] == "sliced"
        d = torch.device("cuda")
        stride = q.qqa_replica_stride(S)
        P = [torch.zeros((n, stride), device=d), torch.full((n, stride), -1.0, device=d)]
        m = torch.zeros_like(P[0])
        v = torch.zeros_like(P[0])
        q.qqa_dev_init(seed, n, S, P[0], m, v)
        q.qqa_dev_run(q.DevGraph(g), problem, sched, S, 0, K, K, seed, P[0], P[1], m, v, "sliced")
        out = [torch.zeros((S,), dtype=torch.int64, device=d) for _ in range(3)]
        best = torch.zeros((1,), dtype=torch.int32, device=d)
        q.qqa_dev_eval(q.DevGraph(g), problem, sched.penalty_lambda, S, P[K & 1], *out, best)
        torch.cuda.synchronize()
        assert np.array_equal(r["obj"], out[2].cpu().numpy()), (problem, over)
        assert r["best_replica"] == int(best.item())
        x = (P[K & 1][:, r["best_replica"]] > 0.5).to(torch.uint8).cpu().numpy()
        assert np.array_equal(r["best_x"], x)
