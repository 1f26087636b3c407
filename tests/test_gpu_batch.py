"""Ragged multi-instance batches through qqa_solve_batch: every instance's result is the
same, bit for bit, as the same solve submitted alone on the whole-row engines, and is
self-consistent."""

import numpy as np
import pytest

import qqa_inputs as qi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_02135_amd as q
    c = q.Context(0)
    yield c
    c.close()


def _instances():
    rng = np.random.default_rng(0)
    out = []
    for k in range(14):
        n = int(rng.integers(50, 3000))
        if k % 3 == 2:
            g = qi.pm1_weights(qi.barabasi_albert(n, 4, k), k)  # split hub rows for the larger ones
            problem = "maxcut"
        else:
            g = qi.erdos_renyi(n, float(rng.uniform(3, 20)), k)
            problem = "mis"
        S = [16, 32, 32, 128, 7, 256][k % 6]
        K = int(rng.integers(40, 160))
        out.append((g, problem, S, K, 100 + k))
    return out


def test_batch_equals_alone_bitwise(ctx):
    inst = _instances()
    gids = [ctx.upload(g, p) for g, p, S, K, seed in inst]
    ids = ctx.solve_batch(gids, [g["n"] for g, *_ in inst], [p for _, p, *_ in inst], [i[2] for i in inst],
                          [i[3] for i in inst], [i[4] for i in inst])
    batched = [ctx.poll(i) for i in ids]
    for (g, p, S, K, seed), gid, b in zip(inst, gids, batched):
        # the sliced engine (automatic from S = 128) rounds the replica statistics differently
        ctx.set_engine("stream")
        alone = ctx.poll(ctx.solve_resident(gid, g["n"], p, S, K, seed))
        assert np.array_equal(b["obj"], alone["obj"]), (g["n"], p, S, K)
        assert np.array_equal(b["size_or_cut"], alone["size_or_cut"])
        assert np.array_equal(b["best_x"], alone["best_x"])
        assert b["best_replica"] == alone["best_replica"]
        assert b["step_loop_ms"] > 0
    ctx.set_engine("auto")
    for gid in gids:
        ctx.release(gid)


def test_batch_of_one_and_repeat(ctx):
    g = qi.erdos_renyi(800, 6.0, 3)
    gid = ctx.upload(g, "mis")
    a = ctx.poll(ctx.solve_batch([gid], [g["n"]], ["mis"], [64], [120], [9])[0])
    b = ctx.poll(ctx.solve_batch([gid, gid], [g["n"]] * 2, ["mis"] * 2, [64, 64], [120, 120], [9, 10])[0])
    ctx.release(gid)
    assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])


def test_batch_rejects_bad_arguments(ctx):
    import paper_2409_02135_amd as q
    g = qi.erdos_renyi(100, 3.0, 1)
    gid = ctx.upload(g, "mis")
    with pytest.raises(q.QQAError) as e:
        ctx.solve_batch([gid], [100], ["maxcut"], [16], [10], [0])
    assert e.value.code == q.QQA_E_ARG
    with pytest.raises(q.QQAError) as e:
        ctx.solve_batch([gid, 999], [100, 100], ["mis", "mis"], [16, 16], [10, 10], [0, 1])
    assert e.value.code == q.QQA_E_ARG
    ctx.release(gid)


def test_batch_equals_alone_with_edge_split_layouts():
    """Layouts with more lanes than a row has quads split each row's edges between lane
    slices; the batch runs them with the same row functions, so results stay identical."""
    import paper_2409_02135_amd as q
    c = q.Context(0)
    for S, lanes in ((1, 8), (4, 16), (32, 64)):
        c.set_replica_layout(S, lanes)
    inst = [(qi.erdos_renyi(900, 12.0, 21), 1, 200, 5), (qi.random_regular_swapped(600, 20, 22), 4, 150, 6),
            (qi.erdos_renyi(1500, 6.0, 23), 32, 120, 7)]
    gids = [c.upload(g, "mis") for g, *_ in inst]
    ids = c.solve_batch(gids, [g["n"] for g, *_ in inst], ["mis"] * 3, [i[1] for i in inst], [i[2] for i in inst],
                        [i[3] for i in inst])
    batched = [c.poll(i) for i in ids]
    for (g, S, K, seed), gid, b in zip(inst, gids, batched):
        alone = c.poll(c.solve_resident(gid, g["n"], "mis", S, K, seed))
        assert np.array_equal(b["obj"], alone["obj"]) and np.array_equal(b["best_x"], alone["best_x"]), S
    for gid in gids:
        c.release(gid)
    c.close()


def _one_width(count, S, seed, n_range=(30, 5000)):
    """`count` ER instances with ragged n, mean degree and update counts, MIS and +-1 max-cut;
    every row below the split threshold, so one replica layout serves all of them."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(*n_range))
        g = qi.erdos_renyi(n, float(rng.uniform(3, 20)), seed * 1000 + k)
        problem = "maxcut" if k % 3 == 1 else "mis"
        if problem == "maxcut":
            g = qi.pm1_weights(g, k)
        out.append((g, problem, S, int(rng.integers(30, 200)), 500 + k))
    return out


def _run_batch(c, inst):
    gids = [c.upload(g, p) for g, p, *_ in inst]
    ids = c.solve_batch(gids, [g["n"] for g, *_ in inst], [p for _, p, *_ in inst], [i[2] for i in inst],
                        [i[3] for i in inst], [i[4] for i in inst])
    return gids, [c.poll(i) for i in ids]


def _check_alone(c, inst, gids, batched):
    c.set_engine("stream")  # the whole-row engines (the automatic policy may slice from S = 128)
    for (g, p, S, K, seed), gid, b in zip(inst, gids, batched):
        alone = c.poll(c.solve_resident(gid, g["n"], p, S, K, seed))
        assert np.array_equal(b["obj"], alone["obj"]), (g["n"], p, S, K)
        assert np.array_equal(b["size_or_cut"], alone["size_or_cut"])
        assert np.array_equal(b["viol"], alone["viol"])
        assert np.array_equal(b["best_x"], alone["best_x"])
        assert b["best_replica"] == alone["best_replica"]
    c.set_engine("auto")
    for gid in gids:
        c.release(gid)


@pytest.mark.parametrize("S", [32, 16, 128])
def test_resident_batch_equals_alone_bitwise(ctx, S):
    """One layout, one quad per lane, no split rows: the whole batch runs in one resident
    launch (teams of workgroups on one XCD, state in registers, P through the XCD's L2), and
    every instance ends with the bits of its solve alone."""
    # at 128 replicas a lane group holds three rows of 32 lanes: about 3,000 rows fit one XCD
    inst = _one_width(40 if S == 32 else 12, S, S, n_range=(30, 2000) if S == 128 else (30, 5000))
    gids, batched = _run_batch(ctx, inst)
    assert all(b["engine"] == "batch_resident" for b in batched), batched[0]["engine"]
    print("S", S, "update loop ms", batched[0]["step_loop_ms"], flush=True)
    _check_alone(ctx, inst, gids, batched)


def test_resident_batch_repeatable_and_policy_fallbacks(ctx):
    inst = _one_width(10, 32, 7)
    gids, a = _run_batch(ctx, inst)
    gb, b = _run_batch(ctx, inst)
    for x, y in zip(a, b):
        assert np.array_equal(x["obj"], y["obj"]) and np.array_equal(x["best_x"], y["best_x"])
    # the slot launches give the same bits
    ctx.set_engine("stream")
    gs, s = _run_batch(ctx, inst)
    ctx.set_engine("auto")
    for gid in gb + gs:
        ctx.release(gid)
    assert all(r["engine"] == "batch" for r in s)
    for x, y in zip(a, s):
        assert np.array_equal(x["obj"], y["obj"]) and np.array_equal(x["best_x"], y["best_x"])
    for gid in gids:
        ctx.release(gid)
    # split rows, several layouts, or an instance beyond one XCD's registers: slot launches
    hub = [(qi.pm1_weights(qi.barabasi_albert(3000, 4, 1), 2), "maxcut", 32, 40, 1)] + _one_width(3, 32, 8)
    mixed = _one_width(3, 32, 9) + _one_width(3, 16, 10)
    big = [(qi.erdos_renyi(20000, 4.0, 11), "mis", 32, 30, 3)] + _one_width(2, 32, 12)
    for inst in (hub, mixed, big):
        gids, res = _run_batch(ctx, inst)
        assert all(r["engine"] == "batch" for r in res)
        _check_alone(ctx, inst, gids, res)


def test_batch_autotune_keeps_results_and_applies_its_choice():
    """The batch autotuner times every replica layout on the slot launches and, for a batch of
    one layout class, the resident engine; later batches run what it kept, and every instance
    still ends with the bits of its solve alone under the same layout."""
    import paper_2409_02135_amd as q
    c = q.Context(0)
    try:
        inst = _one_width(24, 32, 31)
        gids = [c.upload(g, p) for g, p, *_ in inst]
        resident, lanes = c.autotune_batch(gids, [p for _, p, *_ in inst], [32] * len(inst), [i[3] for i in inst])
        print("resident", resident, "lanes", lanes[0], flush=True)
        assert len(set(lanes)) == 1 and lanes[0] in (1, 2, 4, 8, 16, 32, 64)
        assert not resident or lanes[0] == 8  # the resident engine runs one quad per lane
        ids = c.solve_batch(gids, [g["n"] for g, *_ in inst], [p for _, p, *_ in inst], [32] * len(inst),
                            [i[3] for i in inst], [i[4] for i in inst])
        res = [c.poll(i) for i in ids]
        assert all(r["engine"] == ("batch_resident" if resident else "batch") for r in res)
        _check_alone(c, inst, gids, res)
        # two replica counts: a layout per S on the slot launches, never the resident engine
        mixed = _one_width(4, 32, 32) + _one_width(4, 128, 33, n_range=(30, 2000))
        gids = [c.upload(g, p) for g, p, *_ in mixed]
        resident, lanes = c.autotune_batch(gids, [p for _, p, *_ in mixed], [i[2] for i in mixed],
                                           [i[3] for i in mixed])
        assert not resident and len(set(lanes[:4])) == 1 and len(set(lanes[4:])) == 1
        ids = c.solve_batch(gids, [g["n"] for g, *_ in mixed], [p for _, p, *_ in mixed], [i[2] for i in mixed],
                            [i[3] for i in mixed], [i[4] for i in mixed])
        res = [c.poll(i) for i in ids]
        assert all(r["engine"] == "batch" for r in res)
        _check_alone(c, mixed, gids, res)
        # refused under a forced single-solve engine
        g = qi.erdos_renyi(100, 3.0, 1)
        gid = c.upload(g, "mis")
        c.set_engine("sliced")
        with pytest.raises(q.QQAError) as e:
            c.autotune_batch([gid], ["mis"], [32], [10])
        assert e.value.code == q.QQA_E_ARG
        c.set_engine("auto")
        c.release(gid)
    finally:
        c.close()
