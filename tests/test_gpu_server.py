"""The continuous-batching server: requests submitted while others run are admitted as
slots and memory free up, every result equals the same solve run alone (bit for bit), a
tight HBM budget makes requests queue rather than fail, and oversize requests, cancellation
and draining behave as documented."""

import time

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


def mixed_requests(count, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(100, 4000))
        if k % 2:
            g, p = qi.pm1_weights(qi.barabasi_albert(n, 4, k), k), "maxcut"
        else:
            g, p = qi.erdos_renyi(n, float(rng.uniform(3, 20)), k), "mis"
        out.append((g, p, [16, 32, 128, 7][k % 4], int(rng.integers(20, 90)), 500 + k))
    return out


def test_served_results_equal_alone_and_overlap():
    q = qqa()
    reqs = mixed_requests(18)
    ctx = q.Context(0)
    ctx.serve_start(6)
    ids = []
    for i, (g, p, S, K, seed) in enumerate(reqs):
        ids.append(ctx.serve_submit(g, p, S, K, seed))
        if i % 5 == 4:
            time.sleep(0.01)  # later requests arrive while earlier ones run
    served = [ctx.poll(i) for i in ids]
    ctx.serve_stop()
    ctx.set_engine("stream")  # the whole-row engines (the automatic policy may slice from S = 128)
    for (g, p, S, K, seed), r in zip(reqs, served):
        alone = ctx.poll(ctx.solve(g, p, S, K, seed))
        assert np.array_equal(r["obj"], alone["obj"]), (g["n"], p, S, K)
        assert np.array_equal(r["best_x"], alone["best_x"])
        assert r["engine"] == "batch" and r["latency_ms"] >= r["queue_ms"] >= 0
    # with 6 slots for 18 requests some had to wait for a slot
    assert max(r["queue_ms"] for r in served) > 0
    ctx.close()


def test_requests_beyond_one_launch_wait_their_turn_and_equal_alone():
    """Five requests of 3.8 M replica-variables each are more than a round runs at once (about
    8 M per update): the ones with the least remaining work run first, the others keep their
    update index while they wait, and small requests that arrive later go ahead of them.
    Every result still equals the same solve alone."""
    q = qqa()
    big = [(qi.erdos_renyi(30000, 5.0, 40 + k), "mis", 128, K, 900 + k) for k, K in enumerate([150, 60, 120, 90, 30])]
    small = [(qi.pm1_weights(qi.barabasi_albert(2000, 4, 50 + k), k), "maxcut", 32, 40, 950 + k) for k in range(3)]
    ctx = q.Context(0)
    ctx.serve_start(16)
    ids = [ctx.serve_submit(*r) for r in big]
    time.sleep(0.005)
    ids += [ctx.serve_submit(*r) for r in small]
    served = [ctx.poll(i) for i in ids]
    ctx.serve_stop()
    ctx.set_engine("stream")  # the whole-row engines (the automatic policy may slice from S = 128)
    for (g, p, S, K, seed), r in zip(big + small, served):
        alone = ctx.poll(ctx.solve(g, p, S, K, seed))
        assert np.array_equal(r["obj"], alone["obj"]), (g["n"], p, S, K)
        assert np.array_equal(r["best_x"], alone["best_x"])
    # the shortest of the large requests finished before the longest one
    lat = [r["latency_ms"] for r in served[:5]]
    assert lat[4] < lat[0]
    ctx.close()


def test_tight_budget_queues_and_oversize_is_rejected():
    q = qqa()
    small = mixed_requests(6, seed=1)
    ctx = q.Context(0, hbm_budget=24 << 20)
    ctx.serve_start(64)
    ids = [ctx.serve_submit(g, p, S, K, seed) for g, p, S, K, seed in small]
    res = [ctx.poll(i) for i in ids]
    for (g, p, S, K, seed), r in zip(small, res):
        assert r["best_objective"] == r["obj"][r["best_replica"]]
    big = qi.erdos_renyi(60000, 5.0, 0)
    with pytest.raises(q.QQAError) as e:
        ctx.serve_submit(big, "mis", 256, 10, 0)
    assert e.value.code == q.QQA_E_ADMISSION
    ctx.serve_stop()
    ctx.close()


def test_cancel_and_drain():
    q = qqa()
    ctx = q.Context(0)
    ctx.serve_start(1)
    g = qi.erdos_renyi(3000, 5.0, 2)
    first = ctx.serve_submit(g, "mis", 64, 400, 1)
    queued = ctx.serve_submit(g, "mis", 64, 400, 2)  # waits for the single slot
    ctx.cancel(queued)
    with pytest.raises(q.QQAError) as e:
        ctx.poll(queued)
    assert e.value.code == q.QQA_E_CANCELLED
    later = ctx.serve_submit(g, "mis", 64, 50, 3)
    ctx.serve_stop()  # returns once everything submitted has finished
    assert ctx.poll(first, timeout_us=0) is not None
    assert ctx.poll(later, timeout_us=0) is not None
    ctx.close()


def test_shedding_refuses_by_projected_completion_and_admitted_equal_alone():
    """With a deadline, a burst of large requests is admitted only while the projected
    completion (the pending smaller work plus the request's own, at the measured device
    rate) stays within it; the rest are refused at submit with QQA_E_ADMISSION.  Admitted
    requests still equal their solves alone, and the counts add up."""
    q = qqa()
    ctx = q.Context(0)
    ctx.serve_start(64)
    ctx.serve_set_deadline(60.0)
    g = qi.erdos_renyi(30000, 5.0, 7)  # 3.84 M replica-variables per update at S = 128
    admitted, shed = [], 0
    for k in range(20):
        try:
            admitted.append((ctx.serve_submit(g, "mis", 128, 500, 100 + k), 100 + k))
        except q.QQAError as e:
            assert e.code == q.QQA_E_ADMISSION and "shed" in str(e)
            shed += 1
    res = [(ctx.poll(i), sd) for i, sd in admitted]
    st = ctx.serve_stats()
    ctx.serve_stop()
    assert shed > 0 and admitted
    assert st["submitted"] == 20 and st["admitted"] == len(admitted) and st["shed"] == shed
    assert st["completed"] == len(admitted) and st["rate_updates_per_s"] > 0
    ctx.set_engine("stream")  # the whole-row engines (the automatic policy may slice from S = 128)
    for r, sd in res[:3]:
        alone = ctx.poll(ctx.solve(g, "mis", 128, 500, sd))
        assert np.array_equal(r["obj"], alone["obj"]) and np.array_equal(r["best_x"], alone["best_x"])
        assert 0 <= r["queue_ms"] <= r["first_update_ms"] <= r["latency_ms"]
    # without a deadline nothing is shed
    ctx.set_engine("auto")
    ctx.serve_start(64)
    ids = [ctx.serve_submit(g, "mis", 128, 50, 300 + k) for k in range(6)]
    for i in ids:
        ctx.poll(i, want_x=False)
    st = ctx.serve_stats()
    assert st["shed"] == 0 and st["admitted"] == 6
    ctx.serve_stop()
    ctx.close()


def test_shedding_protects_admitted_requests():
    """A large request is admitted with room to spare; small requests then arrive, each of
    which alone would finish well within the deadline.  Least remaining work first runs them
    before the large one, so each delays it: once the next would push it past its deadline,
    the small ones are refused, citing the admitted request."""
    q = qqa()
    ctx = q.Context(0)
    ctx.serve_start(64)
    D = 400.0
    ctx.serve_set_deadline(D)
    R = ctx.serve_stats()["rate_updates_per_s"]  # the rate the projections use
    # few updates of many rows, so that no request's time is set by its updates alone
    stride = q.qqa_replica_stride(128)
    k_big, k_small = 1000, 500
    n_big = int(0.5 * D * 1e-3 * R / (k_big * stride))      # half the deadline
    n_small = int(0.1 * D * 1e-3 * R / (k_small * stride))  # a tenth of it each
    big = qi.erdos_renyi(n_big, 5.0, 11)
    small = qi.erdos_renyi(n_small, 5.0, 12)
    print("rate", R, "rows", n_big, n_small, flush=True)
    first = ctx.serve_submit(big, "mis", 128, k_big, 1)
    admitted, msgs = [], []
    for k in range(12):
        try:
            admitted.append(ctx.serve_submit(small, "mis", 128, k_small, 10 + k))
        except q.QQAError as e:
            assert e.code == q.QQA_E_ADMISSION
            msgs.append(str(e))
    for i in [first] + admitted:
        ctx.poll(i, want_x=False)
    ctx.serve_stop()
    ctx.close()
    # the large one leaves room for about five; every refusal protects an admitted request
    assert 2 <= len(admitted) <= 8 and msgs, (len(admitted), msgs[:1])
    assert all("admitted request" in m for m in msgs), msgs[:2]


def test_server_pool_reuses_buffers_across_many_sizes():
    """Requests of many distinct sizes one after another: the server's device pool reuses
    buffers by size class, so what it holds stays far below the sum of the requests."""
    q = qqa()
    ctx = q.Context(0)
    ctx.serve_start(8)
    total = 0
    for k in range(120):
        n = 1000 + 33 * k
        K = 20 + 3 * k
        ctx.poll(ctx.serve_submit(qi.erdos_renyi(n, 4.0, 200 + k), "mis", 32, K, k), want_x=False)
        total += 16 * n * 32 + 16 * K  # P twice, m, v and the schedule table
    st = ctx.serve_stats()
    ctx.serve_stop()
    ctx.close()
    print("held", st["device_bytes_held"], "cached", st["device_bytes_cached"], "sum", total)
    assert st["device_bytes_held"] < total / 4
