"""The sliced streaming engine (replica axis cut into 8 slices, one per XCD; row statistics
computed by a launch of their own) gives the same bits as the whole-row streaming engine
over many updates: full and ragged slices, the smallest and largest slice widths, split
(hub) rows, max-cut weights, max clique's per-replica sums, the Langevin rule and
non-default lane layouts.  One update matches the oracle, and a context runs it by policy."""

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


def run(q, g, problem, S, t0, t1, K, seed, engine, lanes=0, sched=None, state=None):
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(S)
    sched = sched or q.schedule(problem, g["n"])
    if state is None:
        P0 = torch.zeros((g["n"], stride), device=d)
        m = torch.zeros_like(P0)
        v = torch.zeros_like(P0)
        q.qqa_dev_init(seed, g["n"], S, P0, m, v)
        P = [P0, torch.full_like(P0, -1.0)]
    else:
        P, m, v = [x.clone() for x in state[0]], state[1].clone(), state[2].clone()
    q.qqa_dev_run(q.DevGraph(g), problem, sched, S, t0, t1, K, seed, P[0], P[1], m, v, engine, lanes)
    torch.cuda.synchronize()
    return P, m, v


def rb_graph():
    return qi.rb_model(20, 12, 2.6, 0.25, 0)  # degrees 160-212: split rows


CASES = [
    # name, graph, problem, S, lanes (both engines)
    ("er20000_S256_mis", lambda: qi.erdos_renyi(20000, 5.0, 0), "mis", 256, 0),
    ("er20000_S256_mis_lanes32", lambda: qi.erdos_renyi(20000, 5.0, 0), "mis", 256, 32),
    ("ba5000_S128_maxcut_hubs", lambda: qi.pm1_weights(qi.barabasi_albert(5000, 4, 1), 1), "maxcut", 128, 0),
    ("er4000_S100_mis_ragged", lambda: qi.erdos_renyi(4000, 8.0, 2), "mis", 100, 0),
    ("er4000_S61_mis_narrowest", lambda: qi.erdos_renyi(4000, 8.0, 3), "mis", 61, 0),
    ("er3000_S1000_maxcut", lambda: qi.pm1_weights(qi.erdos_renyi(3000, 6.0, 4), 2), "maxcut", 1000, 0),
    ("rrg2000_S4096_mis_widest", lambda: qi.random_regular(2000, 3, 5), "mis", 4096, 0),
    ("rb_S64_maxclique", rb_graph, "maxclique", 64, 0),
]


@pytest.mark.parametrize("name,make,problem,S,lanes", CASES, ids=[c[0] for c in CASES])
def test_sliced_matches_streaming_bitwise(name, make, problem, S, lanes):
    q = qqa()
    g = make()
    K, seed = 200, 7
    a = run(q, g, problem, S, 0, 23, K, seed, "stream", lanes)
    b = run(q, g, problem, S, 0, 23, K, seed, "sliced", lanes)
    for x, y in zip([a[0][1], a[1], a[2]], [b[0][1], b[1], b[2]]):
        assert torch.equal(x, y), name
    # resumed mid-schedule from the streamed state
    c = run(q, g, problem, S, 23, 40, K, seed, "sliced", lanes, state=a)
    d = run(q, g, problem, S, 0, 40, K, seed, "stream", lanes)
    for x, y in zip([c[0][0], c[1], c[2]], [d[0][0], d[1], d[2]]):
        assert torch.equal(x, y), name


def test_sliced_langevin_matches_streaming_bitwise():
    q = qqa()
    g = qi.erdos_renyi(5000, 6.0, 8)
    sched = q.schedule("mis", g["n"])
    sched.rule = q.QQA_STEP_LANGEVIN
    a = run(q, g, "mis", 160, 0, 15, 100, 3, "stream", sched=sched)
    b = run(q, g, "mis", 160, 0, 15, 100, 3, "sliced", sched=sched)
    assert torch.equal(a[0][1], b[0][1])


def test_sliced_one_update_matches_oracle(orc):
    from test_gpu_parity import check_step, oracle_params, step_sensitivity
    q = qqa()
    g = qi.pm1_weights(qi.barabasi_albert(3000, 4, 2), 3)
    S, K, seed, t = 200, 100, 9, 17
    P, m, v = qi.synthetic_state(g["n"], S, seed=4)
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(S)
    pad = lambda a: np.pad(a, ((0, 0), (0, stride - S)))
    Pt = [torch.as_tensor(pad(P), device=d), torch.full((g["n"], stride), -1.0, device=d)]
    if t % 2:
        Pt = Pt[::-1]
    mt, vt = torch.as_tensor(pad(m), device=d), torch.as_tensor(pad(v), device=d)
    sched = q.schedule("maxcut", g["n"])
    q.qqa_dev_run(q.DevGraph(g), "maxcut", sched, S, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "sliced")
    torch.cuda.synchronize()
    gpu = (Pt[(t + 1) & 1].cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy())
    ref = orc.step(oracle_params(orc, q, sched, "maxcut"), g, t, K, seed, P, m, v)
    m64, v64 = m.astype(np.float64), v.astype(np.float64)
    sens = step_sensitivity(ref, m64, v64, t, sched, True)
    check_step("sliced BA3000 S200", gpu, ref, S, True, sched.beta1, sched.beta2, sens)


def test_sliced_rejects_narrow_replica_counts():
    q = qqa()
    with pytest.raises(q.QQAError) as e:
        run(q, qi.erdos_renyi(500, 5.0, 0), "mis", 60, 0, 3, 10, 1, "sliced")  # 15 quads: < 2 per slice
    assert e.value.code == q.QQA_E_ARG


def test_context_sliced_policy_same_results():
    q = qqa()
    ctx = q.Context(0)
    for g, problem, S in [(qi.pm1_weights(qi.barabasi_albert(6000, 4, 1), 1), "maxcut", 128),
                          (qi.erdos_renyi(20000, 5.0, 0), "mis", 256),
                          (rb_graph(), "maxclique", 96)]:
        gid = ctx.upload(g, problem)
        ctx.set_engine("sliced")
        a = ctx.poll(ctx.solve_resident(gid, g["n"], problem, S, 150, 3))
        ctx.set_engine("stream")
        b = ctx.poll(ctx.solve_resident(gid, g["n"], problem, S, 150, 3))
        ctx.release(gid)
        assert a["engine"] == "sliced" and b["engine"] == "stream"
        assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
        assert a["kernel_us"] > 0
    # automatic policy: sliced for few rows with many replicas, else whole rows
    ctx.set_engine("auto")
    for g, S, engine in [(qi.erdos_renyi(1000, 8.0, 1), 1000, "sliced"), (qi.erdos_renyi(1000, 8.0, 1), 256, "stream"),
                         (qi.erdos_renyi(2000, 8.0, 1), 1000, "stream")]:
        gid = ctx.upload(g, "mis")
        assert ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, 50, 1))["engine"] == engine
        ctx.release(gid)
    ctx.close()
