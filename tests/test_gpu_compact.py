"""The compact engine (one replica per variable: P, m, v as one float per variable) gives the
same bits as the whole-row streaming engine at the same lanes per row (1, or a variable's
edges split over 8 or 64 lanes), over many updates and across a resumed run: MIS and
max-cut, split (hub) rows, the Langevin rule; one update matches the oracle; a context
picks it for S = 1 and rejects it where it does not apply."""

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


def run(q, g, problem, t0, t1, K, seed, engine, lanes=0, sched=None, state=None):
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(1)
    sched = sched or q.schedule(problem, g["n"])
    if state is None:
        P0 = torch.zeros((g["n"], stride), device=d)
        m = torch.zeros_like(P0)
        v = torch.zeros_like(P0)
        q.qqa_dev_init(seed, g["n"], 1, P0, m, v)
        P = [P0, torch.full_like(P0, -1.0)]
    else:
        P, m, v = [x.clone() for x in state[0]], state[1].clone(), state[2].clone()
    q.qqa_dev_run(q.DevGraph(g), problem, sched, 1, t0, t1, K, seed, P[0], P[1], m, v, engine, lanes)
    torch.cuda.synchronize()
    return P, m, v


CASES = [
    ("rrg20000_d20_mis", lambda: qi.random_regular_swapped(20000, 20, 1), "mis"),
    ("er30000_d5_mis", lambda: qi.erdos_renyi(30000, 5.0, 2), "mis"),
    ("ba5000_maxcut_hubs", lambda: qi.pm1_weights(qi.barabasi_albert(5000, 4, 3), 3), "maxcut"),
    ("er1000_d30_maxcut_unweighted", lambda: qi.erdos_renyi(1000, 30.0, 4), "maxcut"),
]


@pytest.mark.parametrize("lanes", [1, 8, 64])
@pytest.mark.parametrize("name,make,problem", CASES, ids=[c[0] for c in CASES])
def test_compact_matches_streaming_bitwise(name, make, problem, lanes):
    q = qqa()
    g = make()
    K, seed = 300, 5
    a = run(q, g, problem, 0, 37, K, seed, "stream", lanes=lanes)
    b = run(q, g, problem, 0, 37, K, seed, "compact", lanes=lanes)
    for x, y in zip([a[0][1], a[1], a[2]], [b[0][1], b[1], b[2]]):
        assert torch.equal(x, y), name
    # resumed mid-schedule from the streamed state
    c = run(q, g, problem, 37, 60, K, seed, "compact", lanes=lanes, state=a)
    d = run(q, g, problem, 0, 60, K, seed, "stream", lanes=lanes)
    for x, y in zip([c[0][0], c[1], c[2]], [d[0][0], d[1], d[2]]):
        assert torch.equal(x, y), name


def test_compact_langevin_matches_streaming_bitwise():
    q = qqa()
    g = qi.erdos_renyi(8000, 7.0, 6)
    sched = q.schedule("mis", g["n"])
    sched.rule = q.QQA_STEP_LANGEVIN
    a = run(q, g, "mis", 0, 25, 100, 3, "stream", lanes=1, sched=sched)
    b = run(q, g, "mis", 0, 25, 100, 3, "compact", sched=sched)
    assert torch.equal(a[0][1], b[0][1])


def test_compact_one_update_matches_oracle(orc):
    from test_gpu_parity import check_step, oracle_params, step_sensitivity
    q = qqa()
    g = qi.pm1_weights(qi.barabasi_albert(3000, 4, 2), 3)
    K, seed, t = 100, 9, 17
    P, m, v = qi.synthetic_state(g["n"], 1, seed=4)
    d = torch.device("cuda")
    pad = lambda a: np.pad(a, ((0, 0), (0, 3)))
    Pt = [torch.as_tensor(pad(P), device=d), torch.full((g["n"], 4), -1.0, device=d)]
    if t % 2:
        Pt = Pt[::-1]
    mt, vt = torch.as_tensor(pad(m), device=d), torch.as_tensor(pad(v), device=d)
    sched = q.schedule("maxcut", g["n"])
    q.qqa_dev_run(q.DevGraph(g), "maxcut", sched, 1, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "compact")
    torch.cuda.synchronize()
    gpu = (Pt[(t + 1) & 1].cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy())
    ref = orc.step(oracle_params(orc, q, sched, "maxcut"), g, t, K, seed, P, m, v)
    sens = step_sensitivity(ref, m.astype(np.float64), v.astype(np.float64), t, sched, True)
    check_step("compact BA3000", gpu, ref, 1, True, sched.beta1, sched.beta2, sens, float(np.float32(sched.comm_alpha)))


def test_full_size_compact_matches_streaming_and_oracle(orc):
    """The scaling study's shape at its largest (random 20-regular graph, n = 10^6, S = 1) at
    the 4-lane edge split: 30 updates bitwise equal to the whole-row kernel's, and one update
    from a synthetic state against the oracle."""
    from test_gpu_parity import check_step, oracle_params, step_sensitivity
    q = qqa()
    g = qi.random_regular_swapped(1000000, 20, 0)
    K, seed = 3000, 2
    a = run(q, g, "mis", 0, 30, K, seed, "stream", lanes=4)
    b = run(q, g, "mis", 0, 30, K, seed, "compact", lanes=4)
    for x, y in zip([a[0][0], a[1], a[2]], [b[0][0], b[1], b[2]]):
        assert torch.equal(x, y)
    t = 2222
    P, m, v = qi.synthetic_state(g["n"], 1, seed=6)
    d = torch.device("cuda")
    pad = lambda a: np.pad(a, ((0, 0), (0, 3)))
    Pt = [torch.as_tensor(pad(P), device=d), torch.full((g["n"], 4), -1.0, device=d)]
    mt, vt = torch.as_tensor(pad(m), device=d), torch.as_tensor(pad(v), device=d)
    sched = q.schedule("mis", g["n"])
    q.qqa_dev_run(q.DevGraph(g), "mis", sched, 1, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "compact", 4)
    torch.cuda.synchronize()
    gpu = (Pt[1].cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy())
    ref = orc.step(oracle_params(orc, q, sched, "mis"), g, t, K, seed, P, m, v)
    sens = step_sensitivity(ref, m.astype(np.float64), v.astype(np.float64), t, sched, True)
    check_step("compact RRG 1e6", gpu, ref, 1, True, sched.beta1, sched.beta2, sens, float(np.float32(sched.comm_alpha)))


def test_compact_rejections():
    q = qqa()
    g = qi.erdos_renyi(500, 5.0, 0)
    d = torch.device("cuda")
    P = [torch.zeros((500, 4), device=d), torch.zeros((500, 4), device=d)]
    m, v = torch.zeros_like(P[0]), torch.zeros_like(P[0])
    with pytest.raises(q.QQAError) as e:  # two replicas
        q.qqa_dev_run(q.DevGraph(g), "mis", None, 2, 0, 3, 10, 1, P[0], P[1], m, v, "compact")
    assert e.value.code == q.QQA_E_ARG
    with pytest.raises(q.QQAError) as e:  # max clique keeps its per-replica sums on the padded layout
        q.qqa_dev_run(q.DevGraph(g), "maxclique", None, 1, 0, 3, 10, 1, P[0], P[1], m, v, "compact")
    assert e.value.code == q.QQA_E_ARG


def test_context_picks_compact_for_one_replica():
    from test_gpu_solve import objective_of
    q = qqa()
    ctx = q.Context(0)
    for (g, problem), lanes in zip([(qi.random_regular_swapped(30000, 20, 7), "mis"),
                                    (qi.pm1_weights(qi.barabasi_albert(4000, 4, 8), 8), "maxcut")], (8, 1)):
        gid = ctx.upload(g, problem)
        ctx.set_replica_layout(1, lanes)
        ctx.set_engine("auto")
        a = ctx.poll(ctx.solve_resident(gid, g["n"], problem, 1, 200, 3))
        ctx.set_engine("stream")
        b = ctx.poll(ctx.solve_resident(gid, g["n"], problem, 1, 200, 3))
        ctx.release(gid)
        assert a["engine"] == "compact" and b["engine"] == "stream" and a["kernel_us"] > 0
        assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
        assert a["best_objective"] == objective_of(g, a["best_x"], problem)
    ctx.set_replica_layout(1, 0)
    ctx.set_engine("auto")
    ctx.close()
