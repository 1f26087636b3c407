"""The persistent engines (state resident in registers across a grid barrier, or P in the
LDS of one workgroup) give the same bits as the streaming engine over many updates, and
one update matches the oracle."""

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


def run(q, g, problem, S, t0, t1, K, seed, engine, state=None):
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(S)
    G = q.DevGraph(g)
    if state is None:
        P0 = torch.zeros((g["n"], stride), device=d)
        m = torch.zeros_like(P0)
        v = torch.zeros_like(P0)
        q.qqa_dev_init(seed, g["n"], S, P0, m, v)
        P1 = torch.full_like(P0, -1.0)
        P = [P0, P1]
    else:
        P, m, v = [x.clone() for x in state[0]], state[1].clone(), state[2].clone()
    q.qqa_dev_run(G, problem, q.schedule(problem, g["n"]), S, t0, t1, K, seed, P[0], P[1], m, v, engine)
    torch.cuda.synchronize()
    return P, m, v


CASES = [
    ("rrg256_S16_mis", lambda: qi.random_regular(256, 3, 0), "mis", 16, "lds_block"),
    ("er300_S32_maxcut", lambda: qi.pm1_weights(qi.erdos_renyi(300, 6.0, 1), 2), "maxcut", 32, "lds_block"),
    # 30,946 column indices (121 KB) do not fit in LDS beside P (128 KB): the gathers read them
    # from global memory (degrees at most 49: no split rows)
    ("er1024_d30_S16_mis", lambda: qi.erdos_renyi(1024, 30.0, 4), "mis", 16, "lds_block"),
    ("er3000_S64_mis", lambda: qi.erdos_renyi(3000, 5.0, 2), "mis", 64, "persistent"),
    ("er6000_S128_maxcut", lambda: qi.pm1_weights(qi.erdos_renyi(6000, 5.0, 3), 4), "maxcut", 128, "persistent"),
    ("er20000_S256_mis", lambda: qi.erdos_renyi(20000, 5.0, 0), "mis", 256, "persistent"),
]


@pytest.mark.parametrize("name,make,problem,S,engine", CASES, ids=[c[0] for c in CASES])
def test_engine_matches_streaming_bitwise(name, make, problem, S, engine):
    q = qqa()
    g = make()
    K, seed = 200, 5
    # the state after update t1 is P[t1 & 1] (the other buffer is scratch), m and v
    a = run(q, g, problem, S, 0, 37, K, seed, "stream")
    b = run(q, g, problem, S, 0, 37, K, seed, engine)
    for x, y in zip([a[0][1], a[1], a[2]], [b[0][1], b[1], b[2]]):
        assert torch.equal(x, y), name
    # resuming mid-schedule from the streamed state gives the same bits as running through
    c = run(q, g, problem, S, 37, 60, K, seed, engine, state=a)
    d = run(q, g, problem, S, 0, 60, K, seed, "stream")
    for x, y in zip([c[0][0], c[1], c[2]], [d[0][0], d[1], d[2]]):
        assert torch.equal(x, y), name


def test_engine_one_update_matches_oracle(orc):
    from test_gpu_parity import check_step, oracle_params, step_sensitivity  # the common per-step contract
    q = qqa()
    g = qi.erdos_renyi(3000, 5.0, 2)
    S, K, seed, t = 64, 100, 9, 17
    P, m, v = qi.synthetic_state(g["n"], S, seed=3)
    d = torch.device("cuda")
    Pt = [torch.as_tensor(P, device=d), torch.full((g["n"], S), -1.0, device=d)]
    if t % 2:
        Pt = Pt[::-1]
    mt, vt = torch.as_tensor(m, device=d), torch.as_tensor(v, device=d)
    sched = q.schedule("mis", g["n"])
    q.qqa_dev_run(q.DevGraph(g), "mis", sched, S, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "persistent")
    torch.cuda.synchronize()
    out = Pt[(t + 1) & 1].cpu().numpy()
    ref = orc.step(oracle_params(orc, q, sched, "mis"), g, t, K, seed, P, m, v)
    sens = step_sensitivity(ref, m.astype(np.float64), v.astype(np.float64), t, sched, True)
    check_step("persistent/t17", (out, mt.cpu().numpy(), vt.cpu().numpy()), ref, S, True, sched.beta1, sched.beta2, sens)


def test_engine_rejections():
    q = qqa()
    hubby = qi.pm1_weights(qi.barabasi_albert(5000, 4, 1), 1)  # rows above the split threshold
    with pytest.raises(q.QQAError) as e:
        run(q, hubby, "maxcut", 128, 0, 3, 10, 1, "persistent")
    assert e.value.code == q.QQA_E_ARG
    with pytest.raises(q.QQAError):
        run(q, qi.erdos_renyi(20000, 5.0, 0), "mis", 256, 0, 3, 10, 1, "lds_block")  # P does not fit in LDS
    with pytest.raises(q.QQAError):
        run(q, qi.erdos_renyi(500, 5.0, 0), "mis", 100, 0, 3, 10, 1, "persistent")  # not a full-width layout


def test_context_engine_policy_same_results():
    q = qqa()
    ctx = q.Context(0)
    g = qi.erdos_renyi(20000, 5.0, 0)
    gid = ctx.upload(g, "mis")
    ctx.set_engine("persistent")
    a = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", 256, 120, 3))
    ctx.set_engine("stream")
    b = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", 256, 120, 3))
    ctx.release(gid)
    assert a["engine"] == "persistent" and np.array_equal(a["obj"], b["obj"])
    # automatic: the LDS engine for an instance that fits one workgroup (same bits as
    # streaming), whole-row streaming for S = 64, slices for S = 128 and 256 (their own tests)
    for g, S, engine in [(qi.random_regular(256, 3, 0), 16, "lds_block"), (qi.erdos_renyi(20000, 5.0, 0), 64, "stream"),
                         (qi.erdos_renyi(20000, 5.0, 0), 128, "sliced"), (qi.erdos_renyi(20000, 5.0, 0), 256, "sliced")]:
        gid = ctx.upload(g, "mis")
        ctx.set_engine("auto")
        a = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, 150, 3))
        ctx.set_engine("stream")
        b = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, 150, 3))
        ctx.release(gid)
        assert a["engine"] == engine and b["engine"] == "stream"
        if engine != "sliced":
            assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    ctx.close()


def test_context_lds_block_noise_chunks_same_results():
    # A context solve on the LDS engine forms its normals ahead of the updates, a bounded
    # table of updates at a time: 1,024 rows at S = 8 (64 KiB of P in LDS) hold 2,048
    # updates per table, so 4,500 updates run in three chunks (P and the moments pass
    # through global memory between them).  The results equal those of the streaming
    # engine, which draws the same normals.  At S = 64 P exceeds the LDS: streaming.
    q = qqa()
    ctx = q.Context(0)
    g = qi.erdos_renyi(1024, 4.0, 7)
    gid = ctx.upload(g, "mis")
    for S, K in [(8, 4500), (64, 40)]:
        ctx.set_engine("auto")
        a = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, K, 11))
        ctx.set_engine("stream")
        b = ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, K, 11))
        assert a["engine"] == ("lds_block" if S == 8 else "stream") and b["engine"] == "stream"
        assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
    ctx.release(gid)
    ctx.close()


def test_dev_run_lds_block_noise_chunks_from_mid_schedule():
    # the per-stage entry point on the LDS engine: updates 100 .. 4,599 of a 5,000-update
    # schedule run as two noise chunks (4,096 updates of 256 rows x 4 quads fit one 64 MiB
    # table), starting mid-schedule: the same bits as the streaming engine
    q = qqa()
    g = qi.random_regular(256, 3, 0)
    S, K, seed = 16, 5000, 8
    a = run(q, g, "mis", S, 0, 100, K, seed, "stream")
    b = run(q, g, "mis", S, 100, 4600, K, seed, "lds_block", state=a)
    c = run(q, g, "mis", S, 100, 4600, K, seed, "stream", state=a)
    for x, y in zip([b[0][0], b[1], b[2]], [c[0][0], c[1], c[2]]):
        assert torch.equal(x, y)
