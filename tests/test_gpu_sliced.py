"""The sliced streaming engine (replica axis cut into 8 slices, one per XCD, or below 256
replicas into 4 slices, one per XCD pair; replica statistics
combined from the slices' partials, which each update leaves for the next): one update
matches the oracle, from a given state and from a state the engine reached itself (so the
partials it wrote are checked); a run interrupted and resumed gives the same bits as one
run through; one update agrees with the whole-row engine to rounding.  Full and ragged
slices, the narrowest and widest slice widths, split (hub) rows, max-cut weights, max
clique's per-replica sums and the Langevin rule.  A context runs it by policy."""

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


def run(q, g, problem, S, t0, t1, K, seed, engine, sched=None, state=None):
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
    q.qqa_dev_run(q.DevGraph(g), problem, sched, S, t0, t1, K, seed, P[0], P[1], m, v, engine)
    torch.cuda.synchronize()
    return P, m, v


def rb_graph():
    return qi.rb_model(20, 12, 2.6, 0.25, 0)  # degrees 160-212: split rows


CASES = [
    # name, graph, problem, S
    ("er20000_S256_mis", lambda: qi.erdos_renyi(20000, 5.0, 0), "mis", 256),
    ("ba5000_S128_maxcut_hubs_four_slices", lambda: qi.pm1_weights(qi.barabasi_albert(5000, 4, 1), 1), "maxcut", 128),
    ("er3000_S200_mis_four_slices_ragged", lambda: qi.erdos_renyi(3000, 7.0, 6), "mis", 200),
    ("er4000_S100_mis_ragged", lambda: qi.erdos_renyi(4000, 8.0, 2), "mis", 100),
    ("er4000_S61_mis_narrowest", lambda: qi.erdos_renyi(4000, 8.0, 3), "mis", 61),
    ("er3000_S1000_maxcut", lambda: qi.pm1_weights(qi.erdos_renyi(3000, 6.0, 4), 2), "maxcut", 1000),
    ("rrg2000_S4096_mis_widest", lambda: qi.random_regular(2000, 3, 5), "mis", 4096),
    ("rb_S64_maxclique", rb_graph, "maxclique", 64),
    ("rb_S1000_maxclique", rb_graph, "maxclique", 1000),
]


@pytest.mark.parametrize("name,make,problem,S", CASES, ids=[c[0] for c in CASES])
def test_sliced_resume_is_bitwise_continuous_and_deterministic(name, make, problem, S):
    q = qqa()
    g = make()
    K, seed = 200, 7
    a = run(q, g, problem, S, 0, 23, K, seed, "sliced")
    a2 = run(q, g, problem, S, 0, 23, K, seed, "sliced")
    for x, y in zip([a[0][1], a[1], a[2]], [a2[0][1], a2[1], a2[2]]):
        assert torch.equal(x, y), name
    # resumed mid-schedule: the first update's partials are formed from P exactly as the
    # previous update would have left them
    c = run(q, g, problem, S, 23, 40, K, seed, "sliced", state=a)
    d = run(q, g, problem, S, 0, 40, K, seed, "sliced")
    for x, y in zip([c[0][0], c[1], c[2]], [d[0][0], d[1], d[2]]):
        assert torch.equal(x, y), name


@pytest.mark.parametrize("name,make,problem,S", CASES, ids=[c[0] for c in CASES])
def test_sliced_one_update_agrees_with_whole_rows(name, make, problem, S):
    q = qqa()
    g = make()
    a = run(q, g, problem, S, 0, 1, 100, 3, "stream")
    b = run(q, g, problem, S, 0, 1, 100, 3, "sliced")
    # the replica statistics are rounded differently; everything else is the same arithmetic.
    # AdamW's first step moves p by -lr g / (|g| + eps): where |g| is tiny that step turns
    # a rounding-level change of g into a visible one, so a handful of elements may differ
    # more (the oracle tests bound those by the step's sensitivity)
    dP = (a[0][1] - b[0][1]).abs()
    assert int((dP > 1e-5).sum()) <= max(4, dP.numel() // 100000), (name, float(dP.max()))
    assert float(dP.max()) <= 2 * 0.1 + 1e-6  # at most the size of two steps
    assert torch.allclose(a[1], b[1], rtol=1e-3, atol=1e-7) and torch.allclose(a[2], b[2], rtol=1e-3, atol=1e-9)


def _check_against_oracle(q, orc, label, g, problem, sched, S, t, K, seed, state_in, gpu_out):
    from test_gpu_parity import check_step, oracle_params, step_sensitivity
    P, m, v = (x[:, :S].astype(np.float32) for x in state_in)
    ref = orc.step(oracle_params(orc, q, sched, problem), g, t, K, seed, P, m, v)
    adam = sched.rule == 0
    sens = step_sensitivity(ref, m.astype(np.float64), v.astype(np.float64), t, sched, adam)
    check_step(label, gpu_out, ref, S, adam, sched.beta1, sched.beta2, sens, float(np.float32(sched.comm_alpha)))


ORACLE_CASES = [
    ("ba3000_S200_maxcut_hubs", lambda: qi.pm1_weights(qi.barabasi_albert(3000, 4, 2), 3), "maxcut", 200),
    ("er3000_S256_mis", lambda: qi.erdos_renyi(3000, 6.0, 5), "mis", 256),
    ("er1000_S1000_mis_ragged", lambda: qi.erdos_renyi(1000, 8.0, 6), "mis", 1000),
    ("er800_S61_mis", lambda: qi.erdos_renyi(800, 5.0, 7), "mis", 61),
    ("rb_S300_maxclique", rb_graph, "maxclique", 300),
]


@pytest.mark.parametrize("name,make,problem,S", ORACLE_CASES, ids=[c[0] for c in ORACLE_CASES])
def test_sliced_one_update_matches_oracle(orc, name, make, problem, S):
    q = qqa()
    g = make()
    K, seed, t = 100, 9, 17
    P, m, v = qi.synthetic_state(g["n"], S, seed=4)
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(S)
    pad = lambda a: np.pad(a, ((0, 0), (0, stride - S)))
    Pt = [torch.as_tensor(pad(P), device=d), torch.full((g["n"], stride), -1.0, device=d)]
    if t % 2:
        Pt = Pt[::-1]
    mt, vt = torch.as_tensor(pad(m), device=d), torch.as_tensor(pad(v), device=d)
    sched = q.schedule(problem, g["n"])
    q.qqa_dev_run(q.DevGraph(g), problem, sched, S, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "sliced")
    torch.cuda.synchronize()
    gpu = (Pt[(t + 1) & 1].cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy())
    _check_against_oracle(q, orc, f"sliced {name}", g, problem, sched, S, t, K, seed, (pad(P), pad(m), pad(v)), gpu)


@pytest.mark.parametrize("name,make,problem,S", ORACLE_CASES[:3], ids=[c[0] for c in ORACLE_CASES[:3]])
def test_sliced_partials_from_its_own_updates_match_oracle(orc, name, make, problem, S):
    """Update t of a run from the start uses the partial statistics update t - 1 wrote."""
    q = qqa()
    g = make()
    K, seed, t = 100, 11, 6
    sched = q.schedule(problem, g["n"])
    before = run(q, g, problem, S, 0, t, K, seed, "sliced")
    after = run(q, g, problem, S, 0, t + 1, K, seed, "sliced")
    state_in = (before[0][t & 1].cpu().numpy(), before[1].cpu().numpy(), before[2].cpu().numpy())
    gpu = (after[0][(t + 1) & 1].cpu().numpy(), after[1].cpu().numpy(), after[2].cpu().numpy())
    _check_against_oracle(q, orc, f"sliced run {name}", g, problem, sched, S, t, K, seed, state_in, gpu)


def test_full_size_sliced_matches_oracle(orc):
    """The sparse MIS benchmark shape (ER n = 20,000, mean degree 5, S = 256, 3,000 updates) in
    the engine a solve picks for it: one update from a synthetic state, then update 6 of a
    run from the start, which combines the partials update 5 wrote."""
    q = qqa()
    g, problem, S, K = qi.erdos_renyi(20000, 5.0, 0), "mis", 256, 3000
    sched = q.schedule(problem, g["n"])
    seed, t = 21, 1234
    P, m, v = qi.synthetic_state(g["n"], S, seed=8)
    d = torch.device("cuda")
    stride = q.qqa_replica_stride(S)
    Pt = [torch.as_tensor(P, device=d), torch.full((g["n"], stride), -1.0, device=d)]
    mt, vt = torch.as_tensor(m, device=d), torch.as_tensor(v, device=d)
    q.qqa_dev_run(q.DevGraph(g), problem, sched, S, t, t + 1, K, seed, Pt[0], Pt[1], mt, vt, "sliced")
    torch.cuda.synchronize()
    gpu = (Pt[1].cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy())
    _check_against_oracle(q, orc, "sliced C2 synthetic", g, problem, sched, S, t, K, seed, (P, m, v), gpu)
    t = 6
    before = run(q, g, problem, S, 0, t, K, seed, "sliced")
    after = run(q, g, problem, S, 0, t + 1, K, seed, "sliced")
    state_in = (before[0][t & 1].cpu().numpy(), before[1].cpu().numpy(), before[2].cpu().numpy())
    gpu = (after[0][(t + 1) & 1].cpu().numpy(), after[1].cpu().numpy(), after[2].cpu().numpy())
    _check_against_oracle(q, orc, "sliced C2 run", g, problem, sched, S, t, K, seed, state_in, gpu)


def test_sliced_langevin_agrees_with_whole_rows():
    q = qqa()
    g = qi.erdos_renyi(5000, 6.0, 8)
    sched = q.schedule("mis", g["n"])
    sched.rule = q.QQA_STEP_LANGEVIN
    a = run(q, g, "mis", 160, 0, 1, 100, 3, "stream", sched=sched)
    b = run(q, g, "mis", 160, 0, 1, 100, 3, "sliced", sched=sched)
    assert float((a[0][1] - b[0][1]).abs().max()) <= 1e-5  # Langevin: p - lr g, well conditioned
    c = run(q, g, "mis", 160, 0, 9, 100, 3, "sliced", sched=sched)
    d = run(q, g, "mis", 160, 0, 4, 100, 3, "sliced", sched=sched)
    e = run(q, g, "mis", 160, 4, 9, 100, 3, "sliced", sched=sched, state=d)
    assert torch.equal(c[0][1], e[0][1])


def test_sliced_rejects_narrow_replica_counts():
    q = qqa()
    with pytest.raises(q.QQAError) as e:
        run(q, qi.erdos_renyi(500, 5.0, 0), "mis", 60, 0, 3, 10, 1, "sliced")  # 15 quads: < 2 per slice
    assert e.value.code == q.QQA_E_ARG


@pytest.mark.parametrize("n,S,problem,family", [(4000, 256, "mis", "er"), (3000, 512, "maxcut", "er"),
                                                (2500, 128, "mis", "er"), (3000, 200, "mis", "er"),
                                                (5000, 128, "maxcut", "ba"), (4000, 256, "mis", "ba")])
def test_context_slice_major_state_equals_row_major(n, S, problem, family):
    """A context's sliced solve keeps its state slice-major where the slices are equal (each
    XCD's slice of P, m, v contiguous, and the split rows' chunk partials per slice) and
    converts P back for the evaluation; the per-stage path runs the same engine on row-major
    buffers.  Same seed, schedule and updates: every replica's exact objective, the best
    replica and its solution agree bit for bit (S = 200 has unequal slices and stays
    row-major in both; the BA graphs have split hub rows)."""
    q = qqa()
    g = qi.erdos_renyi(n, 6.0, 40 + S) if family == "er" else qi.barabasi_albert(n, 4, 40 + S)
    if problem == "maxcut":
        g = qi.pm1_weights(g, 3)
    K, seed = 120, 17
    ctx = q.Context(0)
    gid = ctx.upload(g, problem)
    ctx.set_engine("sliced")
    r = ctx.poll(ctx.solve_resident(gid, n, problem, S, K, seed))
    ctx.release(gid)
    ctx.close()
    assert r["engine"] == "sliced"
    P, _, _ = run(q, g, problem, S, 0, K, K, seed, "sliced")
    d = torch.device("cuda")
    out = [torch.zeros((S,), dtype=torch.int64, device=d) for _ in range(3)]
    best = torch.zeros((1,), dtype=torch.int32, device=d)
    q.qqa_dev_eval(q.DevGraph(g), problem, q.schedule(problem, n).penalty_lambda, S, P[K & 1], *out, best)
    torch.cuda.synchronize()
    assert np.array_equal(r["obj"], out[2].cpu().numpy()), (n, S)
    assert np.array_equal(r["size_or_cut"], out[0].cpu().numpy())
    assert r["best_replica"] == int(best.item())
    x = (P[K & 1][:, r["best_replica"]] > 0.5).to(torch.uint8).cpu().numpy()
    assert np.array_equal(r["best_x"], x)


def test_context_sliced_policy():
    from test_gpu_solve import objective_of
    q = qqa()
    ctx = q.Context(0)
    for g, problem, S in [(qi.pm1_weights(qi.barabasi_albert(6000, 4, 1), 1), "maxcut", 256),
                          (qi.erdos_renyi(20000, 5.0, 0), "mis", 256)]:
        gid = ctx.upload(g, problem)
        ctx.set_engine("sliced")
        a = ctx.poll(ctx.solve_resident(gid, g["n"], problem, S, 150, 3))
        b = ctx.poll(ctx.solve_resident(gid, g["n"], problem, S, 150, 3))
        ctx.release(gid)
        assert a["engine"] == "sliced" and a["kernel_us"] > 0
        assert np.array_equal(a["obj"], b["obj"]) and np.array_equal(a["best_x"], b["best_x"])
        assert a["best_objective"] == objective_of(g, a["best_x"], problem)
    # automatic policy: slices of whole 128-byte lines whose share of P fits an XCD's L2;
    # with the state slice-major (equal slices, no split rows) P up to 64 MiB, and four
    # slices from S = 128 with P up to 32 MiB
    ctx.set_engine("auto")
    hubs = qi.barabasi_albert(5000, 4, 1)  # rows above the split threshold
    for g, S, engine in [(qi.erdos_renyi(2000, 8.0, 1), 256, "sliced"), (qi.erdos_renyi(2000, 8.0, 1), 128, "sliced"),
                         (qi.erdos_renyi(2000, 8.0, 1), 64, "stream"), (hubs, 128, "sliced"), (hubs, 256, "sliced"),
                         (qi.erdos_renyi(1000, 8.0, 1), 1000, "sliced"), (qi.erdos_renyi(30000, 4.0, 1), 256, "sliced"),
                         (qi.erdos_renyi(80000, 4.0, 1), 256, "stream"), (qi.erdos_renyi(40000, 4.0, 1), 200, "stream")]:
        gid = ctx.upload(g, "mis")
        assert ctx.poll(ctx.solve_resident(gid, g["n"], "mis", S, 50, 1))["engine"] == engine, (g["n"], S)
        ctx.release(gid)
    g = rb_graph()
    gid = ctx.upload(g, "maxclique")
    r = ctx.poll(ctx.solve_resident(gid, g["n"], "maxclique", 1000, 400, 2))
    ctx.release(gid)
    assert r["engine"] == "sliced" and r["feasible"] and r["best_size_or_cut"] >= 18  # planted clique: 20
    ctx.close()
