"""Benchmark: replica-variable updates per second of whole PQQA solves on one MI355X.

One benchmark step is one complete solve through the C ABI (U(0,1) init, every update
of the schedule, rounding and exact evaluation) of the workload below, with the graph
already resident in HBM.  Prints one JSON line.

Default workload (the sparse single-instance configuration): maximum independent set
on an Erdos-Renyi graph, n = 20,000, mean degree 5 (seeded G(n, p)), S = 256 replicas,
3,000 updates, float32 state, AdamW + alpha-entropy annealing + STD communication.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "replica-var updates/s (N·S·steps/s); p50/p99 solve latency, batched vs plain"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 compute units at 2.4 GHz
COMPUTE_UNITS = 256

WORKLOADS = {
    # name: (family, n, degree parameter, problem, S, updates)
    "mis_er_n20000_d5_S256_K3000": ("er", 20000, 5.0, "mis", 256, 3000),
    "maxcut_ba_n100000_m4_pm1_S128_K3000": ("ba", 100000, 4, "maxcut", 128, 3000),
    "mis_rrg_n256_d3_S16_K2000": ("rrg", 256, 3, "mis", 16, 2000),
    # dense symmetric Gaussian couplings (Sherrington-Kirkpatrick-like max-cut)
    "maxcut_dense_n4096_gauss_S256_K3000": ("dense", 4096, 0, "maxcut", 256, 3000),
    # the MIS scaling study's shape: random 20-regular graph, one million variables, S = 1
    "mis_rrg_n1000000_d20_S1_K3000": ("rrg_swap", 1000000, 20, "mis", 1, 3000),
    # the study's degree-100 graphs: every row above the split threshold (64 neighbours)
    "mis_rrg_n100000_d100_S1_K3000": ("rrg_swap", 100000, 100, "mis", 1, 3000),
    # max clique on a Model RB instance (20 variables x 12 values, planted clique of 20),
    # the paper's 1,000 parallel runs
    "maxclique_rb20x12_S1000_K3000": ("rb", 240, (20, 12, 2.6, 0.25), "maxclique", 1000, 3000),
    # graph coloring (categorical K-state QQA): the largest queens graph of the paper's
    # coloring table with 13 colours, 1,000 parallel runs; and an ER graph sized to load the GPU
    "coloring_queen13_K13_S1000_K3000": ("queens", 169, 13, "coloring", 1000, 3000),
    "coloring_er_n100000_d10_K8_S32_K1000": ("er_color", 100000, (10.0, 8), "coloring", 32, 1000),
}
DEFAULT = "mis_er_n20000_d5_S256_K3000"


def make_graph(family, n, d, problem, seed=0):
    import qqa_inputs as qi
    if family == "dense":
        return {"n": n, "dense": qi.dense_gaussian(n, seed)}
    if family == "rb":
        return qi.rb_model(*d, seed)
    if family == "queens":
        return qi.queens(int(round(n ** 0.5)))
    if family == "er_color":
        return qi.erdos_renyi(n, d[0], seed)
    if family == "rrg_swap":
        return qi.random_regular_swapped(n, int(d), seed)
    if family == "er":
        g = qi.erdos_renyi(n, d, seed)
    elif family == "ba":
        g = qi.barabasi_albert(n, int(d), seed)
    else:
        g = qi.random_regular(n, int(d), seed)
    if problem == "maxcut":
        g = qi.pm1_weights(g, seed + 1)
    return g


def algorithmic_bytes_per_update_launch(n, nnz, S, stride, weighted):
    """Bytes one update launch must move: the replica state (read P_t, write P_{t+1}, read
    and write m and v: 24 B per replica-variable) plus one pass over the CSR (row_ptr,
    col, weights).  Neighbour-row re-reads are not algorithmic: caches serve them."""
    state = 24 * n * S
    csr = 4 * (n + 1) + 4 * nnz + (4 * nnz if weighted else 0)
    return state + csr


def update_flops(n, nnz, S, maxcut, alpha_e):
    """Arithmetic of one update (AdamW): per replica-variable the statistics (4 flops), the
    penalty, entropy and communication gradient (11 + the alpha_e - 2 multiplies of the
    entropy power; 2 fewer for max-cut, whose gradient is the coupling itself), the moments
    and step (16), noise and clamp (4); per CSR entry and replica a multiply-add (2 more
    for max-cut's 2 p - 1)."""
    per_elem = 31 + (alpha_e - 2) + (0 if maxcut else 2)
    per_edge = 4 if maxcut else 2
    return n * S * per_elem + nnz * S * per_edge


def dense_coupling_us(q, W, n, S, problem, launches=20):
    """Average duration of one launch of the matrix-core coupling product at the solve's
    shape, from HIP events on the stream the kernels are launched on."""
    import torch
    stride = q.qqa_replica_stride(S)
    Wd = torch.as_tensor(W, device="cuda")
    P = torch.rand(n, stride, device="cuda")
    C = torch.empty_like(P)
    st = torch.cuda.current_stream()
    for _ in range(3):
        q.qqa_dev_dense_coupling(Wd, P, C, n, S, problem, st)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # hold the stream on the device while every launch is enqueued, so that the events
    # bracket back-to-back kernels and not the host's launch rate
    torch.cuda._sleep(20_000_000)
    a.record(st)
    for _ in range(launches):
        q.qqa_dev_dense_coupling(Wd, P, C, n, S, problem, st)
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / launches


DEVICE_SOURCES = ["qqa_device.h", "qqa_kernels.hip"]
DENSE_SOURCES = ["qqa_dense.hip"]
SLICE_SOURCES = ["qqa_device.h", "qqa_slice.hip"]
COMPACT_SOURCES = ["qqa_device.h", "qqa_compact.hip"]
SLOT_SOURCES = ["qqa_device.h", "qqa_slots.hip"]
RESIDENT_SOURCES = ["qqa_device.h", "qqa_resident.hip"]
BATCH_WORKLOAD = "batch512_er_n200-5000_d3-20_S32_K2000"


def source_hash(sources):
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2409_02135_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def device_source_hash():
    return source_hash(DEVICE_SOURCES)


def traffic_from_profiles(record, sources, workload):
    """Measured HBM bytes per launch of a kernel on this workload, from a committed rocprofv3
    counter summary (one record, or a list of records for several workloads), if it was
    taken with the current kernel source; else None."""
    try:
        recs = json.load(open(os.path.join(ROOT, "profiles", record)))
    except (OSError, ValueError):
        return None
    for rec in recs if isinstance(recs, list) else [recs]:
        if rec.get("workload") == workload and rec.get("kernel_source_sha256") == source_hash(sources):
            return rec.get("bytes_per_launch")
    return None


def cpu_baseline_batch(gs, S, K, updates=2):
    """The FP64 oracle on a bounded sample of the batched workload: the first `updates`
    updates of every instance from its start, one thread, one instance after another."""
    import oracle
    pr = oracle.Params().as_float32()
    work, dt = 0.0, 0.0
    for k, g in enumerate(gs):
        P = oracle.init(k, g["n"], S)
        z = np.zeros_like(P)
        t0 = time.perf_counter()
        oracle.run(pr, g, 0, updates, K, k, P, z, z)
        dt += time.perf_counter() - t0
        work += float(g["n"]) * S * updates
    return {"value": work / dt, "unit": "updates/s", "cores": 1, "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"the first {updates} of {K} updates of each of the {len(gs)} instances, single-threaded FP64 C"}


def batched_vs_plain(q, count=512, S=32, K=2000, seed=0, plain=True, with_cpu=False, tune=True):
    """The ragged multi-instance configuration: `count` MIS instances on G(n, p) graphs with
    n ~ U{200..5000} and mean degree ~ U[3, 20], S replicas, K updates each; tuned by the
    batch autotuner, then solved as one batch (the engine it kept), on the slot launches (one
    launch per update for all instances, replayed from a captured graph) and as a loop of
    single solves on the same GPU.  All use the same replica layout, so their results must
    be identical."""
    import qqa_inputs as qi
    import torch
    gs = qi.instance_batch(count, seed, n_range=(200, 5000), deg_range=(3.0, 20.0))
    ctx = q.Context(0)
    gids = [ctx.upload(g, "mis") for g in gs]
    ns = [g["n"] for g in gs]
    work = float(sum(ns)) * S * K
    seeds = list(range(count))
    # warm-up of both paths on two instances
    for r in ctx.solve_batch(gids[:2], ns[:2], ["mis"] * 2, [S] * 2, [50] * 2, [0, 1]):
        ctx.poll(r, want_x=False)
    ctx.poll(ctx.solve_resident(gids[0], ns[0], "mis", S, 50, 0), want_x=False)
    # the batch autotuner: replica layouts on the slot launches, then the resident engine,
    # on shortened copies of this batch; the runs below use what it kept
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = ctx.autotune_batch(gids, ["mis"] * count, [S] * count, [K] * count) if tune else None
    t_tune = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = ctx.solve_batch(gids, ns, ["mis"] * count, [S] * count, [K] * count, seeds)
    rb = [ctx.poll(i, want_x=False) for i in ids]
    tb = time.perf_counter() - t0
    # the same batch on the slot launches (one launch per update, replayed from a graph)
    ctx.set_engine("stream")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = ctx.solve_batch(gids, ns, ["mis"] * count, [S] * count, [K] * count, seeds)
    rs = [ctx.poll(i, want_x=False) for i in ids]
    ts = time.perf_counter() - t0
    ctx.set_engine("auto")
    same_slots = all(np.array_equal(a["obj"], b["obj"]) for a, b in zip(rb, rs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = [ctx.solve_resident(gid, n, "mis", S, K, s) for gid, n, s in zip(gids, ns, seeds)] if plain else []
    rp = [ctx.poll(i, want_x=False) for i in ids]
    tp = time.perf_counter() - t0
    same = all(np.array_equal(a["obj"], b["obj"]) for a, b in zip(rb, rp)) if plain else None
    lat_p = np.array([r["latency_ms"] for r in rp]) if plain else np.zeros(1)
    for gid in gids:
        ctx.release(gid)
    ctx.close()
    # the batched update loop against the HBM roofline: every instance's state (24 B per
    # replica-variable) and CSR once per update, over the device time of the update loop
    abytes = sum(algorithmic_bytes_per_update_launch(g["n"], int(g["col"].size), S, 0, False) for g in gs)
    loop_us = float(rb[0]["step_loop_ms"]) * 1e3 / K
    achieved = abytes / (loop_us * 1e-6) / 1e9
    return {"workload": f"{count} MIS instances, ER n~U[200,5000], mean degree~U[3,20], S={S}, {K} updates",
            "sum_n": int(sum(ns)), "batched_updates_per_s": work / tb,
            "plain_updates_per_s": work / tp if plain else None,
            "speedup": tp / tb if plain else None, "batched_s": tb, "plain_s": tp if plain else None,
            "identical_results": same,
            "engine": rb[0]["engine"],
            "autotune": ({"resident_kept": tuned[0], "lanes_per_row": tuned[1][0], "seconds": t_tune}
                         if tuned else None),
            "slot_launches": {"updates_per_s": work / ts, "seconds": ts, "identical_results": bool(same_slots),
                              "update_us": float(rs[0]["step_loop_ms"]) * 1e3 / K},
            "roofline": {"bound": "hbm", "kernel": "resident_kernel" if rb[0]["engine"] == "batch_resident"
                         else "slot_step_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         # measured bytes per update, from the counter record of the engine that ran
                         "traffic": (traffic_from_profiles(*({"batch": ("slot_step_traffic.json", SLOT_SOURCES),
                                                              "batch_resident": ("resident_traffic.json", RESIDENT_SOURCES)}
                                                             [rb[0]["engine"]]), BATCH_WORKLOAD)
                                     if count == 512 and K == 2000 and S == 32 else None),
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_update": abytes, "update_us": loop_us,
                         "basis": "device time of the batched update loop (events on the solver stream) / updates"},
            **({"oracle_context": cpu_baseline_batch(gs, S, K)} if with_cpu else {}),
            "batched_latency_ms": 1e3 * tb,
            "plain_latency_ms": {"p50": float(np.percentile(lat_p, 50)), "p99": float(np.percentile(lat_p, 99))}}


def graph_pool(count, seed=0, n_range=(1e3, 1e5)):
    """A pool of request graphs shaped like the served mix: ER (mean degree ~ U[3,20]) or BA
    (m = 4), n log-uniform in n_range, each with +-1 weights for max-cut use."""
    import qqa_inputs as qi
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(count):
        n = int(round(10 ** rng.uniform(np.log10(n_range[0]), np.log10(n_range[1]))))
        fam = "er" if k % 2 == 0 else "ba"
        g = qi.erdos_renyi(n, float(rng.uniform(3.0, 20.0)), 1000 + k) if fam == "er" else \
            qi.barabasi_albert(n, 4, 1000 + k)
        pool.append({"family": fam, "mis": g, "maxcut": qi.pm1_weights(g, 2000 + k)})
    return pool


def served(q, rate, arrival_window, pool, seed=0, max_slots=256, deadline_ms=0.0):
    """Requests arrive as a Poisson stream at `rate`/s during `arrival_window` s: MIS or +-1
    max-cut (1/2 each) on a graph from the pool, S in {32, 128}, 1000..3000 updates.  The
    server admits them as slots and memory free up; with a deadline it sheds, at submit,
    the requests whose projected completion exceeds it.  Finished results are collected
    while the stream runs."""
    import torch
    rng = np.random.default_rng(seed)
    t, arrivals = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= arrival_window:
            break
        gi = int(rng.integers(len(pool)))
        prob = "mis" if rng.random() < 0.5 else "maxcut"
        arrivals.append((t, gi, prob, int(rng.choice([32, 128])), int(rng.integers(1000, 3001)),
                         int(rng.integers(2 ** 31))))
    ctx = q.Context(0)
    ctx.serve_start(max_slots)
    if deadline_ms > 0:
        ctx.serve_set_deadline(deadline_ms)
    torch.cuda.synchronize()
    pending, done, offered_work, shed = {}, [], 0.0, 0
    last_sweep = 0.0

    def sweep(timeout_us=0):
        for rid in list(pending):
            r = ctx.poll(rid, timeout_us=timeout_us, want_x=False)
            if r is not None:
                done.append((r, pending.pop(rid)))

    t0 = time.perf_counter()
    for (ta, gi, prob, S, K, sd) in arrivals:
        now = time.perf_counter() - t0
        if now - last_sweep > 0.05:
            sweep()
            last_sweep = now
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        g = pool[gi][prob]
        w = float(g["n"]) * q.qqa_replica_stride(S) * K
        offered_work += float(g["n"]) * S * K
        try:
            pending[ctx.serve_submit(g, prob, S, K, sd)] = float(g["n"]) * S * K
        except q.QQAError as e:
            if e.code != q.QQA_E_ADMISSION:
                raise
            shed += 1
    sweep(timeout_us=-1)
    makespan = time.perf_counter() - t0
    stats = ctx.serve_stats()
    ctx.serve_stop()
    ctx.close()
    res = [r for r, _ in done]
    work_done = sum(w for _, w in done)
    lat = np.array([r["latency_ms"] for r in res]) if res else np.zeros(1)
    fst = np.array([r["first_update_ms"] for r in res]) if res else np.zeros(1)
    qms = np.array([r["queue_ms"] for r in res]) if res else np.zeros(1)
    pct = lambda a: {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99))}
    return {"rate_per_s": rate, "arrival_window_s": arrival_window, "deadline_ms": deadline_ms,
            "offered": {"requests": len(arrivals), "updates_per_s": offered_work / arrival_window},
            "admitted": {"requests": len(res), "updates_per_s": work_done / arrival_window},
            "shed_requests": shed, "server_counts": {k: stats[k] for k in ("submitted", "admitted", "shed", "completed")},
            "sustained_updates_per_s": work_done / makespan, "makespan_s": makespan,
            "measured_device_rate_updates_per_s": stats["rate_updates_per_s"],
            "latency_ms": pct(lat), "first_update_ms": pct(fst), "queue_ms": pct(qms),
            **({"met_deadline": {"requests": int(np.sum(lat <= deadline_ms)) if res else 0,
                                 "updates_per_s": sum(w for r, w in done if r["latency_ms"] <= deadline_ms)
                                 / arrival_window}} if deadline_ms > 0 else {}),
            "latency_basis": "admitted requests, submit -> result ready (host clock)",
            "feasible_fraction": float(np.mean([r["feasible"] for r in res])) if res else None}


def host_info(n, S, K, updates, dt):
    """Where the oracle ran, its cost per replica-variable update, and the full run that cost
    extrapolates to (linear in updates)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "ns_per_update": dt / (n * S * updates) * 1e9, "full_run_s_extrapolated": dt * K / updates}


def cpu_baseline(g, problem, S, K, updates=20):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: the first
    `updates` updates of the schedule from the same start, one thread."""
    import oracle
    pr = oracle.Params(problem={"mis": 0, "maxcut": 1, "maxclique": 2}[problem],
                       gamma_min=-20.0 if problem == "maxcut" and g["n"] >= 1000 else
                       (-5.0 if problem == "maxcut" else -2.0)).as_float32()
    P = oracle.init(0, g["n"], S)
    z = np.zeros_like(P)
    og = oracle.graph(W=g["dense"]) if "dense" in g else g
    t0 = time.perf_counter()
    oracle.run(pr, og, 0, updates, K, 0, P, z, z)
    dt = time.perf_counter() - t0
    return {"value": g["n"] * S * updates / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{updates} of {K} updates of the same instance from the same start, single-threaded FP64 C",
            "seconds": round(dt, 3), **host_info(g["n"], S, K, updates, dt)}


def cpu_baseline_coloring(g, colors, S, K, updates=20):
    """The FP64 oracle's categorical update on a bounded sample: the first `updates`
    updates of the same instance from the same start, one thread."""
    import oracle
    pr = oracle.Params().as_float32()
    V = oracle.cat_init(0, g["n"], colors, S)
    z = np.zeros_like(V)
    t0 = time.perf_counter()
    oracle.cat_run(pr, g, 0, updates, K, 0, V, z, z)
    dt = time.perf_counter() - t0
    return {"value": g["n"] * S * updates / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{updates} of {K} updates of the same instance from the same start ({colors} colours), "
                      "single-threaded FP64 C", "seconds": round(dt, 3), **host_info(g["n"], S, K, updates, dt)}


def measure(q, workload, steps, warmup, lanes_arg=-1, engine="auto", updates=0):
    """Time `steps` whole solves of one workload (after `warmup` untimed ones) with the graph
    resident on the device; returns the figures of the JSON line for it."""
    import torch
    family, n, d, problem, S, K = WORKLOADS[workload]
    if updates > 0:
        K = updates
    g = make_graph(family, n, d, problem)
    dense = family == "dense"
    coloring = problem == "coloring"
    colors = (d if family == "queens" else d[1]) if coloring else 0
    nnz = n * (n - 1) if dense else int(g["col"].size)
    ctx = q.Context(0)
    if coloring:
        gid = ctx.upload(g, problem)
        lanes = max(lanes_arg, 0)  # the tuner times the binary update kernel
    elif dense:
        gid = ctx.upload(None, problem, dense=g["dense"])
        lanes = max(lanes_arg, 0)  # the layout only concerns the fused update here
    else:
        gid = ctx.upload(g, problem)
        lanes = ctx.autotune(gid, problem, S) if lanes_arg < 0 else lanes_arg
    ctx.set_replica_layout(S, lanes)
    ctx.set_engine(engine)
    print(f"# workload {workload}: n={n} nnz={nnz} S={S} updates={K} lanes_per_row={lanes}",
          file=sys.stderr, flush=True)

    def submit(seed):
        if coloring:
            return ctx.solve_coloring_resident(gid, n, colors, S, K, seed)
        return ctx.solve_resident(gid, n, problem, S, K, seed)

    for w in range(warmup):
        ctx.poll(submit(1000 + w), want_x=False)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = [submit(s) for s in range(steps)]
    results = [ctx.poll(i, want_x=False) for i in ids]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    value = n * S * K * steps / elapsed
    dev_ms = np.array([r["device_ms"] for r in results])
    loop_ms = np.array([r["step_loop_ms"] for r in results])
    step_us = float(np.mean(loop_ms)) * 1e3 / K  # average duration of one update launch
    stride = q.qqa_replica_stride(S)
    engine_ran = results[0]["engine"]
    if dense:
        # dominant kernel: the FP32 matrix-core product, 2 n^2 S flops per launch, timed by
        # the library with events on sampled launches inside the timed solves
        mm_us = float(np.mean([r["kernel_us"] for r in results]))
        flops = 2.0 * n * n * S
        achieved = flops / (mm_us * 1e-6) / 1e12
        roofline = {"bound": "mfma", "kernel": "dense_tile128_kernel", "achieved": achieved,
                    "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                    "traffic": traffic_from_profiles("dense_tile128_kernel_traffic.json", DENSE_SOURCES, workload),
                    "avg_launch_us": mm_us, "algorithmic_flops_per_launch": flops,
                    "update_loop_us_per_update": step_us,
                    "uniform_random_state_us": dense_coupling_us(q, g["dense"], n, S, problem)}
    elif coloring:
        # one update is one or two launches (gradient over N*K rows, then the per-variable
        # update); algorithmic bytes: V, m, v read and written for every colour, plus the CSR
        abytes = 24 * n * colors * S + 4 * (n + 1) + 4 * nnz
        achieved = abytes / (step_us * 1e-6) / 1e9
        # one launch when the variable's colours x replica quads fit a wavefront (the library's rule)
        nq = stride // 4
        kp = 1 << (colors - 1).bit_length()
        fused = colors <= 8 and nq & (nq - 1) == 0 and kp * nq <= 64 and lanes_arg in (-1, 0, nq)
        roofline = {"bound": "hbm", "kernel": "cat_fused_kernel" if fused else "cat_grad_kernel + cat_update_kernel",
                    "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "avg_launch_us": step_us, "algorithmic_bytes_per_launch": abytes,
                    "sampled_kernel_us": float(np.mean([r["kernel_us"] for r in results]))}
    elif engine_ran == "lds_block":
        # one workgroup on one compute unit runs the whole solve: bound by that unit's vector
        # ALUs (the instance is far too small for memory bandwidth to matter)
        flops = update_flops(n, nnz, S, problem == "maxcut", q.qqa_schedule_default(problem, n).entropy_alpha)
        peak = FP32_VECTOR_PEAK_TFLOPS * 1e3 / COMPUTE_UNITS
        achieved = flops / (step_us * 1e-6) / 1e9
        roofline = {"bound": "alu", "kernel": "lds_block_kernel", "scope": "one compute unit",
                    "achieved": achieved, "peak": peak, "unit": "GFLOP/s", "frac": achieved / peak,
                    "traffic": None, "avg_update_us": step_us, "algorithmic_flops_per_update": flops}
    else:
        abytes = algorithmic_bytes_per_update_launch(n, nnz, S, stride, problem == "maxcut")
        achieved = abytes / (step_us * 1e-6) / 1e9
        kernel = {"sliced": "slice_step_kernel", "compact": "compact_step_kernel", "persistent": "persistent_kernel"}.get(engine_ran, "step_kernel")
        record = {"slice_step_kernel": ("slice_step_traffic.json", SLICE_SOURCES),
                  "compact_step_kernel": ("compact_step_traffic.json", COMPACT_SOURCES),
                  "step_kernel": ("step_kernel_traffic.json", DEVICE_SOURCES)}.get(kernel)
        roofline = {"bound": "hbm", "kernel": kernel,
                    "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": traffic_from_profiles(*record, workload) if record else None,
                    "avg_launch_us": step_us, "algorithmic_bytes_per_launch": abytes,
                    "sampled_launch_us": float(np.mean([r["kernel_us"] for r in results]))}
    ctx.release(gid)
    ctx.close()
    return {
        "graph": g, "problem": problem, "S": S, "K": K, "colors": colors, "dense": dense,
        "value": value, "elapsed": elapsed, "steps": steps,
        "config": {"workload": workload, "problem": problem, "graph": family, "n": n, "nnz": nnz,
                   **({"colors": colors} if coloring else {}),
                   "degree_param": d, "S": S, "updates_per_solve": K, "graph_seed": 0,
                   "lanes_per_row": lanes, "engine": engine_ran, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(dev_ms, 50)), "p99": float(np.percentile(dev_ms, 99)),
                       "basis": "device time per solve (events on the solver stream)"},
        "us_per_update": step_us,
        "roofline": roofline,
        "quality": {"best_objective_mean": float(np.mean([r["best_objective"] for r in results])),
                    "feasible_all": bool(all(r["feasible"] for r in results))},
    }


# The other configurations of the benchmark set, each timed over a few whole solves in the
# default run: the small latency-bound instance, the heavy-tailed max-cut instance and its
# dense matrix-core variant.  The batched and served configurations have blocks of their own.
CONFIG_BLOCKS = [("mis_rrg_n256_d3_S16_K2000", 5, 2, 2000),
                 ("maxcut_ba_n100000_m4_pm1_S128_K3000", 3, 1, 3),
                 ("maxcut_dense_n4096_gauss_S256_K3000", 2, 1, 0)]


def config_block(q, workload, steps, warmup, oracle_updates, with_cpu):
    m = measure(q, workload, steps, warmup)
    out = {"value": m["value"], "unit": "updates/s", "steps": steps, "warmup": warmup,
           "ms_per_step": m["elapsed"] * 1e3 / steps, "us_per_update": m["us_per_update"],
           "config": m["config"], "latency_ms": m["latency_ms"], "roofline": m["roofline"], "quality": m["quality"]}
    if with_cpu and oracle_updates > 0:
        cb = cpu_baseline(m["graph"], m["problem"], m["S"], m["K"], updates=min(oracle_updates, m["K"]))
        out["oracle_context"] = {k: cb[k] for k in ("value", "unit", "cores", "sample", "ns_per_update",
                                                     "full_run_s_extrapolated")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other single-instance configurations")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batch-updates", type=int, default=2000,
                    help="updates per instance of the batched configuration (fewer for runs under counters)")
    ap.add_argument("--batch-no-plain", action="store_true",
                    help="time the batch only, not the loop of plain solves (runs under counters)")
    ap.add_argument("--batch-no-tune", action="store_true",
                    help="skip the batch autotuner: the automatic policy's engine at the default layout "
                         "(the resident engine when the batch fits it; runs under counters)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served request-stream measurement")
    ap.add_argument("--serve-window", type=float, default=60.0,
                    help="arrival window (s) of the served stream at the specified rate of 200 requests/s")
    ap.add_argument("--serve-deadline-ms", type=float, default=2000.0,
                    help="load shedding: requests whose projected completion exceeds this are refused at submit")
    ap.add_argument("--lanes", type=int, default=-1,
                    help="replica layout (lanes per row); -1 = autotune before timing, 0 = default")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB elementwise copy three times (reference for HBM byte counters)")
    ap.add_argument("--engine", default="auto", choices=["auto", "stream", "sliced", "compact", "persistent", "lds_block"],
                    help="engine policy of the solving context")
    ap.add_argument("--updates", type=int, default=0,
                    help="override the updates per solve (short runs under hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this library runs on a "
              "single GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.rand(512 * 1024 * 1024 // 4, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        print("copy calibration: 3 x (read 512 MiB, write 512 MiB)", flush=True)
        return
    import paper_2409_02135_amd as q

    m = measure(q, args.workload, args.steps, args.warmup, args.lanes, args.engine, args.updates)
    out = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["elapsed"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": m["config"],
        "latency_ms": m["latency_ms"],
        "roofline": m["roofline"],
        "quality": m["quality"],
    }
    default_run = args.workload == DEFAULT and args.updates == 0 and args.engine == "auto"
    if default_run and not args.no_configs:
        out["configs"] = {}
        for w, st, wu, oupd in CONFIG_BLOCKS:
            out["configs"][w] = config_block(q, w, st, wu, oupd, not args.no_cpu_baseline)
    if not args.no_batch:
        out["batched_vs_plain"] = batched_vs_plain(q, K=args.batch_updates, plain=not args.batch_no_plain,
                                                   with_cpu=not args.no_cpu_baseline, tune=not args.batch_no_tune)
    if not args.no_serve:
        pool = graph_pool(24)
        spec = served(q, 200.0, args.serve_window, pool, seed=1, deadline_ms=args.serve_deadline_ms)
        # a second stream at about 70 % of the capacity the first one sustained, unshed
        mean_work = spec["offered"]["updates_per_s"] / 200.0
        rate70 = max(1.0, 0.7 * spec["sustained_updates_per_s"] / mean_work)
        low = served(q, rate70, 8.0, pool, seed=2)
        out["served"] = {"workload": "Poisson stream of MIS / +-1 max-cut requests on ER (mean degree U[3,20]) "
                                     "and BA (m=4) graphs, n log-uniform in [1e3,1e5], S in {32,128}, "
                                     "1000-3000 updates", "at_200_per_s": spec, "at_70pct_capacity": low}
    if not args.no_cpu_baseline:
        g, problem, S, K, colors = m["graph"], m["problem"], m["S"], m["K"], m["colors"]
        out["cpu_baseline"] = (cpu_baseline_coloring(g, colors, S, K, updates=5 if g["n"] > 10000 else 20)
                               if problem == "coloring" else
                               cpu_baseline(g, problem, S, K, updates=3 if m["dense"] else 20))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
