"""Writes tests/golden/oracle_stats.json: the FP64 oracle's full-schedule results over
solver seeds 0..9 on the statistics workloads (the only code it runs is oracle/ and the
input generators).  Usage: python tests/golden/make_oracle_stats.py [--jobs 8] [--only NAME ...]
(--only recomputes the named workloads and keeps the stored results of the others)."""

from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

# name: (graph recipe, problem, S, steps); the RB recipe is
# ("rb", variables, domain size, r, p, graph seed, problem, S, steps)
WORKLOADS = {
    "rrg256_d3_mis_S16_K2000": ("rrg", 256, 3, 0, "mis", 16, 2000),
    "er2000_d5_mis_S256_K1000": ("er", 2000, 5.0, 0, "mis", 256, 1000),
    "ba2000_m4_pm1_maxcut_S128_K1000": ("ba", 2000, 4, 0, "maxcut", 128, 1000),
    "dense256_gauss_maxcut_S32_K500": ("dense", 256, 0, 0, "maxcut", 32, 500),
    "rb20x12_maxclique_S32_K1000": ("rb", 20, 12, 2.6, 0.25, 0, "maxclique", 32, 1000),
    # graph coloring: ("queens", board size, colours, graph seed, "coloring", S, steps)
    "queen7_colors7_S32_K1000": ("queens", 7, 7, 0, "coloring", 32, 1000),
}
PROBLEM_CODES = {"mis": 0, "maxcut": 1, "maxclique": 2}
SEEDS = list(range(10))


def make_graph(kind, n, d, gseed, problem):
    import qqa_inputs as qi
    if kind == "dense":
        return qi.dense_gaussian(n, gseed)
    if kind == "rrg":
        g = qi.random_regular(n, d, gseed)
    elif kind == "er":
        g = qi.erdos_renyi(n, d, gseed)
    else:
        g = qi.barabasi_albert(n, d, gseed)
    if problem == "maxcut":
        g = qi.pm1_weights(g, gseed + 1)
    return g


def one(args):
    name, seed = args
    import numpy as np
    import oracle
    import qqa_inputs as qi
    rec = WORKLOADS[name]
    if rec[0] == "queens":
        _, board, colors, _, _, S, K = rec
        r = oracle.cat_solve(oracle.Params().as_float32(), qi.queens(board), colors, S, K, seed)
        c = r["conflicts"]
        return name, seed, {"best_objective": int(c.min()), "best_feasible": bool(c.min() == 0),
                            "mean_objective": float(np.mean(c)), "feasible_fraction": float(np.mean(c == 0)),
                            "mean_size_or_cut": float(np.mean(c))}
    if rec[0] == "rb":
        _, nv, dom, r, p, gseed, problem, S, K = rec
        g = qi.rb_model(nv, dom, r, p, gseed)
        n = g["n"]
    else:
        kind, n, d, gseed, problem, S, K = rec
        g = make_graph(kind, n, d, gseed, problem)
        if kind == "dense":
            g = oracle.graph(W=g)
    pr = oracle.Params(problem=PROBLEM_CODES[problem],
                       gamma_min=-2.0 if problem != "maxcut" else (-20.0 if n >= 1000 else -5.0)).as_float32()
    r = oracle.solve(pr, g, S, K, seed)
    feas = r["viol"] == 0
    return name, seed, {
        "best_objective": int(r["obj"][r["best"]]),
        "best_feasible": bool(r["viol"][r["best"]] == 0),
        "mean_objective": float(np.mean(r["obj"])),
        "feasible_fraction": float(np.mean(feas)),
        "mean_size_or_cut": float(np.mean(r["size_or_cut"])),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--only", nargs="*", default=None, help="recompute only these workloads")
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_stats.json")
    names = list(WORKLOADS) if not args.only else args.only
    tasks = [(w, s) for w in names for s in SEEDS]
    out = {"_about": "FP64 oracle results per solver seed (default schedule, float32-rounded parameters); "
                     "written by tests/golden/make_oracle_stats.py",
           "workloads": {w: {"recipe": list(WORKLOADS[w]), "seeds": {}} for w in names}}
    if args.only and os.path.exists(path):
        kept = json.load(open(path))["workloads"]
        for w, v in kept.items():
            if w not in names and w in WORKLOADS:
                out["workloads"][w] = v
    with ProcessPoolExecutor(args.jobs) as ex:
        for name, seed, res in ex.map(one, tasks):
            out["workloads"][name]["seeds"][str(seed)] = res
            print(name, seed, res, flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
