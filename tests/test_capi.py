"""CPU checks of the C ABI: the library loads, exports every function include/qqa.h
declares, and its host-only logic (defaults, strides, graph validation) behaves.  No
device work is started here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import qqa_inputs as qi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qqa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qqa_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def q():
    import paper_2409_02135_amd as q
    q.lib()
    return q


def test_every_declared_symbol_is_exported(q):
    names = declared_functions()
    assert len(names) >= 20
    L = C.CDLL(q.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_names_match_header(q):
    # the ctypes signature table covers every declared function
    import inspect
    src = inspect.getsource(q.lib)
    missing = [n for n in declared_functions() if f'"{n}"' not in src]
    assert not missing, missing


def test_replica_stride(q):
    for S, want in [(1, 4), (4, 4), (5, 8), (16, 16), (100, 100), (255, 256), (4096, 4096)]:
        assert q.qqa_replica_stride(S) == want
    assert q.qqa_replica_stride(0) == 0


def test_schedule_defaults_follow_the_paper(q):
    s = q.qqa_schedule_default("mis", 20000)
    assert (s.gamma_min, s.entropy_alpha, s.penalty_lambda) == (-2.0, 4, 2)
    assert s.gamma_max == pytest.approx(0.1) and s.weight_decay == pytest.approx(0.01)
    assert s.temperature == pytest.approx(1e-3)
    assert q.qqa_schedule_default("maxcut", 100000).gamma_min == -20.0
    assert q.qqa_schedule_default("maxcut", 125).gamma_min == -5.0


def test_valid_graphs_pass(q):
    for g, p in [(qi.erdos_renyi(500, 5.0, 0), "mis"), (qi.pm1_weights(qi.barabasi_albert(400, 4, 1), 2), "maxcut"),
                 (qi.complete_bipartite(0, 3), "mis")]:
        rc, msg = q.qqa_graph_validate(g, p)
        assert rc == 0, msg
    rc, msg = q.qqa_graph_validate(dense=qi.dense_gaussian(64, 0), problem="maxcut")
    assert rc == 0, msg


def _corrupt(kind):
    g = qi.erdos_renyi(50, 4.0, 3)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    if kind == "asymmetric":
        g["col"][0] = (g["col"][0] + 1) % 50 if (g["col"][0] + 1) % 50 != 0 else 2
    elif kind == "self_loop":
        row0 = 0
        while g["row_ptr"][row0 + 1] == g["row_ptr"][row0]:
            row0 += 1
        g["col"][g["row_ptr"][row0]] = row0
    elif kind == "out_of_range":
        g["col"][3] = 50
    elif kind == "negative_index":
        g["col"][3] = -1
    elif kind == "row_ptr_end":
        g["row_ptr"][-1] -= 1
    elif kind == "non_monotone":
        g["row_ptr"][10], g["row_ptr"][11] = g["row_ptr"][11] + 1, g["row_ptr"][10]
    elif kind == "n_zero":
        g["n"] = 0
    elif kind == "duplicate":
        e = qi.edge_list(g)
        e = np.concatenate([e, e[:1]])
        rows = np.concatenate([e[:, 0], e[:, 1]])
        cols = np.concatenate([e[:, 1], e[:, 0]])
        o = np.lexsort((cols, rows))
        g["col"] = cols[o].astype(np.int32)
        g["row_ptr"] = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=50))]).astype(np.int64)
    return g


@pytest.mark.parametrize("kind", ["asymmetric", "self_loop", "out_of_range", "negative_index", "row_ptr_end",
                                  "non_monotone", "n_zero", "duplicate"])
def test_invalid_graphs_rejected(q, kind):
    rc, msg = q.qqa_graph_validate(_corrupt(kind), "mis")
    assert rc == q.QQA_E_GRAPH and msg


def test_maxcut_weight_rules(q):
    g = qi.pm1_weights(qi.cycle(6), 0)
    g["weight"] = g["weight"].copy()
    g["weight"][0] = 0.3  # off the 2^-16 grid (and breaks symmetry)
    assert q.qqa_graph_validate(g, "maxcut")[0] == q.QQA_E_GRAPH
    g = qi.pm1_weights(qi.cycle(6), 0)
    e = qi.edge_list(g)
    g2 = qi.csr_from_edges(6, e, np.full(len(e), 200.0, np.float32))  # |w| >= 128
    assert q.qqa_graph_validate(g2, "maxcut")[0] == q.QQA_E_GRAPH
    g3 = qi.csr_from_edges(6, e, np.full(len(e), 3.25, np.float32))
    assert q.qqa_graph_validate(g3, "maxcut")[0] == 0
    # MIS ignores weights
    assert q.qqa_graph_validate(g2, "mis")[0] == 0
    W = qi.dense_gaussian(16, 1)
    W2 = W.copy()
    W2[0, 1] += 0.5
    assert q.qqa_graph_validate(dense=W2, problem="maxcut")[0] == q.QQA_E_GRAPH
    W3 = W.copy()
    W3[2, 2] = 1.0
    assert q.qqa_graph_validate(dense=W3, problem="maxcut")[0] == q.QQA_E_GRAPH
    assert q.qqa_graph_validate(dense=(W != 0).astype(np.float32), problem="mis")[0] == 0
    assert q.qqa_graph_validate(dense=W, problem="mis")[0] == q.QQA_E_GRAPH


def test_device_entry_points_refuse_host_and_short_buffers(q):
    # the binding checks every buffer a qqa_dev_* kernel would touch before any launch:
    # host memory, a wrong element type or too few elements never reach the device
    import torch
    n, S = 10, 5  # stride 8
    with pytest.raises(ValueError, match="device memory"):
        q.qqa_dev_init(0, n, S, torch.zeros(n, 8))
    with pytest.raises(ValueError, match="CUDA tensor"):
        q.qqa_dev_init(0, n, S, np.zeros((n, 8), np.float32))
    with pytest.raises(ValueError, match="dtype"):
        q.qqa_dev_init(0, n, S, torch.zeros(n, 8, dtype=torch.float64))
    with pytest.raises(ValueError, match="at least 80"):
        q.qqa_dev_init(0, n, S, torch.zeros(n * 8 - 1))
    g = q.DevGraph.__new__(q.DevGraph)
    g.n = n
    g.struct = q.qqa_dev_graph(n, 0, None, None, None, None)
    with pytest.raises(ValueError, match="P_in: 79 elements"):
        q.qqa_dev_step(g, "mis", None, S, 0, 10, 0, torch.zeros(79), torch.zeros(n, 8), None, None)
    with pytest.raises(ValueError, match="P: dtype"):
        q.qqa_dev_eval(g, "mis", 2, S, torch.zeros(n, 8, dtype=torch.int32), torch.zeros(S, dtype=torch.int64),
                       torch.zeros(S, dtype=torch.int64), torch.zeros(S, dtype=torch.int32),
                       torch.zeros(1, dtype=torch.int32))
