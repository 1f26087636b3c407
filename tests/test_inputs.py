"""Property tests of the seeded synthetic instance generators.  CPU only."""

import numpy as np
import pytest

import qqa_inputs as qi


def check_simple_symmetric(g):
    n = g["n"]
    rp, col = g["row_ptr"], g["col"]
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(rows != col), "self-loop"
    key = rows.astype(np.int64) * n + col
    assert np.unique(key).size == key.size, "duplicate"
    tkey = col.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(key), np.sort(tkey)), "asymmetric"
    if g["weight"] is not None:
        w = dict(zip(key.tolist(), g["weight"].tolist()))
        assert all(w[k] == w[int(t)] for k, t in zip(key.tolist(), tkey.tolist()))


def test_random_regular():
    g = qi.random_regular(256, 3, 0)
    check_simple_symmetric(g)
    assert np.all(np.diff(g["row_ptr"]) == 3)
    g2 = qi.random_regular(256, 3, 0)
    assert np.array_equal(g["col"], g2["col"])
    assert not np.array_equal(g["col"], qi.random_regular(256, 3, 1)["col"])


def test_erdos_renyi_edge_count():
    n, d = 20000, 5.0
    g = qi.erdos_renyi(n, d, 0)
    check_simple_symmetric(g)
    m = g["col"].size // 2
    mean = n * d / 2
    assert abs(m - mean) < 3 * np.sqrt(mean)
    iso = np.sum(np.diff(g["row_ptr"]) == 0)
    assert abs(iso - n * np.exp(-d)) < 5 * np.sqrt(n * np.exp(-d))


def test_barabasi_albert_edge_count_and_tail():
    n, m = 5000, 4
    g = qi.barabasi_albert(n, m, 0)
    check_simple_symmetric(g)
    assert g["col"].size // 2 == m * (m + 1) // 2 + m * (n - m - 1)
    deg = np.diff(g["row_ptr"])
    assert deg.min() >= m and deg.max() > 10 * m


def test_pm1_and_dense_weights():
    g = qi.pm1_weights(qi.erdos_renyi(500, 6.0, 1), 2)
    check_simple_symmetric(g)
    assert set(np.unique(g["weight"]).tolist()) <= {-1.0, 1.0}
    W = qi.dense_gaussian(256, 3)
    assert W.dtype == np.float32 and np.array_equal(W, W.T) and np.all(np.diag(W) == 0)
    q = W.astype(np.float64) * 65536
    assert np.array_equal(q, np.rint(q)) and np.abs(W).max() < 8
    assert abs(W[np.triu_indices(256, 1)].std() - 1) < 0.02


def test_textbook_graphs():
    for g in [qi.petersen(), qi.cycle(7), qi.complete(5), qi.complete_bipartite(3, 4)]:
        check_simple_symmetric(g)
    assert qi.petersen()["col"].size == 30


def test_batch_and_requests_deterministic():
    a = qi.instance_batch(4, 9, n_range=(200, 400))
    b = qi.instance_batch(4, 9, n_range=(200, 400))
    for x, y in zip(a, b):
        assert x["n"] == y["n"] and np.array_equal(x["col"], y["col"])
        check_simple_symmetric(x)
    reqs = qi.poisson_requests(200.0, 2.0, 0)
    assert 300 < len(reqs) < 500
    assert all(1000 <= r["n"] <= 100000 for r in reqs)
    t = [r["arrival"] for r in reqs]
    assert t == sorted(t)


@pytest.mark.parametrize("bad", ["loop", "dup"])
def test_csr_from_edges_rejects(bad):
    e = np.array([[0, 0]]) if bad == "loop" else np.array([[0, 1], [1, 0]])
    with pytest.raises(ValueError):
        qi.csr_from_edges(3, e)


def test_rb_model_structure():
    """Model RB compatibility graph: symmetric CSR without self-loops, no edge between two
    values of one variable, the planted assignment is a clique, so the clique number is
    exactly the number of variables; seeded."""
    import itertools
    g = qi.rb_model(12, 6, 2.6, 0.25, 3)
    n = g["n"]
    assert n == 72
    A = np.zeros((n, n), bool)
    rows = np.repeat(np.arange(n), np.diff(g["row_ptr"]))
    A[rows, g["col"]] = True
    assert np.array_equal(A, A.T) and not A.diagonal().any()
    var = np.arange(n) // 6
    assert not (A & (var[:, None] == var[None, :])).any()
    pc = g["planted_clique"]
    assert len(set(var[pc])) == 12 and all(A[i, j] for i, j in itertools.combinations(pc, 2))
    # constraints removed some cross-variable pairs
    assert A.sum() < (n * n - 12 * 36)
    h = qi.rb_model(12, 6, 2.6, 0.25, 3)
    assert np.array_equal(h["col"], g["col"]) and np.array_equal(h["row_ptr"], g["row_ptr"])


def test_random_regular_swapped_is_simple_and_regular():
    for n, d, seed in ((500, 20, 0), (2000, 40, 1), (64, 7 + 1, 2)):
        g = qi.random_regular_swapped(n, d, seed)
        deg = np.diff(g["row_ptr"])
        assert deg.min() == d and deg.max() == d
        rows = np.repeat(np.arange(n), deg)
        assert not np.any(rows == g["col"])
        key = rows * n + g["col"]
        assert np.unique(key).size == key.size
        h = qi.random_regular_swapped(n, d, seed)
        assert np.array_equal(h["col"], g["col"])
