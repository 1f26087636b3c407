"""Pins of the oracle's rounding + exact evaluation (orc_eval) against brute force and
textbook optima.  CPU only."""

import itertools

import numpy as np
import pytest

import qqa_inputs as qi

MIS, MAXCUT = 0, 1


def dense_adj(g):
    n = g["n"]
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(g["row_ptr"]))
    w = np.ones(g["col"].size) if g["weight"] is None else g["weight"].astype(np.float64)
    A[rows, g["col"]] = w
    return A


def all_assignments(n):
    """P with one replica per x in {0,1}^n (replica s holds the bits of s)."""
    s = np.arange(2 ** n)
    return ((s[None, :] >> np.arange(n)[:, None]) & 1).astype(np.float64)


def quadratic_form_mis(A, X, lam=2.0):
    # l(x) = -c^T x + lambda x^T A x / 2 with c = 1 (the paper's MIS energy)
    return -X.sum(0) + lam * np.einsum("is,ij,js->s", X, A, X) / 2.0


def quadratic_form_maxcut(A, X):
    # l(x) = -sum_{(i,j) in E} A_ij (1 - (2x_i-1)(2x_j-1))/2; the full double sum counts
    # each undirected edge twice
    Z = 2 * X - 1
    return -0.25 * (A.sum() - np.einsum("is,ij,js->s", Z, A, Z))


GRAPHS = {
    "petersen": qi.petersen(),
    "c7": qi.cycle(7),
    "c8": qi.cycle(8),
    "k5": qi.complete(5),
    "k34": qi.complete_bipartite(3, 4),
    "er12": qi.erdos_renyi(12, 4.0, 3),
    "rrg12": qi.random_regular(12, 3, 5),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_mis_eval_equals_brute_force_everywhere(orc, name):
    g = GRAPHS[name]
    X = all_assignments(g["n"])
    r = orc.evaluate(MIS, 2, g, X)
    ref = quadratic_form_mis(dense_adj(g), X)
    assert np.array_equal(r["obj"], ref.astype(np.int64))
    assert np.array_equal(r["size_or_cut"], X.sum(0).astype(np.int64))
    # every global minimiser of l (lambda = 2) is an independent set
    best = r["obj"].min()
    assert np.all(r["viol"][r["obj"] == best] == 0)


@pytest.mark.parametrize("name,alpha", [("petersen", 4), ("c7", 3), ("c8", 4), ("k5", 1), ("k34", 4)])
def test_mis_textbook_independence_numbers(orc, name, alpha):
    g = GRAPHS[name]
    r = orc.evaluate(MIS, 2, g, all_assignments(g["n"]))
    assert r["obj"].min() == -alpha
    assert r["viol"][r["best"]] == 0 and r["obj"][r["best"]] == -alpha


@pytest.mark.parametrize("name,cut", [("c7", 6), ("c8", 8), ("k5", 6), ("k34", 12), ("petersen", 12)])
def test_maxcut_textbook_optima(orc, name, cut):
    g = GRAPHS[name]
    r = orc.evaluate(MAXCUT, 0, g, all_assignments(g["n"]))
    assert r["obj"].min() == -cut * 65536
    assert r["size_or_cut"].max() == cut * 65536


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weighted_maxcut_equals_brute_force(orc, seed):
    g = qi.pm1_weights(qi.erdos_renyi(11, 5.0, seed), seed + 10)
    X = all_assignments(g["n"])
    r = orc.evaluate(MAXCUT, 0, g, X)
    ref = quadratic_form_maxcut(dense_adj(g), X) * 65536
    assert np.array_equal(r["obj"], np.rint(ref).astype(np.int64))
    # cut(x) = cut(1 - x)
    s = np.arange(2 ** g["n"])
    assert np.array_equal(r["obj"], r["obj"][(2 ** g["n"] - 1) ^ s])


def test_dense_quantised_maxcut_exact(orc):
    W = qi.dense_gaussian(10, 7)
    X = all_assignments(10)
    r = orc.evaluate(MAXCUT, 0, orc.graph(W=W), X)
    q = np.rint(W.astype(np.float64) * 65536).astype(np.int64)
    Z = (X > 0.5).astype(np.int64)
    # integer brute force: sum over i<j of q_ij [x_i != x_j]
    diff = Z[:, None, :] != Z[None, :, :]
    ref = np.einsum("ij,ijs->s", np.triu(q, 1), diff.astype(np.int64))
    assert np.array_equal(r["size_or_cut"], ref)
    # dense and CSR views of the same instance agree
    r2 = orc.evaluate(MAXCUT, 0, qi.dense_to_csr(W), X)
    assert np.array_equal(r["obj"], r2["obj"])


def test_rounding_threshold_is_strict(orc):
    g = qi.cycle(4)
    P = np.array([[0.5, np.nextafter(0.5, 1.0), 0.0, 1.0]] * 4)
    r = orc.evaluate(MIS, 2, g, P)
    assert list(r["size_or_cut"]) == [0, 4, 0, 4]


def test_best_replica_prefers_feasible_then_objective_then_index(orc):
    g = qi.cycle(4)  # edges 0-1, 1-2, 2-3, 3-0
    cols = [
        [1, 1, 1, 1],  # infeasible, l = -4 + 2*4 = 4
        [1, 0, 0, 0],  # feasible, l = -1
        [1, 0, 1, 0],  # feasible, l = -2
        [0, 1, 0, 1],  # feasible, l = -2 (tie, larger index)
        [1, 1, 0, 0],  # infeasible, l = -2 + 2 = 0
    ]
    P = np.array(cols, dtype=np.float64).T
    r = orc.evaluate(MIS, 2, g, P)
    assert list(r["obj"]) == [4, -1, -2, -2, 0]
    assert r["best"] == 2
    # an all-infeasible set picks the lowest objective
    r = orc.evaluate(MIS, 2, g, P[:, [0, 4]])
    assert r["best"] == 1


def test_off_grid_weight_rejected(orc):
    g = qi.pm1_weights(qi.cycle(5), 0)
    g["weight"] = g["weight"] * np.float32(1.0 + 2.0 ** -20)
    with pytest.raises(ValueError):
        orc.evaluate(MAXCUT, 0, g, np.ones((5, 1)))
