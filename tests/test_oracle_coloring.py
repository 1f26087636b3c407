"""Pins of the oracle's categorical K-state variant (appendix "Generalization to discrete
optimization problems", "Transformation for general discrete variables"; coloring energy of
the appendix "Energy Function of Benchmark Problems"): the K = 2 reduction of the entropy to
the binary alpha-entropy (the appendix proposition), the entropy's extremes, the energy at
one-hot points against the conflict count, exact evaluation against brute force and textbook
chromatic numbers, central finite differences through the Clamp-normalisation, and the
scale invariance of sigma along each row.  CPU only."""

import itertools

import numpy as np
import pytest

import qqa_inputs as qi


def onehot(colors, K):
    n, S = colors.shape
    V = np.zeros((n, K, S))
    for s in range(S):
        V[np.arange(n), colors[:, s], s] = 1.0
    return V


def conflicts_direct(g, col):
    rows = np.repeat(np.arange(g["n"]), np.diff(g["row_ptr"]))
    keep = rows < g["col"]
    return int(np.sum(col[rows[keep]] == col[g["col"][keep]]))


def test_queens_graphs_match_paper_statistics():
    # node and edge counts of the queens graphs in the appendix's coloring statistics table
    for n, edges in ((5, 160), (6, 290), (7, 476), (8, 728), (9, 1056)):
        g = qi.queens(n)
        assert g["n"] == n * n and g["col"].size == 2 * edges


def test_entropy_k2_reduces_to_binary_alpha_entropy(orc):
    # appendix proposition: s_2(sigma) = s(p) with sigma = (p, 1 - p)
    rng = np.random.default_rng(0)
    n, S = 7, 3
    p = rng.random((n, S))
    sigma = np.stack([p, 1 - p], axis=1)
    s2 = orc.cat_entropy(sigma, 4)
    g = qi.complete_bipartite(0, n)  # no edges: the binary energy is -sum p + gamma s(p)
    pr = orc.Params(comm_alpha=0.0, lam=0.0)
    for s in range(S):
        sb = orc.energy(pr, g, p[:, [s]], 1.0) - orc.energy(pr, g, p[:, [s]], 0.0)
        assert s2[s] == pytest.approx(sb, abs=1e-12)


@pytest.mark.parametrize("K", [2, 3, 5, 11])
def test_entropy_extremes(orc, K):
    # maximum N at sigma = 1/K, zero at every one-hot point
    n, S = 6, 2
    uniform = np.full((n, K, S), 1.0 / K)
    assert orc.cat_entropy(uniform, 4) == pytest.approx([n] * S, abs=1e-12)
    rng = np.random.default_rng(K)
    col = rng.integers(0, K, (n, S))
    assert orc.cat_entropy(onehot(col, K), 4) == pytest.approx([0.0] * S, abs=1e-12)
    for _ in range(10):
        sg, _ = orc.cat_sigma(rng.random((n, K, S)))
        assert np.all(orc.cat_entropy(sg, 4) <= n + 1e-12)


def test_energy_at_onehot_points_is_conflict_count(orc):
    g = qi.cycle(7)
    K = 3
    pr = orc.Params(comm_alpha=0.0)
    for col in itertools.islice(itertools.product(range(K), repeat=7), 0, 3 ** 7, 53):
        c = np.array(col)[:, None]
        e = orc.cat_energy(pr, g, onehot(c, K), gamma_value=0.7)
        assert e == pytest.approx(conflicts_direct(g, c[:, 0]), abs=1e-12)


@pytest.mark.parametrize("graph,K,best", [
    (lambda: qi.cycle(5), 2, 1), (lambda: qi.cycle(5), 3, 0), (lambda: qi.complete(4), 3, 1),
    (lambda: qi.complete(4), 4, 0), (lambda: qi.petersen(), 2, 3), (lambda: qi.petersen(), 3, 0)])
def test_eval_brute_force_minimum(orc, graph, K, best):
    g = graph()
    n = g["n"]
    cols = np.array(list(itertools.product(range(K), repeat=n))).T  # (n, K^n)
    V = onehot(cols, K)
    ev = orc.cat_eval(g, V)
    assert np.array_equal(ev["colors"], cols)
    for s in range(0, cols.shape[1], 97):
        assert ev["conflicts"][s] == conflicts_direct(g, cols[:, s])
    assert ev["conflicts"].min() == best
    assert ev["conflicts"][ev["best"]] == best


def test_eval_argmax_first_maximum(orc):
    g = qi.cycle(3)
    V = np.array([[0.2, 0.7, 0.7], [1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])[:, :, None]
    ev = orc.cat_eval(g, V)
    assert list(ev["colors"][:, 0]) == [1, 0, 0]


@pytest.mark.parametrize("K", [2, 3, 5])
def test_gradient_matches_central_differences(orc, K):
    g = qi.erdos_renyi(9, 4.0, 2)
    rng = np.random.default_rng(3)
    S = 3
    V = rng.uniform(0.05, 0.95, (9, K, S))
    pr = orc.Params(comm_alpha=0.3)
    gamma = -0.6
    gV, _ = orc.cat_grad(pr, g, V, gamma)
    h = 1e-6
    for i in range(9):
        for k in range(K):
            for s in range(S):
                Vp, Vm = V.copy(), V.copy()
                Vp[i, k, s] += h
                Vm[i, k, s] -= h
                fd = (orc.cat_energy(pr, g, Vp, gamma) - orc.cat_energy(pr, g, Vm, gamma)) / (2 * h)
                assert gV[i, k, s] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_gradient_is_orthogonal_to_each_row(orc):
    # sigma(c V_i) = sigma(V_i): R does not change along V_i, so sum_k V_ik dR/dV_ik = 0
    g = qi.queens(5)
    rng = np.random.default_rng(4)
    V = rng.uniform(0.1, 1.0, (25, 5, 4))
    gV, _ = orc.cat_grad(orc.Params(comm_alpha=0.2), g, V, 0.3)
    assert np.max(np.abs(np.sum(V * gV, axis=1))) < 1e-12


def test_solve_finds_proper_colorings(orc):
    # heuristic pin: the paper reports zero conflicts on queen5-5 with 5 colours
    r = orc.cat_solve(orc.Params(), qi.queens(5), 5, 16, 1000, 0)
    assert r["conflicts"].min() == 0
    r = orc.cat_solve(orc.Params(), qi.petersen(), 3, 8, 500, 1)
    assert r["conflicts"].min() == 0
