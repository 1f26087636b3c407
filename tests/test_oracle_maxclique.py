"""Pins of the oracle's max-clique energy (appendix "Energy Function of Benchmark Problems",
Max Clique): exact evaluation against brute force over every x of small graphs and
textbook clique numbers, the relaxed energy at binary points and in closed form, central
finite differences of the gradient, and the complement-graph identity
    gf_clique(G)_i = gf_MIS(complement of G)_i + lambda (p_i - 1/2),
which goes through the oracle's MIS branch on a different graph.  CPU only."""

import itertools

import numpy as np
import pytest

import qqa_inputs as qi

MIS, MAXCUT, MAXCLIQUE = 0, 1, 2


def adjacency(g):
    n = g["n"]
    A = np.zeros((n, n), np.int64)
    rows = np.repeat(np.arange(n), np.diff(g["row_ptr"]))
    A[rows, g["col"]] = 1
    return A


def complement(g):
    A = adjacency(g)
    n = g["n"]
    comp = 1 - A - np.eye(n, dtype=np.int64)
    return qi.dense_to_csr(comp.astype(np.float32))


def all_x(n):
    return ((np.arange(2 ** n)[None, :] >> np.arange(n)[:, None]) & 1).astype(np.float64)


def brute_clique_number(A):
    n = A.shape[0]
    best = 0
    for k in range(n, 0, -1):
        for sub in itertools.combinations(range(n), k):
            if all(A[i, j] for i, j in itertools.combinations(sub, 2)):
                return k
    return best


def nonadjacent_selected_pairs(A, x):
    sel = np.nonzero(x)[0]
    return sum(1 for i, j in itertools.combinations(sel, 2) if not A[i, j])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_eval_counts_nonadjacent_pairs_and_minimum_is_clique_number(orc, seed):
    g = qi.erdos_renyi(10, 5.0, seed)
    A = adjacency(g)
    X = all_x(10)
    ev = orc.evaluate(MAXCLIQUE, 2, g, X)
    for s in range(0, X.shape[1], 7):
        x = X[:, s].astype(int)
        v = nonadjacent_selected_pairs(A, x)
        assert ev["size_or_cut"][s] == x.sum()
        assert ev["viol"][s] == v
        assert ev["obj"][s] == -x.sum() + 2 * v
    # with lambda = 2 every infeasible x is improved by dropping a node, so the minimum
    # of l over {0,1}^N is minus the clique number
    omega = brute_clique_number(A)
    assert ev["obj"].min() == -omega
    b = ev["best"]
    assert ev["viol"][b] == 0 and ev["size_or_cut"][b] == omega


@pytest.mark.parametrize("graph,omega", [
    (lambda: qi.complete(6), 6), (lambda: qi.petersen(), 2), (lambda: qi.cycle(5), 2),
    (lambda: qi.cycle(3), 3), (lambda: qi.complete_bipartite(3, 4), 2), (lambda: qi.complete_bipartite(0, 5), 1)])
def test_textbook_clique_numbers(orc, graph, omega):
    g = graph()
    X = all_x(g["n"])
    ev = orc.evaluate(MAXCLIQUE, 2, g, X)
    assert ev["obj"].min() == -omega


def test_energy_at_binary_points_is_discrete_objective(orc):
    g = qi.erdos_renyi(9, 4.0, 3)
    X = all_x(9)
    ev = orc.evaluate(MAXCLIQUE, 2, g, X)
    pr = orc.Params(problem=MAXCLIQUE, comm_alpha=0.0)
    for s in range(0, X.shape[1], 29):
        assert orc.energy(pr, g, X[:, [s]], gamma_value=-1.5) == pytest.approx(ev["obj"][s], abs=1e-12)


def test_energy_closed_form_complete_graph_at_half(orc):
    # K_n, p = 1/2: 1^T p = n/2, p^T A p = n(n-1)/4, so l = -n/2 + (lambda/2)(-n/4)
    n, lam = 7, 2.0
    g = qi.complete(n)
    P = np.full((n, 1), 0.5)
    pr = orc.Params(problem=MAXCLIQUE, comm_alpha=0.0, lam=lam)
    assert orc.energy(pr, g, P, 0.0) == pytest.approx(-n / 2 - lam * n / 8, abs=1e-12)


@pytest.mark.parametrize("dense", [False, True])
def test_gradient_matches_central_differences(orc, dense):
    g = qi.erdos_renyi(12, 6.0, 4)
    rng = np.random.default_rng(5)
    S = 3
    P = rng.uniform(0.05, 0.95, (g["n"], S))
    pr = orc.Params(problem=MAXCLIQUE, comm_alpha=0.3, lam=2.0)
    G = orc.graph(W=adjacency(g).astype(np.float64)) if dense else g
    gamma = -0.7
    gf, ge, gc, _ = orc.grad(pr, G, P, gamma)
    total = gf + ge + gc
    h = 1e-6
    for i in range(g["n"]):
        for s in range(S):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, s] += h
            Pm[i, s] -= h
            fd = (orc.energy(pr, G, Pp, gamma) - orc.energy(pr, G, Pm, gamma)) / (2 * h)
            assert total[i, s] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_gradient_equals_mis_gradient_on_complement(orc):
    g = qi.erdos_renyi(15, 7.0, 6)
    gc_ = complement(g)
    rng = np.random.default_rng(7)
    P = rng.random((g["n"], 5))
    lam = 2.0
    gf_clique, _, _, _ = orc.grad(orc.Params(problem=MAXCLIQUE, lam=lam), g, P, 0.0)
    gf_mis, _, _, _ = orc.grad(orc.Params(problem=MIS, lam=lam), gc_, P, 0.0)
    assert np.allclose(gf_clique, gf_mis + lam * (P - 0.5), rtol=0, atol=1e-12)


def test_step_uses_column_sums(orc):
    # one update from a state where only one replica differs: the other replicas' column
    # sums, hence their updates, must not change
    g = qi.erdos_renyi(20, 6.0, 8)
    rng = np.random.default_rng(9)
    P = rng.random((20, 4))
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    pr = orc.Params(problem=MAXCLIQUE, comm_alpha=0.0)
    a = orc.step(pr, g, 3, 100, 1, P, m, v)
    P2 = P.copy()
    P2[5, 2] = 1.0 - P2[5, 2]
    b = orc.step(pr, g, 3, 100, 1, P2, m, v)
    for s in (0, 1, 3):
        assert np.array_equal(a["P"][:, s], b["P"][:, s])
    assert not np.array_equal(a["P"][:, 2], b["P"][:, 2])
