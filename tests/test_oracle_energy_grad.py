"""Pins of the oracle's relaxed energy R^ and its gradient: values at binary points,
closed forms at P = 1/2 and for the STD maximiser, central finite differences of every
term.  CPU only."""

import json
import math
import os

import numpy as np
import pytest

import qqa_inputs as qi

MIS, MAXCUT = 0, 1
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def params(orc, **kw):
    return orc.Params(**kw)


def test_energy_at_binary_points_is_discrete_objective(orc):
    # the relaxation agrees with l(x) on {0,1}^N; the entropy vanishes there
    g = qi.erdos_renyi(9, 3.0, 1)
    X = ((np.arange(2 ** 9)[None, :] >> np.arange(9)[:, None]) & 1).astype(np.float64)
    ev = orc.evaluate(MIS, 2, g, X)
    for s in range(0, 2 ** 9, 37):
        e = orc.energy(params(orc, comm_alpha=0.0), g, X[:, [s]], gamma_value=-3.0)
        assert e == pytest.approx(ev["obj"][s], abs=1e-12)
    gw = qi.pm1_weights(g, 4)
    ev = orc.evaluate(MAXCUT, 0, gw, X)
    for s in range(0, 2 ** 9, 41):
        e = orc.energy(params(orc, problem=MAXCUT, comm_alpha=0.0), gw, X[:, [s]], 0.7)
        assert e * 65536 == pytest.approx(ev["obj"][s], abs=1e-9)


def test_entropy_closed_forms(orc):
    # s(1/2) = N is the maximum, s(x) = 0 at binary x (Eq. 7)
    g = qi.complete_bipartite(0, 6)  # six isolated nodes: l^ = -sum p for MIS
    n = g["n"]
    half = np.full((n, 1), 0.5)
    pr = params(orc, comm_alpha=0.0, lam=0.0)
    e0 = orc.energy(pr, g, half, 0.0)
    assert e0 == pytest.approx(-n / 2)
    assert orc.energy(pr, g, half, 1.5) - e0 == pytest.approx(1.5 * n)
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = rng.random((n, 1))
        # gamma * s(P) < gamma * s(1/2) for gamma > 0 unless P = 1/2
        assert orc.energy(pr, g, P, 1.0) - orc.energy(pr, g, P, 0.0) < n
    assert GOLD["alpha_entropy_exponent"]["value"] == 4


@pytest.mark.parametrize("S", [2, 4, 8, 16, 3, 5, 7, 9])
def test_std_term_maximiser_proposition(orc, S):
    """Appendix proposition: sum_i STD is maximal with S/2 zeros and S/2 ones per row;
    maximum variance 1/4 (even S), (S^2-1)/(4 S^2) (odd S)."""
    n = 3
    g = qi.complete_bipartite(0, n)
    pr = params(orc, comm_alpha=1.0, lam=0.0)
    row = np.array([0.0] * (S // 2) + [1.0] * (S - S // 2))
    P = np.tile(row, (n, 1))
    base = orc.energy(params(orc, comm_alpha=0.0, lam=0.0), g, P, 0.0)
    std_sum = -(orc.energy(pr, g, P, 0.0) - base) / S
    var = GOLD["std_max_variance_even_S"]["value"] if S % 2 == 0 else (S * S - 1) / (4 * S * S)
    assert std_sum == pytest.approx(n * math.sqrt(var), rel=1e-12)
    rng = np.random.default_rng(S)
    for _ in range(200):
        Q = rng.random((n, S))
        if rng.random() < 0.5:
            Q = np.round(Q)
        b = orc.energy(params(orc, comm_alpha=0.0, lam=0.0), g, Q, 0.0)
        assert -(orc.energy(pr, g, Q, 0.0) - b) / S <= std_sum + 1e-12


def _fd(orc, pr, g, P, gam, h=1e-6, picks=24, seed=0):
    rng = np.random.default_rng(seed)
    n, S = P.shape
    out = []
    for _ in range(picks):
        i, s = int(rng.integers(n)), int(rng.integers(S))
        Pp, Pm = P.copy(), P.copy()
        Pp[i, s] += h
        Pm[i, s] -= h
        out.append((i, s, (orc.energy(pr, g, Pp, gam) - orc.energy(pr, g, Pm, gam)) / (2 * h)))
    return out


def interior_state(n, S, seed):
    rng = np.random.default_rng(seed)
    return 0.1 + 0.8 * rng.random((n, S))


CASES = {
    "mis_er": (MIS, lambda: qi.erdos_renyi(30, 4.0, 2)),
    "maxcut_ba_pm1": (MAXCUT, lambda: qi.pm1_weights(qi.barabasi_albert(30, 3, 3), 5)),
    "maxcut_dense": (MAXCUT, lambda: qi.dense_gaussian(12, 9)),
}


@pytest.mark.parametrize("case", ["mis_er", "maxcut_ba_pm1", "maxcut_dense"])
@pytest.mark.parametrize("term", ["objective", "entropy", "communication", "total"])
def test_gradient_matches_finite_differences(orc, case, term):
    problem, make = CASES[case]
    g = make()
    n = g.shape[0] if isinstance(g, np.ndarray) else g["n"]
    S = 6
    P = interior_state(n, S, 11)
    kw = dict(problem=problem)
    gam = -1.7
    if term == "objective":
        kw.update(comm_alpha=0.0); gam = 0.0
    elif term == "entropy":
        kw.update(comm_alpha=0.0, lam=0.0)
        if problem == MAXCUT:
            g = qi.complete_bipartite(0, n)
    elif term == "communication":
        kw.update(comm_alpha=0.37, lam=0.0); gam = 0.0
        if problem == MAXCUT:
            g = qi.complete_bipartite(0, n)
    else:
        kw.update(comm_alpha=0.37)
    pr = params(orc, **kw)
    gf, ge, gc, sigma = orc.grad(pr, g, P, gam)
    if term == "objective":
        G = gf
    elif term == "entropy":
        G = ge + (gf if problem == MIS else 0)  # lam = 0: MIS gf is the constant -1
    elif term == "communication":
        G = gc + (gf if problem == MIS else 0)
    else:
        G = gf + ge + gc
    for i, s, fd in _fd(orc, pr, g, P, gam):
        assert G[i, s] == pytest.approx(fd, rel=1e-6, abs=1e-6), (i, s)


def test_communication_gradient_rows_sum_to_zero_and_sigma_zero_rule(orc):
    g = qi.cycle(5)
    pr = params(orc, comm_alpha=0.5)
    P = interior_state(5, 8, 3)
    P[2, :] = 0.25  # all replicas equal: sigma = 0, gradient defined as 0
    gf, ge, gc, sigma = orc.grad(pr, g, P, 0.0)
    assert np.all(np.abs(gc.sum(1)) < 1e-12)
    assert sigma[2] == 0.0 and np.all(gc[2] == 0.0)
    assert np.all(np.isfinite(gc))
    # |gc| <= alpha_c sqrt(S - 1)
    assert np.abs(gc).max() <= 0.5 * math.sqrt(7) + 1e-12


@pytest.mark.parametrize("problem", [MIS, MAXCUT])
def test_gradient_at_half_is_objective_gradient(orc, problem):
    """At P = 1/2 the entropy gradient vanishes (odd power of 0) and every row has
    sigma = 0, so the total gradient is that of l^: deg_i - 1 for MIS with lambda = 2,
    zero for max-cut."""
    g = qi.erdos_renyi(40, 5.0, 6)
    if problem == MAXCUT:
        g = qi.pm1_weights(g, 1)
    P = np.full((40, 4), 0.5)
    gf, ge, gc, sigma = orc.grad(params(orc, problem=problem, comm_alpha=0.3), g, P, -7.0)
    total = gf + ge + gc
    deg = np.diff(g["row_ptr"]).astype(np.float64)
    want = (deg - 1)[:, None] * np.ones((1, 4)) if problem == MIS else np.zeros((40, 4))
    assert np.array_equal(total, want)


def test_negative_gamma_entropy_term_minimised_at_half(orc):
    # for gamma < 0, gamma * s(P) has its unique minimum at P = 1/2
    g = qi.complete_bipartite(0, 5)
    pr = params(orc, comm_alpha=0.0, lam=0.0)
    half = orc.energy(pr, g, np.full((5, 1), 0.5), -2.0) - orc.energy(pr, g, np.full((5, 1), 0.5), 0.0)
    rng = np.random.default_rng(1)
    for _ in range(100):
        P = rng.random((5, 1))
        val = orc.energy(pr, g, P, -2.0) - orc.energy(pr, g, P, 0.0)
        assert val > half
