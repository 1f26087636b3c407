"""Pins of the oracle's update (orc_step / orc_run): the AdamW first-step closed form,
projected gradient descent, the fixed point on a regular graph (closed-form root), the
linear schedule's endpoints and the injected noise.  CPU only."""

import numpy as np
import pytest
from scipy import optimize, stats

import qqa_inputs as qi

MIS, MAXCUT = 0, 1
ADAMW, LANGEVIN = 0, 1


def test_schedule_endpoints(orc):
    pr = orc.Params(gamma_min=-2.0, gamma_max=0.1)
    assert orc.gamma(pr, 0, 3000) == -2.0
    assert orc.gamma(pr, 2999, 3000) == pytest.approx(0.1, abs=1e-15)
    assert orc.gamma(pr, 1500, 3001) == pytest.approx(-0.95, abs=1e-15)
    assert orc.gamma(pr, 0, 1) == -2.0


def test_adamw_first_step_closed_form(orc):
    """k = 1: m = (1-b1) g, v = (1-b2) g^2, so the update is
    p' = p (1 - eta wd) - eta g / (|g| + eps), before noise and clamp."""
    g = qi.erdos_renyi(50, 4.0, 0)
    pr = orc.Params(temperature=0.0, lr=0.01, comm_alpha=0.2)
    rng = np.random.default_rng(2)
    P = 0.2 + 0.6 * rng.random((50, 8))
    z = np.zeros_like(P)
    out = orc.step(pr, g, 0, 100, 7, P, z, z)
    gam = orc.gamma(pr, 0, 100)
    gf, ge, gc, _ = orc.grad(pr, g, P, gam)
    G = gf + ge + gc
    want = P * (1 - pr.lr * pr.weight_decay) - pr.lr * G / (np.abs(G) + pr.adam_eps)
    np.testing.assert_allclose(out["P"], want, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["m"], (1 - pr.beta1) * G, rtol=1e-14, atol=0)
    np.testing.assert_allclose(out["v"], (1 - pr.beta2) * G * G, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(out["g"], G)


def test_adamw_bias_correction_at_step_k(orc):
    """At update index t (k = t + 1) with given moments, the step uses m/(1-b1^k) and
    v/(1-b2^k)."""
    g = qi.cycle(6)
    pr = orc.Params(temperature=0.0, lr=0.05)
    rng = np.random.default_rng(3)
    P = 0.3 + 0.4 * rng.random((6, 4))
    m0 = rng.standard_normal((6, 4))
    v0 = rng.random((6, 4)) + 0.1
    t = 9
    out = orc.step(pr, g, t, 50, 1, P, m0, v0)
    gf, ge, gc, _ = orc.grad(pr, g, P, orc.gamma(pr, t, 50))
    G = gf + ge + gc
    m1 = pr.beta1 * m0 + (1 - pr.beta1) * G
    v1 = pr.beta2 * v0 + (1 - pr.beta2) * G * G
    k = t + 1
    want = P * (1 - pr.lr * pr.weight_decay) - pr.lr * (m1 / (1 - pr.beta1 ** k)) / (
        np.sqrt(v1 / (1 - pr.beta2 ** k)) + pr.adam_eps)
    np.testing.assert_allclose(out["P"], np.clip(want, 0, 1), atol=1e-13)


def test_langevin_without_noise_is_projected_gradient_descent(orc):
    g = qi.pm1_weights(qi.barabasi_albert(40, 3, 1), 2)
    pr = orc.Params(problem=MAXCUT, rule=LANGEVIN, temperature=0.0, lr=0.1, comm_alpha=0.1)
    rng = np.random.default_rng(4)
    P = rng.random((40, 8))
    out = orc.step(pr, g, 3, 10, 0, P, np.zeros_like(P), np.zeros_like(P))
    gf, ge, gc, _ = orc.grad(pr, g, P, orc.gamma(pr, 3, 10))
    np.testing.assert_allclose(out["P"], np.clip(P - 0.1 * (gf + ge + gc), 0, 1), atol=1e-14)
    np.testing.assert_allclose(out["pre_clamp"], P - 0.1 * (gf + ge + gc), atol=1e-14)


@pytest.mark.parametrize("gamma_fixed,expected", [(-2.0, 0.310907), (-20.0, 0.3974)])
def test_regular_graph_fixed_point(orc, gamma_fixed, expected):
    """On a d-regular graph with all variables equal, projected gradient descent at fixed
    gamma stays uniform and converges to the root of
        -1 + lambda d p - 2 alpha gamma (2p - 1)^(alpha - 1) = 0."""
    d, lam, alpha = 3, 2.0, 4
    root = optimize.brentq(lambda p: -1 + lam * d * p - 2 * alpha * gamma_fixed * (2 * p - 1) ** (alpha - 1), 0.0, 0.5,
                           xtol=1e-15)
    assert root == pytest.approx(expected, abs=1e-4)
    g = qi.complete(4)  # K4 is 3-regular
    pr = orc.Params(rule=LANGEVIN, temperature=0.0, comm_alpha=0.3, lr=0.01,
                    gamma_min=gamma_fixed, gamma_max=gamma_fixed)
    P = np.full((4, 5), 0.8)
    P, _, _ = orc.run(pr, g, 0, 4000, 4000, 0, P, np.zeros_like(P), np.zeros_like(P))
    np.testing.assert_allclose(P, root, atol=1e-10)
    # as gamma -> -inf the fixed point approaches 1/2 like |gamma|^(-1/3)
    r1 = optimize.brentq(lambda p: -1 + 6 * p + 8 * 1e4 * (2 * p - 1) ** 3, 0, 0.5)
    r2 = optimize.brentq(lambda p: -1 + 6 * p + 8 * 8e4 * (2 * p - 1) ** 3, 0, 0.5)
    assert (0.5 - r1) / (0.5 - r2) == pytest.approx(2.0, rel=0.02)


def test_noise_injection_scale_and_distribution(orc):
    """Isolated MIS nodes have gradient -1 + ge + gc; with comm_alpha = 0 and gamma = 0 the
    update is p - eta*(-1) + sqrt(2 eta T) xi, so the residual exposes xi."""
    n, S = 2000, 16
    g = qi.complete_bipartite(0, n)
    pr = orc.Params(rule=LANGEVIN, temperature=0.5, lr=0.001, comm_alpha=0.0, gamma_min=0.0, gamma_max=0.0)
    P = np.full((n, S), 0.5)
    out = orc.step(pr, g, 4, 10, 123, P, np.zeros_like(P), np.zeros_like(P))
    xi = (out["pre_clamp"] - (P + pr.lr)) / np.sqrt(2 * pr.lr * pr.temperature)
    np.testing.assert_allclose(xi, orc.noise(123, n, S, 5), atol=1e-9)
    flat = xi.ravel()
    assert abs(flat.mean()) < 0.02 and abs(flat.var() - 1) < 0.03
    assert stats.kstest(flat, "norm").pvalue > 1e-3


def test_clamp_keeps_box(orc):
    g = qi.erdos_renyi(100, 6.0, 9)
    pr = orc.Params(lr=1.0, temperature=0.05)
    P = orc.init(1, 100, 8)
    P, m, v = orc.run(pr, g, 0, 20, 20, 1, P, np.zeros_like(P), np.zeros_like(P))
    assert P.min() >= 0.0 and P.max() <= 1.0
    assert np.any(P == 0.0) and np.any(P == 1.0)


def test_small_graph_quality_reaches_brute_force_optimum(orc):
    """Heuristic expectation (not a theorem): best-of-S on the Petersen graph and a few
    small random graphs finds the maximum independent set."""
    hits = 0
    for seed, g, alpha in [(0, qi.petersen(), 4), (1, qi.cycle(9), 4), (2, qi.complete_bipartite(3, 5), 5),
                           (3, qi.petersen(), 4), (4, qi.cycle(12), 6)]:
        r = orc.solve(orc.Params(), g, 16, 300, seed)
        hits += int(r["obj"][r["best"]] == -alpha and r["viol"][r["best"]] == 0)
    assert hits >= 4
