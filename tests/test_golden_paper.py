"""The paper's printed numbers (tests/golden/paper_facts.json) against the
oracle and against exact arithmetic."""
import json
import math
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_newton_50_nests_is_2_pow_50_terms():
    g = GOLD["newton_50_nests"]
    assert g["series_terms"] == 2 ** g["nests"]
    assert g["products"] == g["nests"] * (g["depth"] + 1)
    # on a diagonal, 50 Newton nests reproduce 1 - (1 - mu)^(2^50) exactly
    # up to rounding; pick mu so that the series is far from converged
    a = np.array([1.0, 2.0, 4.0])
    X, info = oracle.nn_ref(np.diag(a), d=1, fixed_iter=50, x0=oracle.X0_GIVEN,
                            X_init=np.diag(np.full(3, 1e-15)))
    mu = a * 1e-15
    expect = -np.expm1(2.0 ** 50 * np.log1p(-mu)) / a
    np.testing.assert_allclose(np.diag(X), expect, rtol=1e-6)


def test_optimal_depth():
    g = GOLD["optimal_depth"]
    assert math.isclose(g["continuous_optimum"], math.e - 1)
    # products needed for a series of order >= Gamma, per depth: k (L+1)
    # with (L+1)^k >= Gamma; depth 2 is cheapest for every large Gamma
    for Gamma in (10 ** 6, 10 ** 12, 10 ** 18):
        cost = {L: (L + 1) * math.ceil(math.log(Gamma) / math.log(L + 1) - 1e-12) for L in (1, 2, 3, 4)}
        assert min(cost, key=cost.get) == g["integer_best"], cost


def test_depth_2_and_1_order_counts():
    """Corollary 4: after i+1 nests, depth 1 gives 2^(i+1) terms, depth 2
    gives 3^(i+1) — seen on a diagonal where each term is a known power."""
    a = np.array([3.0])
    for d, base in ((1, 2), (2, 3)):
        for k in (1, 2, 3):
            X, _ = oracle.nn_ref(np.diag(a), d=d, fixed_iter=k, x0=oracle.X0_GIVEN,
                                 X_init=np.diag([0.1]))
            r0 = 1 - 0.3
            expect = 0.1 * sum(r0 ** n for n in range(base ** k))
            assert math.isclose(X[0, 0], expect, rel_tol=1e-13)


def test_cond_1e6_nests():
    g = GOLD["cond_1e6_nests"]
    # closed form: worst residual eigenvalue (1 - 1/(cond^2 N))^(3^nests)
    for N in (16, 256, 4096):
        log_res = (g["depth"] + 1) ** g["nests"] * math.log1p(-1.0 / (g["cond"] ** 2 * N))
        assert log_res < math.log(1e-15)
