"""Pins of the oracle for Algorithm 2, the multi-product newsvendor (Section 3.2, oracle/newsvendor.c).

The cost Eq. (6) in closed form against numerical integration of its definition; the gradient
Eq. (8) against a finite difference of that cost; the estimator Eq. (9) unbiased for Eq. (8); the
vertex of the linear subproblem against a linear-programming solver; the signature identity; the
deterministic limit; and the long-run iterate against the constrained optimum from the KKT
conditions.
"""
import numpy as np
import pytest
from scipy import integrate, optimize, stats

import oracle
from paper_2404_11631_amd import workloads


def inst(n, seed=0):
    return workloads.newsvendor_instance(seed, 0, n)


def test_cost_closed_form_against_integration():
    """f_j(x) = k x + h E(x - xi)^+ + v E(xi - x)^+ with xi ~ N(mu, sigma^2), by quadrature of the
    definition over the demand density (the whole line, whose derivative is Eq. (8))."""
    I = inst(5)
    O = oracle.NvOracle(I, S=10)
    rng = np.random.default_rng(0)
    for _ in range(4):
        x = rng.uniform(0, 80, 5)
        ref = 0.0
        for j in range(5):
            pdf = stats.norm(I["mu"][j], I["sigma"][j]).pdf
            over = integrate.quad(lambda xi: (x[j] - xi) * pdf(xi), -np.inf, x[j])[0]
            under = integrate.quad(lambda xi: (xi - x[j]) * pdf(xi), x[j], np.inf)[0]
            ref += I["k"][j] * x[j] + I["h"][j] * over + I["v"][j] * under
        assert O.cost(x) == pytest.approx(ref, rel=1e-9)


def test_gradient_formula_is_the_derivative_of_the_cost():
    """Eq. (8): f_j'(x) = k - v + (h + v) Phi((x - mu)/sigma), against a central difference of the cost."""
    I = inst(6, seed=2)
    O = oracle.NvOracle(I, S=10)
    x = np.linspace(5, 70, 6)
    eps = 1e-5
    for j in range(6):
        e = np.zeros(6)
        e[j] = eps
        fd = (O.cost(x + e) - O.cost(x - e)) / (2 * eps)
        exact = I["k"][j] - I["v"][j] + (I["h"][j] + I["v"][j]) * stats.norm.cdf((x[j] - I["mu"][j]) / I["sigma"][j])
        assert fd == pytest.approx(exact, abs=1e-6)


def test_estimator_counts_and_unbiasedness():
    """Eq. (9) counts the samples at or below x_j (checked against the oracle's own normals), and its
    mean over many epochs is Eq. (8) within a 5-sigma band."""
    n, S = 8, 25
    I = inst(n, seed=3)
    O = oracle.NvOracle(I, S=S, seed=9)
    x = np.linspace(10, 60, n)
    g, cnt = O.gradient(0, 0, x)
    z = oracle.normals(9, 4, 0, 0, 0, 0, S * n).reshape(S, n)
    d = I["mu"] + I["sigma"] * z
    assert np.array_equal(cnt, (d <= x).sum(axis=0))
    assert np.allclose(g, I["k"] - I["v"] + (I["h"] + I["v"]) * cnt / S, rtol=1e-15)
    E = 2000
    acc = np.zeros(n)
    for e in range(E):
        acc += O.gradient(1, e, x)[0]
    mean = acc / E
    p = stats.norm.cdf((x - I["mu"]) / I["sigma"])
    exact = I["k"] - I["v"] + (I["h"] + I["v"]) * p
    sd = (I["h"] + I["v"]) * np.sqrt(p * (1 - p) / (S * E))
    assert np.all(np.abs(mean - exact) <= 5 * sd + 1e-12)


def test_first_vertex_against_linear_programming():
    """At x_0 = 0 the decision is the vertex of X = {c'x <= C, x >= 0} minimising s'g (linprog over
    the same gradient), and the oracle's x_1 is that vertex."""
    n = 12
    I = inst(n, seed=4)
    for seed in range(5):
        O = oracle.NvOracle(I, S=25, seed=seed)
        g, _ = O.gradient(0, 0, np.zeros(n))
        lp = optimize.linprog(g, A_ub=I["c"][None, :], b_ub=[I["C"]], bounds=[(0, None)] * n, method="highs")
        o = O.path(0, 1)
        a = int(o["decisions"][0])
        val = 0.0 if a == 0 else g[a - 1] * I["C"] / I["c"][a - 1]
        assert val == pytest.approx(lp.fun, rel=1e-9, abs=1e-9)
        x1 = np.zeros(n)
        if a:
            x1[a - 1] = I["C"] / I["c"][a - 1]
        assert o["y"] == pytest.approx(O.cost(x1), rel=1e-14)


def test_identity_replay_and_checkpoints():
    I = inst(50, seed=5)
    O = oracle.NvOracle(I, S=25, seed=1, ckpt=(10, 200))
    o = O.path(2, 200, uroff=2.0 ** -24)
    assert o["identity_err"] < 1e-13
    assert int(o["cnt"].sum()) == 200
    assert o["f_ckpt"][1] == o["y"]
    again = O.path(2, 200, replay=o["decisions"], uroff=2.0 ** -24)
    assert again["n_mismatch"] == 0 and again["y"] == o["y"]
    bad = o["decisions"].copy()
    bad[100] = (bad[100] % 50) + 1 if bad[100] != 0 else 1
    if bad[100] == o["decisions"][100]:
        bad[100] = 0
    w = O.path(2, 200, replay=bad, uroff=0.0)
    assert w["n_mismatch"] >= 1 and w["first_mismatch"] == 100


def test_zero_noise_decisions():
    """sigma = 0: every sample equals mu, so the gradient is k - v below mu and k + h at or above it;
    from the origin the first vertex is the product of smallest (k - v)/c."""
    n = 30
    I = inst(n, seed=6)
    I = dict(I, sigma=np.zeros(n))
    O = oracle.NvOracle(I, S=5)
    o = O.path(0, 40)
    assert int(o["decisions"][0]) == int(np.argmin((I["k"] - I["v"]) / I["c"])) + 1
    x = np.zeros(n)
    for t in range(40):
        g = np.where(x < I["mu"], I["k"] - I["v"], I["k"] + I["h"])
        r = g / I["c"]
        j = int(np.argmin(r))
        a = j + 1 if r[j] < 0 else 0
        assert int(o["decisions"][t]) == a
        s = np.zeros(n)
        if a:
            s[j] = I["C"] / I["c"][j]
        x = x + 2.0 / (t + 2) * (s - x)
    assert o["y"] == pytest.approx(O.cost(x), rel=1e-12)


def kkt_optimum(I):
    """The constrained optimum: Phi_j(x_j) = (v - k - lam c)/(h + v) clipped at x_j >= 0, lam >= 0
    set by bisection so that c'x = C when the budget binds."""
    def x_of(lam):
        q = (I["v"] - I["k"] - lam * I["c"]) / (I["h"] + I["v"])
        q = np.clip(q, 1e-300, 1 - 1e-16)
        return np.maximum(0.0, I["mu"] + I["sigma"] * stats.norm.ppf(q))
    if I["c"] @ x_of(0.0) <= I["C"]:
        return x_of(0.0)
    lo, hi = 0.0, float(np.max((I["v"] - I["k"]) / I["c"]))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if I["c"] @ x_of(mid) > I["C"]:
            lo = mid
        else:
            hi = mid
    return x_of(hi)


def test_long_run_reaches_the_constrained_optimum():
    """With many samples per gradient and many iterations the iterate's cost approaches the optimum of
    Eq. (7) from above (Frank-Wolfe's O(1/T) rate), never below it."""
    n = 3
    I = inst(n, seed=7)
    fstar = oracle.NvOracle(I, S=1).cost(kkt_optimum(I))
    O = oracle.NvOracle(I, S=400, seed=3)
    o = O.path(0, 3000)
    assert o["y"] >= fstar - 1e-9
    assert (o["y"] - fstar) / abs(fstar) < 2e-3


# ---- Eq. (7) with M resource rows ---------------------------------------------------------------

def test_lp_primitive_against_vertex_enumeration():
    """The general oracle's linear subproblem (HiGHS) against brute force over every basis of the
    standard form [A I][s; slack] = C (n = 6 products, M = 2 rows): the smallest s'g over the feasible
    basic solutions, for gradients of both signs."""
    import itertools
    n, M = 6, 2
    I = inst(n, seed=4)
    A, C = workloads.newsvendor_constraints(4, 0, n, M)
    O = oracle.NvLpOracle(I, A, C, S=5)
    full = np.hstack([A, np.eye(M)])
    rng = np.random.default_rng(1)
    for trial in range(40):
        g = rng.normal(size=n) - (0.5 if trial % 2 else -0.2)
        best = 0.0                                  # the origin (the slack basis)
        for cols in itertools.combinations(range(n + M), M):
            B = full[:, cols]
            if abs(np.linalg.det(B)) < 1e-12:
                continue
            xb = np.linalg.solve(B, C)
            if np.any(xb < -1e-12):
                continue
            s = np.zeros(n + M)
            s[list(cols)] = xb
            best = min(best, float(g @ s[:n]))
        val, s = O.lp(g)
        assert val == pytest.approx(best, rel=1e-9, abs=1e-12)
        assert np.all(s >= -1e-12) and np.all(A @ s <= C * (1 + 1e-9))
        assert float(g @ s) == pytest.approx(val, rel=1e-9, abs=1e-12)


def test_one_row_general_path_equals_the_ratio_rule_path():
    """With A = c (one row) the general oracle's vertices are the ratio rule's: the two oracle paths
    give the same iterates and outcomes."""
    n, T = 12, 150
    I = inst(n, seed=2)
    single = oracle.NvOracle(I, S=9, M=2, seed=5, ckpt=(50, 150)).path(0, T)
    general = oracle.NvLpOracle(I, I["c"][None, :], [I["C"]], S=9, M=2, seed=5, ckpt=(50, 150)).path(0, T)
    assert general["y"] == pytest.approx(single["y"], rel=1e-10)
    assert np.allclose(general["f_ckpt"], single["f_ckpt"], rtol=1e-10)
    xT = (I["C"] / I["c"]) * 2.0 * single["wsum"].astype(np.float64) / (T * (T + 1.0))
    assert np.allclose(general["x"], xT, rtol=1e-9, atol=1e-9 * float(np.max(I["C"] / I["c"])))


def test_general_constraints_long_run_reaches_the_optimum():
    """With many samples and iterations the iterate's cost approaches the optimum of Eq. (7) over
    {A x <= C, x >= 0} (three rows; the optimum by SLSQP on Eq. (6) in closed form) from above."""
    n, M = 4, 3
    I = inst(n, seed=11)
    A, C = workloads.newsvendor_constraints(11, 0, n, M)
    O = oracle.NvLpOracle(I, A, C, S=400, seed=2)
    res = optimize.minimize(O.cost, np.zeros(n), method="SLSQP", bounds=[(0, None)] * n,
                            constraints=[dict(type="ineq", fun=lambda x: C - A @ x, jac=lambda x: -A)],
                            options=dict(ftol=1e-14, maxiter=500))
    assert res.success
    fstar = res.fun
    o = O.path(0, 3000)
    assert np.all(A @ o["x"] <= C * (1 + 1e-12)) and np.all(o["x"] >= 0)
    assert o["y"] >= fstar - 1e-7 * abs(fstar)
    assert (o["y"] - fstar) / abs(fstar) < 3e-3
