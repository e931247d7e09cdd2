"""Pins of the oracle's control-variate pieces against what mathematics fixes.

* Reference-decision probabilities: they sum to one, reduce to normal CDFs for one asset and to
  equal shares for a symmetric instance, and match brute-force Monte Carlo of the argmin.
* Path features: the raw summaries' exact moments (E count_c = p_c S2, Cov = S4 (p_c [c = c'] -
  p_c p_c'), the same with (t+1) weights, and the correlation of the two weightings), for M = 1,
  M = 3 with a short last epoch, and t noise; the T = 1 case against the argmin of the raw normals.
* Aux draws: category frequencies against p (chi-square goodness of fit), the same moments, and
  agreement with path features.
* Surrogate gradient: central finite differences of the unrounded network, and torch's autograd
  (float64) on an independent formulation of the rounded network.
* bfloat16 rounding: torch's float32 -> bfloat16 conversion, ties included.
* Estimator: unbiasedness and its variance formula on a synthetic pair with known moments.
"""
import math

import numpy as np
import pytest
import scipy.stats as ss

import oracle


def _instance(d, seed=3):
    g = np.random.default_rng(seed)
    mu = g.uniform(0.1, 0.6, d)
    sigma = g.uniform(0.2, 0.7, d)
    return mu, sigma


def _ref(mu, sigma, N, scale=0.6):
    """A reference gradient near the problem's: 2 lambda Sigma w - mu at an interior point."""
    d = mu.shape[0]
    w = np.full(d, scale / d)
    return sigma ** 2 * w - mu


@pytest.mark.parametrize("d", [1, 3, 10, 32])
def test_pick_probs_sum_to_one(d):
    g = np.random.default_rng(d)
    for _ in range(3):
        b = g.uniform(-0.8, 0.3, d)
        s = g.uniform(0.05, 0.5, d)
        p, tot = oracle.cv_pick_probs(b, s)
        assert abs(tot - 1.0) < 1e-11 and np.all(p >= 0)


def test_pick_probs_closed_forms():
    p, _ = oracle.cv_pick_probs([-0.3], [0.4])
    assert math.isclose(p[0], ss.norm.cdf(-0.75), rel_tol=1e-12)
    assert math.isclose(p[1], ss.norm.sf(-0.75), rel_tol=1e-12)
    d = 5
    p, _ = oracle.cv_pick_probs(np.full(d, -0.2), np.full(d, 0.3))
    p0 = ss.norm.cdf(-0.2 / 0.3) ** d
    assert math.isclose(p[0], p0, rel_tol=1e-12)
    assert np.allclose(p[1:], (1 - p0) / d, rtol=1e-11)


def test_pick_probs_monte_carlo():
    g = np.random.default_rng(11)
    d = 6
    b = g.uniform(-0.5, 0.1, d)
    s = g.uniform(0.1, 0.4, d)
    p, _ = oracle.cv_pick_probs(b, s)
    n = 2_000_000
    V = b - s * g.standard_normal((n, d))
    j = V.argmin(1)
    cat = np.where(V[np.arange(n), j] < 0, j + 1, 0)
    freq = np.bincount(cat, minlength=d + 1) / n
    se = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(freq - p) < 5 * se + 1e-12)


def _paths(d, N, M, T, R, noise=oracle.NOISE_GAUSS, seed=3):
    mu, sigma = _instance(d)
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, noise=noise, nu=4, seed=seed, instance=2,
                             cv_ref=_ref(mu, sigma, N))
    outs = P.run(R, T)
    C = np.array([[o.cv_count[c] for c in range(d + 1)] for o in outs])
    C1 = np.array([[o.cv_count1[c] for c in range(d + 1)] for o in outs])
    return P, C, C1


def _check_moments(C, C1, law, tol=5.0):
    """Weighted sums of i.i.d. categorical indicators: E count_c = p_c S2, Var = p_c (1 - p_c) S4,
    Cov(count_c, count_c') = -p_c p_c' S4; for the (t+1) weights S1, S11, and
    Cov(count1_c, count_c) = p_c (1 - p_c) S12."""
    n = C.shape[0]
    p, S2, S4, S1, S11, S12 = law.probs, law.S2, law.S4, law.S1, law.S11, law.S12
    for cnt, mw, vw in ((C, S2, S4), (C1, S1, S11)):
        mean = p * mw
        var = p * (1 - p) * vw
        ok = var > 0
        z = (cnt.mean(0) - mean)[ok] / np.sqrt(var[ok] / n)
        assert np.all(np.abs(z) < tol), z
        # variances of the categories that are neither rare nor dominant (sums of many weighted
        # indicators, close to normal): the sample variance scatters by about sqrt(2/n) (relative)
        mid = (p > 0.05) & (p < 0.95)
        rv = cnt.var(0, ddof=1)[mid] / var[mid]
        assert np.all(np.abs(rv - 1) < tol * math.sqrt(2.0 / n) + 0.02), rv
    a, b = np.argsort(p)[-2:]
    cov = np.cov(C[:, a], C[:, b])[0, 1]
    assert abs(cov + p[a] * p[b] * S4) < tol * math.sqrt(p[a] * (1 - p[a]) * p[b] * (1 - p[b])) * S4 / math.sqrt(n) * 1.5
    c = law.top
    corr = np.corrcoef(C[:, c], C1[:, c])[0, 1]
    exact = S12 / math.sqrt(S4 * S11)
    assert abs(corr - exact) < tol * (1 - exact ** 2) / math.sqrt(n) + 0.01, (corr, exact)


@pytest.mark.parametrize("d,N,M,T,noise", [
    (3, 5, 1, 40, oracle.NOISE_GAUSS),
    (2, 4, 3, 40, oracle.NOISE_GAUSS),      # 14 epochs, the last one a single iteration
    (3, 3, 1, 30, oracle.NOISE_T),          # the features use the Gaussian numerators
])
def test_path_feature_law(d, N, M, T, noise):
    P, C, C1 = _paths(d, N, M, T, 3000, noise=noise)
    law = oracle.CvLaw(P, T)
    assert abs(law.total - 1) < 1e-11
    assert np.allclose(C.sum(1), law.S2) and np.allclose(C1.sum(1), law.S1)
    _check_moments(C, C1, law)


def test_weights_closed_form():
    S2, S4, S1, S11, S12 = oracle.cv_weights(4, 1)
    assert S2 == 1 + 4 + 9 + 16 and S4 == 1 + 16 + 81 + 256
    assert S1 == 10 and S11 == 30 and S12 == 1 + 8 + 27 + 64
    S2, S4, S1, S11, S12 = oracle.cv_weights(7, 3)       # epochs {1,2,3}, {4,5,6}, {7}
    assert S2 == 140 and S4 == 14 ** 2 + 77 ** 2 + 49 ** 2
    assert S1 == 28 and S11 == 6 ** 2 + 15 ** 2 + 7 ** 2 and S12 == 6 * 14 + 15 * 77 + 7 * 49


def test_single_iteration_pick_is_the_argmin_of_the_sample_mean():
    d, N = 4, 6
    mu, sigma = _instance(d)
    b = _ref(mu, sigma, N)
    P = oracle.OracleProblem(mu, sigma, N=N, seed=11, instance=0, cv_ref=b)
    for r in range(20):
        o = P.path(r, 1)
        Z = oracle.normals(11, 0, 0, r, 0, 0, N * d).reshape(N, d)
        v = b - sigma * Z.mean(axis=0)
        cat = int(v.argmin()) + 1 if v.min() < 0 else 0
        expect = np.zeros(d + 1)
        expect[cat] = 1.0
        assert np.array_equal([o.cv_count[c] for c in range(d + 1)], expect)
        assert np.array_equal([o.cv_count1[c] for c in range(d + 1)], expect)


def test_aux_categories_follow_the_probabilities():
    d, N = 4, 5
    mu, sigma = _instance(d)
    P = oracle.OracleProblem(mu, sigma, N=N, seed=21, instance=4, cv_ref=_ref(mu, sigma, N, 0.3))
    law = oracle.CvLaw(P, 1)
    X, C, C1 = law.aux(0, 20000)
    obs = C.sum(0)
    exp = law.probs * C.shape[0]
    keep = exp > 5
    chi = (((obs - exp) ** 2) / exp)[keep].sum()
    assert ss.chi2(keep.sum() - 1).sf(chi) > 1e-3


@pytest.mark.parametrize("d,N,M,T", [(3, 5, 1, 40), (1, 2, 1, 6), (2, 4, 3, 40), (6, 3, 1, 25)])
def test_aux_law(d, N, M, T):
    mu, sigma = _instance(d)
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, seed=21, instance=4, cv_ref=_ref(mu, sigma, N))
    law = oracle.CvLaw(P, T)
    X, C, C1 = law.aux(0, 4000)
    assert np.allclose(C.sum(1), law.S2) and np.allclose(C1.sum(1), law.S1)
    _check_moments(C, C1, law)


def test_standardized_features_have_unit_variance():
    """Slot by slot: x_j is vertex e_j's count, x_d the origin's, x_{d+1} the (t+1)-weighted count of
    the most probable category; each has mean 0 and, away from rare categories, variance 1. The
    reference gradient leaves the origin a large share here."""
    d, N, T = 3, 4, 30
    mu, sigma = _instance(d)
    b = _ref(mu, sigma, N) + 0.9 * mu
    P = oracle.OracleProblem(mu, sigma, N=N, seed=5, instance=1, cv_ref=b)
    law = oracle.CvLaw(P, T)
    assert 0.1 < law.probs[0] < 0.9
    X, _, _ = law.aux(0, 6000)
    cat = np.concatenate([law.probs[1:], law.probs[:1], [law.probs[law.top]]])
    for j in range(d + 2):
        assert abs(X[:, j].mean()) < 5 / math.sqrt(6000)
        if 0.05 < cat[j] < 0.95:
            assert abs(X[:, j].var() - 1) < 0.1, j


def test_top_category():
    assert oracle.lib().or_cv_top(3, oracle._dptr(np.array([0.1, 0.4, 0.4, 0.1]))) == 1


def test_aux_matches_path_features():
    d, N, M, T = 2, 4, 3, 40
    P, C, C1 = _paths(d, N, M, T, 3000)
    law = oracle.CvLaw(P, T)
    Xa, _, _ = law.aux(0, 3000)
    Xp = np.array([law.standardize(C[i], C1[i]) for i in range(C.shape[0])])
    for j in range(d + 2):
        assert ss.ks_2samp(Xp[:, j], Xa[:, j]).pvalue > 1e-3
    assert np.allclose(Xp.mean(0), 0.0, atol=0.15)


def _theta(F, seed, scale=0.4):
    g = np.random.default_rng(seed)
    return g.normal(0.0, scale, oracle.mlp_param_count(F))


def test_param_count():
    assert oracle.mlp_param_count(12) == 5057


def test_mlp_gradient_finite_differences():
    F, n = 4, 7
    g = np.random.default_rng(1)
    th = _theta(F, 2)
    x = g.normal(size=(n, F))
    y = g.normal(size=n)
    loss, grad = oracle.mlp_grad(th, F, x, y)
    assert math.isclose(loss, np.mean((oracle.mlp_forward(th, F, x) - y) ** 2), rel_tol=1e-13)
    h = 1e-6
    fd = np.zeros_like(th)
    for i in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (np.mean((oracle.mlp_forward(tp, F, x) - y) ** 2) -
                 np.mean((oracle.mlp_forward(tm, F, x) - y) ** 2)) / (2 * h)
    assert np.max(np.abs(fd - grad)) <= 1e-7 * max(1.0, np.max(np.abs(grad)))


def _torch_model(th, F, x, y, quantize):
    """Independent float64 torch formulation; quantization points as the matrix cores take them:
    operands rounded going in (straight through for their own gradients), and the gradient that
    flows back into each product rounded before the product's backward."""
    import torch

    def q(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    class STE(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return q(t)

        @staticmethod
        def backward(ctx, g):
            return g

    class GradRound(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return q(g)

    Q = STE.apply if quantize else (lambda t: t)
    G = GradRound.apply if quantize else (lambda t: t)
    t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = t[o:o + 64 * F].view(64, F); o += 64 * F
    b1 = t[o:o + 64]; o += 64
    W2 = t[o:o + 4096].view(64, 64); o += 4096
    b2 = t[o:o + 64]; o += 64
    w3 = t[o:o + 64]; o += 64
    b3 = t[o]
    X = torch.tensor(x, dtype=torch.float64)
    Y = torch.tensor(y, dtype=torch.float64)
    gelu = torch.nn.functional.gelu           # exact erf form
    h1 = gelu(G(Q(X) @ Q(W1).T) + b1)
    h2 = gelu(G(Q(h1) @ Q(W2).T) + b2)
    out = h2 @ w3 + b3
    loss = torch.mean((out - Y) ** 2)
    loss.backward()
    return loss.item(), t.grad.numpy()


@pytest.mark.parametrize("quantize", [False, True])
def test_mlp_matches_torch_autograd(quantize):
    F, n = 12, 33
    g = np.random.default_rng(7)
    th = _theta(F, 8, 0.3)
    x = g.normal(size=(n, F))
    y = g.normal(size=n)
    loss, grad = oracle.mlp_grad(th, F, x, y, quantize=quantize)
    tl, tg = _torch_model(th, F, x, y, quantize)
    assert math.isclose(loss, tl, rel_tol=1e-12)
    assert np.max(np.abs(grad - tg)) <= 1e-11 * np.max(np.abs(tg))
    if quantize:
        _, g0 = oracle.mlp_grad(th, F, x, y, quantize=False)
        assert np.max(np.abs(grad - g0)) > 1e-6 * np.max(np.abs(g0))   # the rounding is really applied


def test_bf16_rounding_matches_torch():
    import torch
    g = np.random.default_rng(0)
    v = np.concatenate([g.normal(size=2000) * 10.0 ** g.integers(-5, 5, 2000), [0.0, -0.0, 1.0, -2.5]])
    # exact ties: low half 0x8000 with even and odd upper halves
    bits = (g.integers(0x3F000000, 0x40800000, 200, dtype=np.uint32) & 0xFFFF0000) | 0x8000
    v = np.concatenate([v, bits.view(np.float32).astype(np.float64)])
    ours = np.array([oracle.bf16(x) for x in v])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_estimator_unbiased_with_stated_variance():
    """Y = 1 + 2 xi + e (Var e = 1/4), h = xi, beta = 2, aux xi' ~ N(0,1): E Y_cv = 1 and
    Var Y_cv = 0.25 / n + 4 / n_aux; over 400 seeds the estimates scatter as the formula says."""
    n, n_aux, reps = 400, 4000, 400
    g = np.random.default_rng(5)
    est, var = [], []
    for _ in range(reps):
        xi = g.normal(size=n)
        Y = 1.0 + 2.0 * xi + 0.5 * g.normal(size=n)
        st = oracle.cv_estimate(Y, xi, g.normal(size=n_aux), 2.0)
        est.append(st.mean_cv)
        var.append(st.var_est)
        assert math.isclose(st.mean_plain, Y.mean(), rel_tol=1e-12)
    est, var = np.array(est), np.array(var)
    v_true = 0.25 / n + 4.0 / n_aux
    assert abs(est.mean() - 1.0) < 4.0 * math.sqrt(v_true / reps)
    assert abs(var.mean() / v_true - 1.0) < 0.05
    ratio = est.var(ddof=1) / v_true            # ~ chi2(reps-1)/(reps-1)
    lo, hi = ss.chi2(reps - 1).ppf([1e-4, 1 - 1e-4]) / (reps - 1)
    assert lo < ratio < hi


def test_beta_closed_form():
    g = np.random.default_rng(2)
    H = g.normal(size=500)
    b, r2 = oracle.cv_beta(3.0 - 2.5 * H, H)
    assert math.isclose(b, -2.5, rel_tol=1e-12) and math.isclose(r2, 1.0, rel_tol=1e-12)
    b, r2 = oracle.cv_beta(g.normal(size=500), H)
    assert abs(b) < 0.25 and r2 < 0.05


def test_dense_factor_features_follow_the_product_law():
    """With a dense factor the reference decision reads each noise coordinate against L_jj, so the
    counts follow the same product-form law as with L = diag(L_jj), whatever the off-diagonal
    entries; the paths themselves use the full L."""
    d, N, M, T, R = 3, 4, 1, 30, 3000
    mu, sigma = _instance(d)
    g = np.random.default_rng(5)
    L = np.diag(sigma) + np.tril(g.uniform(-0.4, 0.4, (d, d)), -1)
    P = oracle.OracleProblem(mu, chol=L, N=N, M=M, seed=8, instance=4, cv_ref=_ref(mu, sigma, N))
    outs = P.run(R, T)
    C = np.array([[o.cv_count[c] for c in range(d + 1)] for o in outs])
    C1 = np.array([[o.cv_count1[c] for c in range(d + 1)] for o in outs])
    law = oracle.CvLaw(P, T)
    assert np.allclose(C.sum(1), law.S2)
    _check_moments(C, C1, law)
    # one iteration: the pick is the argmin of b - diag(L) zbar over the vertices and the origin
    b = _ref(mu, sigma, N)
    for r in range(20):
        o = P.path(r, 1)
        Z = oracle.normals(8, 0, 4, r, 0, 0, N * d).reshape(N, d)
        v = b - np.diag(L) * Z.mean(axis=0)
        cat = int(v.argmin()) + 1 if v.min() < 0 else 0
        assert [o.cv_count[c] for c in range(d + 1)] == [1.0 if c == cat else 0.0 for c in range(d + 1)]
