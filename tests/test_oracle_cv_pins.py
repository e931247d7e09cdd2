"""Pins of the oracle's control-variate pieces against what mathematics fixes.

* Path features: their joint law is exact by construction (sample means and sample variances of
  Gaussian samples): xi ~ N(0, I_d), eta ~ N(0, 1) with Cov(xi_j, eta) = a, zeta a standardized
  chi-square(E d (N-1)) independent of both. Checked by KS tests and correlation bounds over
  oracle paths, for M = 1, for M = 3 with a short last epoch, and with t noise (whose Gaussian
  numerators carry the features).
* Aux draws: the same law (KS per coordinate, correlations), including the gamma sampler at
  shapes below, at and above one, and a two-sample KS against path features.
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


def _features(d, N, M, T, R, noise=oracle.NOISE_GAUSS, nu=3, seed=3):
    mu = np.linspace(0.1, 0.4, d)
    sigma = np.linspace(0.3, 0.6, d)
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, noise=noise, nu=nu, seed=seed, instance=2)
    outs = P.run(R, T)
    X = np.array([[o.feat[j] for j in range(d + 2)] for o in outs])
    return P, X


def _check_law(X, d, N, M, T, alpha=1e-3):
    n = X.shape[0]
    for j in range(d):
        assert ss.kstest(X[:, j], "norm").pvalue > alpha, f"xi_{j}"
    assert ss.kstest(X[:, d], "norm").pvalue > alpha, "eta"
    E = -(-T // M)
    k = E * d * (N - 1)
    chi = X[:, d + 1] * math.sqrt(2 * k) + k
    assert ss.kstest(chi, ss.chi2(k).cdf).pvalue > alpha, "zeta"
    a = oracle.cv_eta_corr(T, M, d)
    se = 4.5 / math.sqrt(n)
    for j in range(d):
        assert abs(np.corrcoef(X[:, j], X[:, d])[0, 1] - a) < se, f"corr(xi_{j}, eta)"
        assert abs(np.corrcoef(X[:, j], X[:, d + 1])[0, 1]) < se, f"corr(xi_{j}, zeta)"
        for i in range(j):
            assert abs(np.corrcoef(X[:, j], X[:, i])[0, 1]) < se
    assert abs(np.corrcoef(X[:, d], X[:, d + 1])[0, 1]) < se


@pytest.mark.parametrize("d,N,M,T,noise", [
    (3, 5, 1, 40, oracle.NOISE_GAUSS),
    (2, 4, 3, 40, oracle.NOISE_GAUSS),      # 14 epochs, the last one a single iteration
    (3, 3, 1, 30, oracle.NOISE_T),
])
def test_path_feature_law(d, N, M, T, noise):
    P, X = _features(d, N, M, T, 3000, noise=noise)
    _check_law(X, d, N, M, T)


def test_feature_constants():
    # M = 1, T = 4: weights 1..4, norm sqrt(30); the late window is one epoch (the last)
    assert math.isclose(oracle.cv_weight_norm(4, 1), math.sqrt(30.0), rel_tol=1e-15)
    assert oracle.cv_late_epochs(4) == 1 and oracle.cv_late_epochs(10) == 1 and oracle.cv_late_epochs(11) == 2
    assert math.isclose(oracle.cv_eta_corr(4, 1, 2), 4.0 / (math.sqrt(30.0) * math.sqrt(2.0)), rel_tol=1e-15)
    # M = 3, T = 7: epochs {0,1,2}, {3,4,5}, {6} with weights 6, 15, 7
    assert math.isclose(oracle.cv_weight_norm(7, 3), math.sqrt(36 + 225 + 49), rel_tol=1e-15)
    # Cauchy-Schwarz keeps the eta mixture valid: d a^2 <= 1
    for T, M, d in [(10_000, 1, 10), (1000, 1, 64), (7, 3, 1), (1, 1, 1)]:
        assert d * oracle.cv_eta_corr(T, M, d) ** 2 <= 1.0 + 1e-15


def test_single_iteration_features_are_sample_summaries():
    """T = 1: xi is sqrt(N) times the sample mean of the one draw and zeta is the standardized
    pooled within-asset sum of squares; eta (one late epoch) is the sum of xi over sqrt(d)."""
    d, N = 3, 6
    P = oracle.OracleProblem(np.zeros(d), np.ones(d), N=N, seed=11, instance=0)
    o = P.path(5, 1)
    Z = oracle.normals(11, 0, 0, 5, 0, 0, N * d).reshape(N, d)
    xi = Z.mean(axis=0) * math.sqrt(N)
    k = d * (N - 1)
    ssq = ((Z - Z.mean(axis=0)) ** 2).sum()
    assert np.allclose([o.feat[j] for j in range(d)], xi, rtol=1e-13, atol=1e-14)
    assert math.isclose(o.feat[d], xi.sum() / math.sqrt(d), rel_tol=1e-13)
    assert math.isclose(o.feat[d + 1], (ssq - k) / math.sqrt(2 * k), rel_tol=1e-12, abs_tol=1e-14)


@pytest.mark.parametrize("d,N,M,T", [(3, 5, 1, 40), (1, 2, 1, 1), (1, 3, 1, 1), (1, 2, 1, 6), (10, 10, 1, 10_000)])
def test_aux_law(d, N, M, T):
    """k = E d (N-1) of 1, 2 and 6 run the gamma sampler at shapes 1/2, 1 and 3; 9e5 at the
    control-variate workload's size."""
    P = oracle.OracleProblem(np.zeros(d), np.ones(d), N=N, M=M, seed=21, instance=4)
    X, tries = oracle.cv_aux(P, T, 0, 4000)
    assert np.all(tries >= 1)
    _check_law(X, d, N, M, T)


def test_aux_matches_path_features():
    d, N, M, T = 2, 4, 3, 40
    P, Xp = _features(d, N, M, T, 3000)
    Xa, _ = oracle.cv_aux(P, T, 0, 3000)
    for j in range(d + 2):
        assert ss.ks_2samp(Xp[:, j], Xa[:, j]).pvalue > 1e-3


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
