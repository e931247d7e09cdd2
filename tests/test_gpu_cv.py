"""Control-variate pieces on the device vs the CPU oracle through the C ABI (needs an MI355X).

Features: each path's d+2 features against the oracle's (same noise stream, replayed decisions).
The reference decisions are taken from binary32 sample means on the device and FP64 ones in the
oracle, so an epoch whose reference margin is below 1e-4 may fall in another category; the
tolerance is that weight (the oracle reports it) times the standardization, plus 5e-5 for the
binary32 chi-square summary and storage. At sizes the oracle cannot follow: the exact moments of
the features' law.
"""
import math
import sys

import numpy as np
import pytest
import scipy.stats as ss

import oracle
from paper_2404_11631_amd import sim, workloads
from tests import parity

pytestmark = pytest.mark.gpu

FEAT_ATOL = 5e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    s = sim.Sim(0)
    yield s
    s.close()


def _ref(mu, sigma, scale=0.8):
    d = mu.shape[0]
    return sigma ** 2 * np.full(d, scale / d) - mu


@pytest.mark.parametrize("case", [
    dict(d=10, N=10, M=1, T=200, R=300, noise=sim.NOISE_GAUSS),
    dict(d=3, N=4, M=3, T=100, R=200, noise=sim.NOISE_GAUSS),
    dict(d=6, N=5, M=1, T=120, R=150, noise=sim.NOISE_T),
    dict(d=20, N=3, M=2, T=61, R=130, noise=sim.NOISE_GAUSS),
], ids=lambda c: f"d{c['d']}N{c['N']}M{c['M']}{'t' if c['noise'] else 'g'}")
def test_features_match_oracle(ctx, case):
    d, R, T = case["d"], case["R"], case["T"]
    mu, sigma = workloads.diag_instance(9, d, d)
    b = _ref(mu, sigma)
    p = sim.Problem(mu=mu, sigma=sigma, N=case["N"], M=case["M"], noise=case["noise"], nu=4,
                    checkpoints=(T,), gap_eps=0.05, instance_id=30 + d, keep_paths=True,
                    log_reps=(0, R), cv_features=True, cv_ref=b)
    say(f"[cv] features d={d} N={case['N']} M={case['M']} noise={case['noise']} R={R} T={T}")
    ctx.run(p, R, T, 77)
    g = ctx.paths()
    assert g["x"].shape == (d + 2, R)
    P = parity.oracle_problem(p, 77)
    law = oracle.CvLaw(P, T)
    inv = np.concatenate([1.0 / np.sqrt(law.S4 * np.maximum(law.probs * (1 - law.probs), 1e-4)),
                          [1.0 / np.sqrt(law.S11 * max(law.probs[law.top] * (1 - law.probs[law.top]), 1e-4))]])
    amb1 = 1.0 / math.sqrt(law.S11 * max(law.probs[law.top] * (1 - law.probs[law.top]), 1e-4))
    err, amb = 0.0, 0
    for r in range(R):
        o = parity.check_rep(P, g, r, T, oracle.U32, decisions=g["decisions"][:, r])
        ref = law.path_features(o)
        e = np.abs(g["x"][:, r].astype(np.float64) - ref)
        tol = FEAT_ATOL + 1e-6 * np.abs(ref)
        # a flipped epoch moves its (t+1)^2 weight between two counts, and at most its (t+1)
        # weight (<= the square root of the former) into or out of the top category's count
        tol[: d + 1] += o.cv_amb * inv[: d + 1].max()
        tol[d + 1] += math.sqrt(o.cv_amb) * amb1 * 4
        amb += o.cv_amb > 0
        err = max(err, e.max())
        assert np.all(e <= tol), f"rep {r}: feature errors {e}"
    say(f"[cv] max feature error {err:.2e}; replications with a near-tie reference decision: {amb}")


def test_features_do_not_change_the_paths(ctx):
    d, R, T = 10, 2000, 300
    mu, sigma = workloads.diag_instance(1, 2, d)
    base = dict(mu=mu, sigma=sigma, N=10, checkpoints=(100, T), keep_paths=True)
    ctx.run(sim.Problem(**base), R, T, 5)
    a = ctx.paths()
    ctx.run(sim.Problem(**base, cv_features=True, cv_ref=_ref(mu, sigma)), R, T, 5)
    b = ctx.paths()
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["wsum"], b["wsum"])
    assert "x" not in a and "x" in b


def test_feature_law_at_scale(ctx):
    """The control-variate workload's shape (d = 10, N = 10) at R = 2e5, T = 1000: the device's
    features have their law's exact means and variances, and the chi-square summary its law."""
    d, R, T = 10, 200_000, 1000
    mu, sigma = workloads.diag_instance(0, 0, d)
    b = _ref(mu, sigma)
    p = sim.Problem(mu=mu, sigma=sigma, N=10, checkpoints=(T,), cv_features=True, cv_ref=b)
    ctx.run(p, R, T, 100)
    X = ctx.paths()["x"].astype(np.float64)
    probs, S2, S4 = sim.cv_law(p, T)
    top = int(np.argmax(probs))
    cat = np.concatenate([probs[1:], probs[:1], [probs[top]]])   # vertices, the origin, the top count
    v = cat * (1 - cat) / np.maximum(cat * (1 - cat), 1e-4)
    for j in range(d + 2):
        if v[j] > 0:
            assert abs(X[j].mean()) < 5 * math.sqrt(v[j] / R), f"feature {j} mean"
        if 0.05 < cat[j] < 0.95:
            assert abs(X[j].var() / v[j] - 1) < 5 * math.sqrt(2 / R) + 0.01, f"feature {j} variance"
    say(f"[cv] law ok at R={R}: probabilities {np.round(probs, 3)}")


# ---- surrogate primitives ------------------------------------------------------------------
# The device rounds the operands of each matrix product to bfloat16 where the oracle (quantize)
# does, but accumulates in FP32: an activation whose FP32 and FP64 values straddle a bfloat16
# rounding boundary rounds differently (one bfloat16 ulp, 2^-8 relative), so a few elements per
# batch differ at the 1e-3 level. Tolerances: forward, median relative error 1e-5 and every row
# within 5e-3 of the output scale; gradient, 1e-3 relative Frobenius error per tensor.

def _theta(F, seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.normal(0.0, scale, sim.mlp_param_count(F)).astype(np.float32)


def _tensors(F):
    o = 0
    out = {}
    for name, size in (("W1", 64 * F), ("b1", 64), ("W2", 4096), ("b2", 64), ("w3", 64), ("b3", 1)):
        out[name] = slice(o, o + size)
        o += size
    return out


def test_cv_run_needs_a_fit(ctx):
    mu, sigma = workloads.diag_instance(0, 0, 4)
    with pytest.raises(sim.SimError) as e:
        ctx.run_cv(sim.Problem(mu=mu, sigma=sigma, N=4), 100, 10, 1, 100)
    assert e.value.code == -4


@pytest.mark.parametrize("F,n", [(12, 300), (66, 257), (3, 128), (17, 1000)])
def test_mlp_forward_matches_oracle(ctx, F, n):
    th = _theta(F, F)
    x = np.random.default_rng(F + 1).normal(size=(F, n)).astype(np.float32)
    ctx.mlp_set_params(F, th)
    assert np.array_equal(ctx.mlp_get_params(F), th)
    out = ctx.mlp_forward(x).astype(np.float64)
    ref = oracle.mlp_forward(th.astype(np.float64), F, x.T.astype(np.float64), quantize=True)
    err = np.abs(out - ref)
    scale = np.sqrt(np.mean(ref ** 2))
    say(f"[cv] forward F={F} n={n}: max err {err.max():.2e}, median rel {np.median(err / np.abs(ref)):.2e}")
    assert np.median(err / np.abs(ref)) <= 1e-5
    assert err.max() <= 5e-3 * scale


@pytest.mark.parametrize("F,n", [(12, 300), (66, 200), (12, 4096)])
def test_mlp_grad_matches_oracle(ctx, F, n):
    g = np.random.default_rng(100 + F)
    th = _theta(F, 200 + F)
    x = g.normal(size=(F, n)).astype(np.float32)
    y = g.normal(size=n).astype(np.float32)
    ctx.mlp_set_params(F, th)
    loss, grad = ctx.mlp_grad(x, y)
    loss2, grad2 = ctx.mlp_grad(x, y)
    assert loss == loss2 and np.array_equal(grad, grad2)          # fixed reduction order
    lref, gref = oracle.mlp_grad(th.astype(np.float64), F, x.T.astype(np.float64), y.astype(np.float64),
                                 quantize=True)
    assert abs(loss - lref) <= 1e-4 * lref
    for name, sl in _tensors(F).items():
        rel = np.linalg.norm(grad[sl] - gref[sl]) / np.linalg.norm(gref[sl])
        say(f"[cv] grad F={F} n={n} {name}: rel Frobenius error {rel:.2e}")
        assert rel <= 1e-3, name


@pytest.mark.parametrize("d,N,M,T,n", [(10, 10, 1, 10_000, 300), (1, 2, 1, 1, 2000), (3, 5, 2, 41, 2000),
                                       (32, 100, 1, 1000, 300)])
def test_aux_draws_match_oracle(ctx, d, N, M, T, n):
    mu, sigma = workloads.diag_instance(4, d, d)
    b = _ref(mu, sigma)
    p = sim.Problem(mu=mu, sigma=sigma, N=N, M=M, instance_id=5, cv_ref=b)
    x = ctx.cv_aux_draws(p, T, 123, 1000, n)
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, seed=123, instance=5, cv_ref=b)
    ref, _, _ = oracle.CvLaw(P, T).aux(1000, n)
    err = np.abs(x.T.astype(np.float64) - ref)
    say(f"[cv] aux d={d} T={T}: max err {err.max():.2e}")
    assert np.all(err <= 2e-6 + 1e-6 * np.abs(ref))


def test_aux_draws_dense_factor_match_oracle(ctx):
    """d = 64 with a dense factor (the stress shape): the law of the features reads L_jj."""
    d, N, T, n = 64, 100, 1000, 300
    mu, L = workloads.dense_instance(0, 0, d)
    b = _ref(mu, np.diag(L))
    p = sim.Problem(mu=mu, chol=L, N=N, noise=sim.NOISE_T, nu=3, instance_id=6, cv_ref=b)
    x = ctx.cv_aux_draws(p, T, 124, 77, n)
    P = oracle.OracleProblem(mu, chol=L, N=N, noise=oracle.NOISE_T, nu=3, seed=124, instance=6, cv_ref=b)
    ref, _, _ = oracle.CvLaw(P, T).aux(77, n)
    err = np.abs(x.T.astype(np.float64) - ref)
    say(f"[cv] aux dense d={d} T={T}: max err {err.max():.2e}")
    assert np.all(err <= 2e-6 + 1e-6 * np.abs(ref))


def test_cv_fit_and_estimate(ctx):
    """Train on the device, fit beta on a pilot, estimate: the estimator's arithmetic matches the
    oracle's on the same arrays, h matches the oracle's surrogate on the same features, the estimate
    agrees with the plain mean of the same paths, and its variance is smaller."""
    d, N, T = 10, 10, 300
    mu, sigma = workloads.diag_instance(100, 0, d)
    p = sim.Problem(mu=mu, sigma=sigma, N=N)
    fit = ctx.cv_fit(p, T, 1, n_runs=2, epochs=4, R_train=1 << 16, R_pilot=1 << 15, batch=4096, lr=2e-3)
    say(f"[cv] fit: loss {fit.loss_first_epoch:.4f} -> {fit.loss_last_epoch:.4f}, beta {fit.beta:.3f}, "
        f"rho2 {fit.rho2:.3f}, sim {fit.sim_ms:.0f} ms, train {fit.train_ms:.0f} ms ({fit.steps} steps)")
    assert fit.n_train == 2 << 16 and fit.steps == 4 * 32
    assert fit.loss_last_epoch < fit.loss_first_epoch
    R, R_aux = 20_000, 400_000
    st = ctx.run_cv(p, R, T, 100, R_aux)
    v = ctx.cv_paths()
    assert v["h_aux"].shape == (R_aux,) and 0 < st.paths_ms < st.kernel_ms and 0 < st.aux_ms < st.kernel_ms
    ost = oracle.cv_estimate(v["y"], v["h"].astype(np.float64), v["h_aux"].astype(np.float64), st.beta)
    for a, b, tol in ((st.mean_plain, ost.mean_plain, 1e-12), (st.var_plain, ost.var_plain, 1e-9),
                      (st.mean_resid, ost.mean_resid, 1e-12), (st.var_resid, ost.var_resid, 1e-8),
                      (st.mean_h_aux, ost.mean_h_aux, 1e-12), (st.var_h_aux, ost.var_h_aux, 1e-9),
                      (st.mean_cv, ost.mean_cv, 1e-12), (st.var_est, ost.var_est, 1e-8)):
        assert abs(a - b) <= tol * max(abs(a), abs(b), 1e-300), (a, b)
    theta = ctx.mlp_get_params(d + 2).astype(np.float64)
    href = fit.y_mean + fit.y_sd * oracle.mlp_forward(theta, d + 2, v["x"][:, :512].T.astype(np.float64),
                                                      quantize=True)
    assert np.max(np.abs(v["h"][:512] - href)) <= 2e-3 * fit.y_sd
    joint = math.sqrt(st.ci95_plain ** 2 + st.ci95_cv ** 2) / 1.96
    gain = (st.var_plain / R) / st.var_est
    say(f"[cv] plain {st.mean_plain:.6f} +- {st.ci95_plain:.2e}, cv {st.mean_cv:.6f} +- {st.ci95_cv:.2e}, "
        f"variance gain {gain:.2f}, rho2 {st.rho2:.3f}, {st.kernel_ms:.1f} ms")
    assert abs(st.mean_cv - st.mean_plain) <= 4.5 * joint
    assert gain > 1.2


@pytest.mark.parametrize("case", [
    dict(d=32, N=6, M=1, T=80, R=128, noise=sim.NOISE_GAUSS),
    dict(d=64, N=5, M=2, T=40, R=64, noise=sim.NOISE_T),
], ids=lambda c: f"dense{c['d']}N{c['N']}M{c['M']}{'t' if c['noise'] else 'g'}")
def test_dense_features_match_oracle(ctx, case):
    """Features of the dense-factor kernel (reference decisions read each noise coordinate against
    L_jj) against the oracle's, path by path, with the oracle replaying the logged decisions."""
    d, R, T = case["d"], case["R"], case["T"]
    mu, L = workloads.dense_instance(12, d, d)
    b = _ref(mu, np.diag(L))
    p = sim.Problem(mu=mu, chol=L, N=case["N"], M=case["M"], noise=case["noise"], nu=3,
                    checkpoints=(T,), gap_eps=0.05, instance_id=50 + d, keep_paths=True,
                    log_reps=(0, R), cv_features=True, cv_ref=b)
    say(f"[cv] dense features d={d} N={case['N']} M={case['M']} noise={case['noise']} R={R} T={T}")
    ctx.run(p, R, T, 78)
    g = ctx.paths()
    assert g["x"].shape == (d + 2, R)
    P = parity.oracle_problem(p, 78)
    law = oracle.CvLaw(P, T)
    inv = 1.0 / np.sqrt(law.S4 * np.maximum(law.probs * (1 - law.probs), 1e-4))
    amb1 = 1.0 / math.sqrt(law.S11 * max(law.probs[law.top] * (1 - law.probs[law.top]), 1e-4))
    err, amb = 0.0, 0
    for r in range(R):
        o = parity.check_rep(P, g, r, T, oracle.U32, decisions=g["decisions"][:, r])
        ref = law.path_features(o)
        e = np.abs(g["x"][:, r].astype(np.float64) - ref)
        tol = FEAT_ATOL + 1e-6 * np.abs(ref)
        tol[: d + 1] += o.cv_amb * inv.max()
        tol[d + 1] += math.sqrt(o.cv_amb) * amb1 * 4
        amb += o.cv_amb > 0
        err = max(err, e.max())
        assert np.all(e <= tol), f"rep {r}: feature errors {e}"
    say(f"[cv] dense max feature error {err:.2e}; replications with a near-tie reference decision: {amb}")


def test_dense_cv_fit_and_estimate(ctx):
    """The control variate on the dense-factor kernel (stress shape at a reduced horizon): trained on
    the device, the estimate agrees with the plain mean of the same paths within their joint CI;
    the variance ratio is reported."""
    d, N, T = 64, 100, 60
    mu, L = workloads.dense_instance(0, 0, d)
    p = sim.Problem(mu=mu, chol=L, N=N, noise=sim.NOISE_T, nu=3)
    fit = ctx.cv_fit(p, T, 5, n_runs=1, epochs=4, R_train=1 << 16, R_pilot=1 << 15, batch=4096, lr=2e-3)
    say(f"[cv] dense fit: loss {fit.loss_first_epoch:.4f} -> {fit.loss_last_epoch:.4f}, beta {fit.beta:.3f}, "
        f"rho2 {fit.rho2:.3f}")
    R, R_aux = 1 << 15, 1 << 19
    st = ctx.run_cv(p, R, T, 105, R_aux)
    joint = math.sqrt(st.ci95_plain ** 2 + st.ci95_cv ** 2) / 1.96
    gain = (st.var_plain / R) / st.var_est
    say(f"[cv] dense plain {st.mean_plain:.6f} +- {st.ci95_plain:.2e}, cv {st.mean_cv:.6f} +- {st.ci95_cv:.2e}, "
        f"variance gain {gain:.3f}, rho2 {st.rho2:.3f}")
    assert abs(st.mean_cv - st.mean_plain) <= 4.5 * joint
    assert math.isfinite(gain) and gain > 0
