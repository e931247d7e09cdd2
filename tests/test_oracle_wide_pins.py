"""Pins of the oracle for Algorithm 1 at the paper's experimental shape (oracle/wide.c).

Section 4.1 runs Algorithm 1 with many assets (d up to 1e5), N = 25 or 50 samples per gradient and
a diagonal Sigma. The wide oracle takes sigma as a vector and sizes its arrays by d; these tests pin
it to the narrow oracle where both apply, to closed forms, to an independent covariance evaluation
and to the rounding bound it reports.
"""
import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import workloads


def wide_and_narrow(d, N, M=1, seed=3, w0=None, ckpt=(), regime="unit", instance=0):
    mu, sig = workloads.diag_instance(seed, instance, d, regime)
    W = oracle.WideOracle(mu, sig, N=N, M=M, seed=seed, w0=w0, ckpt=ckpt, instance=instance)
    P = oracle.OracleProblem(mu, sig, N=N, M=M, seed=seed, w0=w0, ckpt=ckpt, instance=instance)
    return W, P


@pytest.mark.parametrize("d,N,M,T,use_w0", [(2, 2, 1, 60, False), (12, 5, 1, 80, False), (40, 9, 3, 70, True),
                                            (64, 25, 1, 30, False)])
def test_wide_equals_narrow_oracle(d, N, M, T, use_w0):
    """Where both apply (d <= 64, diagonal Sigma) the two oracles take the same decisions and give
    the same f(w_T), checkpoints, counts and signatures."""
    w0 = np.full(d, 0.5 / d) if use_w0 else None
    W, P = wide_and_narrow(d, N, M, w0=w0, ckpt=(5, T))
    for rep in (0, 7):
        o = W.path(rep, T)
        po, dec = P.path(rep, T, want_decisions=True)
        assert np.array_equal(o["decisions"], dec.astype(np.uint32))
        assert o["y"] == pytest.approx(po.y, rel=1e-14, abs=1e-15)
        assert np.allclose(o["f_ckpt"], list(po.f_ckpt[:2]), rtol=1e-14, atol=1e-15)
        assert list(o["cnt"]) == list(po.cnt[:d + 1])
        assert list(o["wsum"]) == list(po.wsum[:d])
        assert o["tau"] == po.tau


@pytest.mark.parametrize("d", [7, 1000])
def test_zero_noise_closed_form(d):
    """sigma = 0: every gradient is -mu, so the path picks the asset of largest mean at every step
    (the origin when every mean is negative) and f(w_T) = -max(max_j mu_j, 0)."""
    rng = np.random.default_rng(d)
    for shift in (0.0, -2.0):
        mu = rng.uniform(-1, 1, d) + shift
        W = oracle.WideOracle(mu, np.zeros(d), N=4, seed=1)
        o = W.path(0, 50)
        best = int(np.argmax(mu))
        if mu[best] > 0:
            assert (o["decisions"] == best + 1).all()
            assert o["y"] == pytest.approx(-mu[best], abs=1e-15)
        else:
            assert (o["decisions"] == 0).all()
            assert o["y"] == 0.0


def test_gradient_against_numpy_covariance():
    """The sample gradient 2 lambda Sigma_hat w - Rbar of Eq. (4)-(5) against numpy's own sample
    covariance (ddof 1) of the same returns, at a random point of W."""
    d, N, seed = 300, 7, 11
    mu, sig = workloads.diag_instance(seed, 0, d, "paper")
    W = oracle.WideOracle(mu, sig, N=N, seed=seed, lam=0.7)
    rng = np.random.default_rng(0)
    w = rng.dirichlet(np.ones(d)) * 0.8
    for rep, epoch in ((0, 0), (3, 5)):
        z = oracle.normals(seed, 0, 0, rep, epoch, 0, N * d).reshape(N, d)
        R = mu + sig * z
        ref = 2 * 0.7 * (np.cov(R.T, ddof=1) @ w) - R.mean(0)
        g, _ = W.gradient(rep, epoch, w)
        assert np.allclose(g, ref, rtol=1e-11, atol=1e-14)


def test_identity_and_replay():
    """The signature identity w_T = 2 wsum / (T (T+1)); replaying the oracle's own decisions is
    clean, and a wrong decision at a step whose margin exceeds the bound is a mismatch."""
    W, _ = wide_and_narrow(200, 25, regime="paper", ckpt=(10, 100))
    o = W.path(1, 100, uroff=2.0 ** -24)
    assert o["identity_err"] < 1e-13
    again = W.path(1, 100, replay=o["decisions"], uroff=2.0 ** -24)
    assert again["n_mismatch"] == 0 and again["y"] == o["y"]
    bad = o["decisions"].copy()
    t = 50
    bad[t] = 0 if bad[t] != 0 else 1
    w = W.path(1, 100, replay=bad, uroff=0.0)
    assert w["n_mismatch"] >= 1 and w["first_mismatch"] == t


@pytest.mark.parametrize("d,N", [(100, 25), (3000, 50)])
def test_bound_covers_a_binary32_evaluation(d, N):
    """The rounding bound the oracle reports for unit roundoff 2^-24 covers a binary32 evaluation of
    the same gradient in noise coordinates (numpy float32: sums over samples in order, sums over
    assets pairwise), at points of W along the path."""
    seed = 5
    mu, sig = workloads.diag_instance(seed, 0, d, "paper")
    W = oracle.WideOracle(mu, sig, N=N, seed=seed)
    rng = np.random.default_rng(1)
    for k in range(3):
        w = rng.dirichlet(np.ones(d)) * rng.uniform(0.2, 1.0)
        g64, bound = W.gradient(0, k, w, uroff=2.0 ** -24)
        z = oracle.normals(seed, 0, 0, 0, k, 0, N * d).reshape(N, d).astype(np.float32)
        v = (sig * w).astype(np.float32)
        dots = (z * v).sum(axis=1, dtype=np.float32)
        s1 = np.zeros(d, np.float32)
        s2 = np.zeros(d, np.float32)
        for i in range(N):
            s1 += z[i]
            s2 += z[i] * dots[i]
        qn = np.float32((s1 * v).sum(dtype=np.float32) / np.float32(N))
        c2 = (2 * 0.5 * sig / (N - 1)).astype(np.float32)
        g32 = c2 * (s2 - s1 * qn) - mu.astype(np.float32) - (sig / N).astype(np.float32) * s1
        err = np.abs(g32.astype(np.float64) - g64).max()
        assert err <= bound, (err, bound)
        assert bound < 1e-2 * np.abs(g64).max()


# ---- adaptive sample sizes N_k (Algorithm 1 lets the resample size depend on the epoch) ----------

def test_constant_schedule_is_the_plain_run():
    mu, sig = workloads.diag_instance(4, 0, 30)
    plain = oracle.WideOracle(mu, sig, N=7, M=2, seed=4, ckpt=(9, 40))
    sched = oracle.WideOracle(mu, sig, N=7, M=2, seed=4, ckpt=(9, 40), n_sched=[7] * 20)
    for rep in (0, 3):
        a, b = plain.path(rep, 40), sched.path(rep, 40)
        assert np.array_equal(a["decisions"], b["decisions"]) and a["y"] == b["y"]
        assert np.array_equal(a["f_ckpt"], b["f_ckpt"])


def test_schedule_applies_each_epochs_size():
    """The gradient of epoch k with a schedule is the plain gradient with N = N_k (same stream: the
    first N_k returns of the (replication, epoch) draw), and the path's decisions are those of a
    path whose epochs are run with their own N."""
    d = 20
    mu, sig = workloads.diag_instance(5, 0, d)
    sch = [2, 9, 3, 30, 4]
    S = oracle.WideOracle(mu, sig, N=5, M=3, seed=6, n_sched=sch)
    w = np.random.default_rng(0).dirichlet(np.ones(d)) * 0.8
    for k, Nk in enumerate(sch):
        g, _ = S.gradient(1, k, w)
        ref, _ = oracle.WideOracle(mu, sig, N=Nk, M=3, seed=6).gradient(1, k, w)
        assert np.array_equal(g, ref)
    full = S.path(1, 15)
    for k, Nk in enumerate(sch):
        # epoch k alone, from the iterate the schedule's path reached, with the plain oracle at N_k:
        # the first decision of the epoch is the vertex of that gradient
        t = 3 * k
        dec = full["decisions"][:t]
        wt = np.zeros(d)
        for s, a in enumerate(dec):
            gamma = 2.0 / (s + 2.0)
            wt = (1 - gamma) * wt
            if a:
                wt[a - 1] += gamma
        g, _ = oracle.WideOracle(mu, sig, N=Nk, M=3, seed=6).gradient(1, k, wt)
        own = int(np.argmin(g)) + 1 if g.min() < 0 else 0
        assert full["decisions"][t] == own


def test_schedule_sample_mean_variance_and_covariance_bias():
    """At w = 0 the gradient is -Rbar with Rbar_j ~ N(mu_j, sigma_j^2 / N_k): the spread over epochs
    scales with 1/N_k (chi-square bounds); at w != 0, (g + Rbar)/(2 lambda) = Sigma_hat w averages to
    Sigma w for every N_k (the 1/(N_k - 1) of Eq. (4)), here with N_k = 3 where 1/N_k would be off by 1/3."""
    from scipy import stats
    d = 6
    mu, sig = workloads.diag_instance(7, 0, d)
    E = 600
    sch = [4 if k % 2 == 0 else 64 for k in range(E)]
    S = oracle.WideOracle(mu, sig, N=4, seed=8, n_sched=sch)
    g = np.array([S.gradient(0, k, np.zeros(d))[0] for k in range(E)])
    for par, Nk in ((0, 4), (1, 64)):
        x = g[par::2]
        q = ((x + mu) ** 2 / (sig ** 2 / Nk)).sum(axis=0)          # sum of E/2 chi2(1) per asset
        lo, hi = stats.chi2.ppf([1e-4, 1 - 1e-4], E // 2)
        assert np.all((q > lo) & (q < hi)), (Nk, q)
    w = np.full(d, 1.0 / d)
    S3 = oracle.WideOracle(mu, sig, N=3, seed=9, n_sched=[3] * 4000)
    est = []
    for k in range(4000):
        gk, _ = S3.gradient(0, k, w)
        est.append(gk)
    # E g = 2 lambda Sigma w - mu with lambda = 1/2
    m = np.mean(est, axis=0)
    se = np.std(est, axis=0, ddof=1) / np.sqrt(4000)
    assert np.all(np.abs(m - (sig ** 2 * w - mu)) < 5 * se)
