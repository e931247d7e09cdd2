"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test would fail under a plausible slip in the oracle: a wrong Philox word or key schedule,
a biased uniform, a Box-Muller swap, N instead of N-1 in Eq. (4), a sign flip in the gradient,
the wrong triangle of L, independent instead of elliptical t noise, the wrong step size or
update, a dropped 1/2 in Eq. (3), a wrong tie rule in the linear subproblem, or a reduction slip.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import optimize, stats

import oracle
from paper_2404_11631_amd import workloads
from tests import exact_d1

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------------------------------
# Philox4x32-10 and the uniform / normal maps
# ------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_helper():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp(prefix="philox_pin_")
    exe = os.path.join(d, "rocrand_philox")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "pins", "rocrand_philox.cpp")])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_helper):
    """Library cross-check: rocRAND's philox4x32_10 on the same key and counter."""
    g = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(200):
        k0, k1, c0, c2, c3 = (int(x) for x in g.integers(0, 2 ** 32, 5))
        c1 = int(g.integers(0, 2 ** 30))          # keeps 4*(c0 | c1 << 32) inside 64 bits
        cases.append((k0, k1, c0, c1, c2, c3))
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    res = subprocess.run([rocrand_helper], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for c, line in zip(cases, lines):
        want = [int(v) for v in line.split()]
        got = oracle.philox([c[2], c[3], c[4], c[5]], [c[0], c[1]])
        assert got == want, (c, got, want)


def test_uniform_is_exact_odd_multiple():
    for x in [0, 1, 0x7FFFFF, 0x800000, 0xFFFFFFFF, 0x12345678, 0xDEADBEEF]:
        u = oracle.uniform(x)
        k = x & 0x7FFFFF
        assert u == (2 * k + 1) * 2.0 ** -24
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u        # identical in binary32 and binary64
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0x7FFFFF) == 1.0 - 2.0 ** -24


def test_normals_distribution():
    z = np.concatenate([oracle.normals(7, 0, 3, r, 11, 0, 4000) for r in range(50)])
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 4.0 * math.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 4.0 * math.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # Box-Muller truncation: |z| <= sqrt(-2 ln 2^-24)
    assert np.abs(z).max() <= math.sqrt(48.0 * math.log(2.0)) + 1e-12
    # the cos and sin halves of each pair are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 4.0 / math.sqrt(n / 2)


def test_normals_stream_layout():
    """Normal q depends only on Philox block q/4 of counter (block, epoch, rep, domain|instance)."""
    a = oracle.normals(5, 0, 9, 4, 2, 0, 12)
    b = oracle.normals(5, 0, 9, 4, 2, 4, 8)
    assert np.array_equal(a[4:], b)
    c = oracle.normals(5, 0, 9, 4, 3, 0, 12)     # another epoch: another block
    assert not np.any(a == c)
    x = oracle.philox([1, 2, 4, (0 << 24) | 9], [5, 0])
    u1, u2 = oracle.uniform(x[0]), oracle.uniform(x[1])
    r = math.sqrt(-2.0 * math.log(u1))
    assert a[4] == pytest.approx(r * math.cos(2 * math.pi * u2), rel=1e-15, abs=1e-15)
    assert a[5] == pytest.approx(r * math.sin(2 * math.pi * u2), rel=1e-15, abs=1e-15)


# ------------------------------------------------------------------------------------------
# Sampling laws behind Eq. (4)-(5)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dense", [False, True])
@pytest.mark.parametrize("N", [2, 7])
def test_sample_covariance_chi2_law(dense, N):
    """(N-1) w'Sigma_hat w / w'Sigma w ~ chi2_{N-1} and Rbar ~ N(mu, Sigma/N) for Gaussian returns."""
    d = 5
    if dense:
        mu, L = workloads.dense_instance(3, 1, d)
    else:
        mu, sigma = workloads.diag_instance(3, 1, d)
        L = np.diag(sigma)
    P = oracle.OracleProblem(mu, chol=L, N=N, seed=17)
    Sigma = L @ L.T
    w = np.array([0.1, 0.3, 0.0, 0.2, 0.25])
    u = np.array([0.4, -0.2, 0.5, 0.1, -0.3])       # direction for the mean test
    q, m = [], []
    for r in range(3000):
        g, rbar, sw = P.sample_gradient(r, 0, w)
        q.append((N - 1) * (w @ sw) / (w @ Sigma @ w))
        m.append((u @ (rbar - mu)) / math.sqrt(u @ Sigma @ u / N))
    assert stats.kstest(q, stats.chi2(N - 1).cdf).pvalue > 1e-3
    assert stats.kstest(m, "norm").pvalue > 1e-3


def test_gradient_unbiased():
    """E[2 lambda Sigma_hat w - Rbar] = 2 lambda Sigma w - mu, the gradient of Eq. (3)."""
    d, N, lam = 4, 5, 0.5
    mu, L = workloads.dense_instance(11, 0, d)
    P = oracle.OracleProblem(mu, chol=L, N=N, lam=lam, seed=3)
    w = np.array([0.2, 0.1, 0.4, 0.05])
    G = np.array([P.sample_gradient(r, 1, w)[0] for r in range(6000)])
    want = 2 * lam * (L @ L.T) @ w - mu
    se = G.std(axis=0, ddof=1) / math.sqrt(G.shape[0])
    assert np.all(np.abs(G.mean(axis=0) - want) < 4.5 * se)


def test_student_t_noise_is_elliptical_and_standardised():
    d, N, nu = 3, 4, 3
    P = oracle.OracleProblem(np.zeros(d), chol=np.eye(d), N=N, noise=oracle.NOISE_T, nu=nu, seed=21)
    Y = np.concatenate([P.draw_returns(r, 0) for r in range(4000)])
    scale = math.sqrt((nu - 2) / nu)
    assert stats.kstest(Y[:, 0], stats.t(nu, scale=scale).cdf).pvalue > 1e-3
    # one chi2 per sample scales all coordinates: ratios of coordinates are standard Cauchy
    assert stats.kstest(Y[:, 1] / Y[:, 2], "cauchy").pvalue > 1e-3
    # the quadratic form y'y / d follows an F(d, nu) law up to the (nu-2)/nu scale
    F = (Y ** 2).sum(axis=1) / d / ((nu - 2) / nu)
    assert stats.kstest(F, stats.f(d, nu).cdf).pvalue > 1e-3


# ------------------------------------------------------------------------------------------
# Algorithm 1: identity of the step rule, feasibility, invariants
# ------------------------------------------------------------------------------------------
def kkt_fstar(mu, sigma, lam):
    """min over W of lambda sum sigma_j^2 w_j^2 - mu'w by KKT water-filling."""
    mu = np.asarray(mu, float)
    a = 2.0 * lam * np.asarray(sigma, float) ** 2

    def w_of(nu):
        return np.maximum(0.0, (mu - nu) / a)

    if w_of(0.0).sum() <= 1.0:
        w = w_of(0.0)
    else:
        lo, hi = 0.0, float(mu.max())
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if w_of(mid).sum() > 1.0:
                lo = mid
            else:
                hi = mid
        w = w_of(hi)
    return float(lam * np.sum(np.asarray(sigma) ** 2 * w ** 2) - mu @ w), w


def test_kkt_matches_generic_solver():
    for inst in range(5):
        mu, sigma = workloads.diag_instance(1, inst, 6)
        for lam in (0.5, 1.0):
            f, w = kkt_fstar(mu, sigma, lam)
            obj = lambda x: lam * np.sum(sigma ** 2 * x ** 2) - mu @ x
            res = optimize.minimize(obj, np.full(6, 1.0 / 6), method="SLSQP", bounds=[(0, 1)] * 6,
                                    constraints=[{"type": "ineq", "fun": lambda x: 1.0 - x.sum()}],
                                    options={"ftol": 1e-14, "maxiter": 500})
            assert res.fun >= f - 1e-9
            assert abs(res.fun - f) < 1e-7


@pytest.mark.parametrize("M", [1, 5])
@pytest.mark.parametrize("lam", [0.5, 1.0])
def test_identity_invariants_and_lower_bound(M, lam):
    d, N, T = 6, 4, 300
    mu, sigma = workloads.diag_instance(2, 5, d)
    w0 = np.array([0.1, 0.0, 0.2, 0.0, 0.3, 0.1])
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, lam=lam, w0=w0, seed=9, ckpt=(1, 50, 300))
    fstar, _ = kkt_fstar(mu, sigma, lam)
    for r in range(40):
        out, dec = P.path(r, T, want_decisions=True)
        # w_T = 2/(T(T+1)) sum_t (t+1) s_t, whatever w_0 is (step 2/(t+2) makes gamma_0 = 1)
        assert out.identity_err < 1e-12
        cnt = np.bincount(dec, minlength=d + 1)
        assert np.array_equal(cnt, np.array(out.cnt[: d + 1]))
        for j in range(d):
            assert out.wsum[j] == int(np.sum(np.nonzero(dec == j + 1)[0] + 1))
        assert sum(out.cnt[: d + 1]) == T
        wT = 2.0 * np.array(out.wsum[:d], dtype=float) / (T * (T + 1.0))
        assert np.all(wT >= 0) and wT.sum() <= 1.0 + 1e-15
        # every outcome is a feasible objective value: Y >= min over W
        assert out.y >= fstar - 1e-12
        assert out.f_ckpt[2] == out.y
        # after the first step w_1 = s_0: the checkpoint at 1 is f at a vertex
        a0 = dec[0]
        f1 = 0.0 if a0 == 0 else lam * sigma[a0 - 1] ** 2 - mu[a0 - 1]
        assert out.f_ckpt[0] == pytest.approx(f1, rel=1e-14, abs=1e-15)


def test_epoch_layout_of_resampling():
    """Steps kM .. kM+M-1 all use the sample of epoch k (counter word 1 = k): each decision equals
    the vertex rule applied to that epoch's gradient at the iterate w_t = 2 S_t/(t(t+1))."""
    d, N, M, T = 3, 4, 5, 40
    mu, sigma = np.array([0.5, 0.55, 0.45]), np.array([0.6, 0.7, 0.5])
    P = oracle.OracleProblem(mu, sigma, N=N, M=M, seed=13)
    out, dec = P.path(1, T, want_decisions=True)
    assert len(set(dec.tolist())) >= 3           # the case exercises several vertices
    S = np.zeros(d)
    for t in range(T):
        w = np.zeros(d) if t == 0 else 2.0 * S / (t * (t + 1.0))
        g = P.sample_gradient(1, t // M, w)[0]
        j = int(np.argmin(g))
        a = j + 1 if g[j] < 0 else 0
        assert dec[t] == a
        if a:
            S[a - 1] += t + 1


def test_zero_noise_picks_best_mean():
    """sigma = 0: the gradient is -mu, every step picks argmax mu, Y = -max(mu)_+."""
    mu = np.array([0.2, 0.9, 0.9, 0.1])
    P = oracle.OracleProblem(mu, np.zeros(4), N=3, seed=1, ckpt=(10,))
    out, dec = P.path(0, 64, want_decisions=True)
    assert np.all(dec == 2)                      # tie between assets 2 and 3 goes to the lower index
    assert out.y == -0.9
    P = oracle.OracleProblem(-mu, np.zeros(4), N=3, seed=1)
    out, dec = P.path(0, 64, want_decisions=True)
    assert np.all(dec == 0) and out.y == 0.0     # all means negative: stay at the origin


def test_zero_minimum_goes_to_origin():
    """A zero smallest gradient entry keeps the origin (the vertex 0 of W attains the same value)."""
    mu = np.array([-0.5, 0.0, -0.2])
    P = oracle.OracleProblem(mu, np.zeros(3), N=2, seed=1)
    out, dec = P.path(0, 16, want_decisions=True)
    assert np.all(dec == 0) and out.cnt[0] == 16


def test_dominant_asset_pins_half_variance():
    """One asset dominates every sample: w_T = e_1 and Y = sigma_1^2/2 - mu_1 (Eq. (3) at a vertex)."""
    mu = np.array([50.0, 0.1, 0.2])
    sigma = np.array([0.3, 0.2, 0.1])
    for lam in (0.5, 1.0):
        P = oracle.OracleProblem(mu, sigma, N=5, lam=lam, seed=4)
        out = P.path(3, 200)
        assert out.cnt[1] == 200
        assert out.y == pytest.approx(lam * 0.09 - 50.0, rel=1e-15)


def test_fixed_sample_converges_on_sample_objective():
    """M = T keeps one sample: Algorithm 1 is deterministic Frank-Wolfe on f_hat of Eq. (4), and
    f_hat(w_t) - min f_hat <= 8 lambda lambda_max(Sigma_hat)/(t+2) (Jaggi 2013, Theorem 1)."""
    d, N, T, lam = 5, 8, 400, 0.5
    mu, L = workloads.dense_instance(4, 2, d)
    P = oracle.OracleProblem(mu, chol=L, N=N, M=T, lam=lam, seed=8)
    for r in range(5):
        out = P.path(r, T)
        Rm = P.draw_returns(r, 0)
        S = np.cov(Rm, rowvar=False, ddof=1)
        rbar = Rm.mean(axis=0)
        fhat = lambda x: lam * x @ S @ x - rbar @ x
        res = optimize.minimize(fhat, np.full(d, 1.0 / d), method="SLSQP", bounds=[(0, 1)] * d,
                                constraints=[{"type": "ineq", "fun": lambda x: 1.0 - x.sum()}],
                                options={"ftol": 1e-15, "maxiter": 1000})
        wT = 2.0 * np.array(out.wsum[:d], dtype=float) / (T * (T + 1.0))
        gap = fhat(wT) - res.fun
        assert gap >= -1e-9
        assert gap <= 8 * lam * np.linalg.eigvalsh(S).max() / (T + 2)


# ------------------------------------------------------------------------------------------
# Exact law at d = 1 (dynamic program over the integer signature)
# ------------------------------------------------------------------------------------------
def test_d1_pick_probability_closed_form_and_mc():
    mu, sigma, N, lam = 0.3, 0.8, 4, 0.5
    assert exact_d1.pick_probability(0.0, mu, sigma, N, lam)[0] == pytest.approx(
        stats.norm.cdf(mu * math.sqrt(N) / sigma), rel=1e-12)
    g = np.random.default_rng(0)
    X = g.normal(mu, sigma, size=(400_000, N))
    w = 0.6
    p_mc = np.mean(2 * lam * X.var(axis=1, ddof=1) * w - X.mean(axis=1) < 0)
    p = exact_d1.pick_probability(w, mu, sigma, N, lam)[0]
    assert abs(p_mc - p) < 4 * math.sqrt(p * (1 - p) / 400_000)


def test_d1_dynamic_program_matches_enumeration():
    for (mu, sigma, N, lam, w0) in [(0.3, 0.8, 2, 0.5, 0.0), (0.5, 0.4, 5, 1.0, 0.7)]:
        a = exact_d1.wsum_law(7, mu, sigma, N, lam, w0)
        b = exact_d1.wsum_law_bruteforce(7, mu, sigma, N, lam, w0)
        assert np.allclose(a, b, atol=1e-14)
        assert a.sum() == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("mu,sigma,N,lam", [(0.3, 0.8, 2, 0.5), (0.5, 0.4, 5, 1.0), (0.2, 1.0, 3, 0.5)])
def test_d1_oracle_matches_exact_law(mu, sigma, N, lam):
    T, R = 20, 20_000
    P = oracle.OracleProblem([mu], [sigma], N=N, lam=lam, seed=2024)
    outs = P.run(R, T)
    S = np.array([o.wsum[0] for o in outs])
    Y = np.array([o.y for o in outs])
    law = exact_d1.wsum_law(T, mu, sigma, N, lam)
    m, v = exact_d1.outcome_moments(T, mu, sigma, N, lam)
    assert abs(Y.mean() - m) < 4.0 * math.sqrt(v / R)
    # chi-square goodness of fit of S_T, pooling cells with expected count < 20
    exp = law * R
    obs = np.bincount(S, minlength=law.shape[0]).astype(float)
    order = np.arange(law.shape[0])
    cells_o, cells_e, acc_o, acc_e = [], [], 0.0, 0.0
    for i in order:
        acc_o += obs[i]
        acc_e += exp[i]
        if acc_e >= 20:
            cells_o.append(acc_o)
            cells_e.append(acc_e)
            acc_o = acc_e = 0.0
    cells_o[-1] += acc_o
    cells_e[-1] += acc_e
    chi2 = float(np.sum((np.array(cells_o) - np.array(cells_e)) ** 2 / np.array(cells_e)))
    dof = len(cells_o) - 1
    assert stats.chi2(dof).sf(chi2) > 1e-4


# ------------------------------------------------------------------------------------------
# Reductions and Table 2's relative squared error
# ------------------------------------------------------------------------------------------
def test_reduce_against_fsum():
    d, T = 3, 120
    mu, sigma = workloads.diag_instance(0, 7, d)
    ck = (50, 100, 120)
    P = oracle.OracleProblem(mu, sigma, N=3, seed=5, ckpt=ck, gap_eps=0.05)
    outs = P.run(500, T)
    st = P.reduce(outs, T)
    Y, F, cnt, wsum, tau = oracle.path_arrays(outs, d, len(ck))
    mean = math.fsum(Y) / len(Y)
    assert st.mean == pytest.approx(mean, rel=1e-15)
    var = math.fsum((y - mean) ** 2 for y in Y) / (len(Y) - 1)
    assert st.var == pytest.approx(var, rel=1e-13)
    assert st.ci95 == pytest.approx(1.96 * math.sqrt(var / len(Y)), rel=1e-13)
    assert st.ymin == Y.min() and st.ymax == Y.max()
    for c in range(len(ck)):
        ok = F[:, c] != 0
        rse = ((F[ok, c] - Y[ok]) / F[ok, c]) ** 2
        assert st.rse_undef[c] == int((~ok).sum())
        assert st.rse_mean[c] == pytest.approx(math.fsum(rse) / len(rse), rel=1e-13)
        assert st.rse_sd[c] == pytest.approx(np.std(rse, ddof=1), rel=1e-10)
        assert st.f_mean[c] == pytest.approx(math.fsum(F[:, c]) / len(Y), rel=1e-13)
    assert st.rse_mean[2] == 0.0                # the last checkpoint is the final value
    assert list(st.decision_total)[: d + 1] == list(cnt.sum(axis=0))
    hit = tau != oracle.TAU_NONE
    assert st.tau_count == int(hit.sum())
    assert st.tau_mean == pytest.approx(tau[hit].mean(), rel=1e-15)


def test_rse_undefined_at_origin():
    mu = -np.ones(2)
    P = oracle.OracleProblem(mu, np.full(2, 0.01), N=2, seed=1, ckpt=(5,))
    outs = P.run(10, 5)
    st = P.reduce(outs, 5)
    assert st.rse_undef[0] == 10 and st.mean == 0.0


def test_ambiguity_replay_protocol():
    """A replayed sequence equal to the oracle's own is never a mismatch; a replayed sequence
    that differs at an unambiguous step is."""
    d, T = 4, 200
    mu, sigma = workloads.diag_instance(0, 1, d)
    P = oracle.OracleProblem(mu, sigma, N=5, seed=3)
    out, dec = P.path(2, T, want_decisions=True)
    same = P.path(2, T, replay=dec, uroff=oracle.U32)
    assert same.n_mismatch == 0 and same.n_replayed == 0
    assert same.y == out.y
    bad = dec.copy()
    bad[150] = (bad[150] + 1) % (d + 1)
    worse = P.path(2, T, replay=bad, uroff=oracle.U64)
    assert worse.n_mismatch >= 1 and worse.first_mismatch == 150


# ------------------------------------------------------------------------------------------
# Per-epoch sample sizes N_k (the remark on Algorithm 1's resampling step)
# ------------------------------------------------------------------------------------------
def test_constant_schedule_is_the_plain_run():
    d, T, M = 4, 90, 3
    mu, sigma = workloads.diag_instance(3, 1, d)
    plain = oracle.OracleProblem(mu, sigma, N=6, M=M, seed=7, ckpt=(30, 90), gap_eps=0.05)
    sched = oracle.OracleProblem(mu, sigma, N=6, M=M, seed=7, ckpt=(30, 90), gap_eps=0.05,
                                 n_sched=[6] * (T // M))
    for r in range(5):
        a, b = plain.path(r, T), sched.path(r, T)
        assert a.y == b.y and list(a.cnt) == list(b.cnt) and list(a.wsum) == list(b.wsum)
        assert a.tau == b.tau and list(a.f_ckpt) == list(b.f_ckpt)


def test_schedule_draws_epoch_k_with_its_own_size():
    """An epoch with N_k samples draws normals 0 .. N_k d - 1 of its stream: the first decision of a
    schedule starting at N_0 equals the plain run's with N = N_0, and the runs part once N_k moves."""
    d, T = 3, 40
    mu, sigma = workloads.diag_instance(4, 2, d)
    grow = [2 + k for k in range(T)]
    sched = oracle.OracleProblem(mu, sigma, N=2, seed=9, n_sched=grow)
    for r in range(40):
        _, ds = sched.path(r, 1, want_decisions=True)
        _, dp = oracle.OracleProblem(mu, sigma, N=2, seed=9).path(r, 1, want_decisions=True)
        assert ds[0] == dp[0]
    same = sum(sched.path(r, T).y == oracle.OracleProblem(mu, sigma, N=2, seed=9).path(r, T).y for r in range(40))
    assert same < 40
    with pytest.raises(ValueError):
        oracle.OracleProblem(mu, sigma, N=2, seed=9, n_sched=[2, 1] + grow[2:]).path(0, T)


@pytest.mark.parametrize("sched", ["growing", "geometric"])
def test_d1_schedule_matches_exact_law(sched):
    """d = 1, fresh samples every step with N_t from a schedule: the oracle's S_T against the exact
    dynamic program with the same per-step sample sizes."""
    mu, sigma, lam, T, R = 0.3, 0.8, 0.5, 20, 20_000
    Ns = [2 + t for t in range(T)] if sched == "growing" else [int(2 * 1.25 ** t) for t in range(T)]
    P = oracle.OracleProblem([mu], [sigma], N=2, lam=lam, seed=4048, n_sched=Ns)
    outs = P.run(R, T)
    S = np.array([o.wsum[0] for o in outs])
    law = exact_d1.wsum_law(T, mu, sigma, Ns, lam)
    # the constant-N law is visibly different, so the test can tell a schedule that is ignored
    const = exact_d1.wsum_law(T, mu, sigma, 2, lam)
    idx = np.arange(law.shape[0])
    assert abs((law * idx).sum() - (const * idx).sum()) > 6 * math.sqrt((law * idx ** 2).sum() / R)
    exp = law * R
    obs = np.bincount(S, minlength=law.shape[0]).astype(float)
    cells_o, cells_e, acc_o, acc_e = [], [], 0.0, 0.0
    for i in range(law.shape[0]):
        acc_o += obs[i]
        acc_e += exp[i]
        if acc_e >= 20:
            cells_o.append(acc_o)
            cells_e.append(acc_e)
            acc_o = acc_e = 0.0
    cells_o[-1] += acc_o
    cells_e[-1] += acc_e
    chi2 = float(np.sum((np.array(cells_o) - np.array(cells_e)) ** 2 / np.array(cells_e)))
    assert stats.chi2(len(cells_o) - 1).sf(chi2) > 1e-4
