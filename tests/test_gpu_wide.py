"""Algorithm 1 at the paper's experimental shape (sim_run_wide: many assets, diagonal Sigma, a few
replications, parallel over assets and samples) vs the CPU oracle through the C ABI (needs an
MI355X).

Protocol: the oracle for this shape (oracle/wide.c) replays the device's decisions; every decision
outside the oracle's rounding bound for a binary32 system must be the oracle's own (bit-exact
vertex), counts and signatures must then match exactly, f(w_T) and f(w_c) to 1e-11 relative (FP64
from the exact signature on both sides), tau inside the bound's range, statistics to 1e-10 / 1e-8.
Section 4.1's d = 1e4 run (N = 25, K = 1500) is replayed in full; at its largest shape (d = 1e5,
N = 50, K = 1500) the oracle checks sampled iterations: the gradient at the device's own iterate and
the vertex the device took there.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import sim, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    s = sim.Sim(0)
    yield s
    s.close()


def close(a, b, rtol, atol):
    return abs(a - b) <= atol + rtol * abs(b)


def problem(d, N, M=1, seed=0, regime="paper", w0=False, ckpt=(), lam=0.5, instance=0, gap_eps=1e-2):
    mu, sig = workloads.diag_instance(seed, instance, d, regime)
    w = np.full(d, 0.5 / d) if w0 else None
    return sim.Problem(mu=mu, sigma=sig, N=N, M=M, lam=lam, w0=w, checkpoints=ckpt, instance_id=instance,
                       gap_eps=gap_eps)


def wide_oracle(p, seed):
    return oracle.WideOracle(p.mu, p.sigma, N=p.N, M=p.M, lam=p.lam, w0=p.w0, seed=seed, instance=p.instance_id,
                             ckpt=p.checkpoints, gap_eps=p.gap_eps, n_sched=p.n_schedule)


def run_and_compare(ctx, p, R, T, seed):
    d = len(p.mu)
    say(f"[wide] d={d} N={p.N} M={p.M} lam={p.lam} w0={p.w0 is not None} R={R} T={T} seed={seed} "
        f"schedule={None if p.n_schedule is None else (min(p.n_schedule), max(p.n_schedule))}")
    ctx.run_wide(p, R, T, seed)
    st = ctx.wide_stats()
    g = ctx.wide_paths()
    W = wide_oracle(p, seed)
    ys, fcs, replayed = [], [], 0
    for r in range(R):
        o = W.path(r, T, replay=g["decisions"][r], uroff=oracle.U32)
        assert o["n_mismatch"] == 0, f"rep {r}: {o['n_mismatch']} mismatches, first at {o['first_mismatch']}"
        replayed += o["n_replayed"]
        assert np.array_equal(g["decisions"][r], o["decisions"])
        assert np.array_equal(g["cnt"][r], o["cnt"]), f"rep {r} cnt"
        assert np.array_equal(g["wsum"][r], o["wsum"]), f"rep {r} wsum"
        assert close(g["y"][r], o["y"], 1e-11, 1e-14), (g["y"][r], o["y"])
        for c in range(len(p.checkpoints)):
            assert close(g["f_ckpt"][c, r], o["f_ckpt"][c], 1e-11, 1e-14)
        assert o["tau_lo"] <= int(g["tau"][r]) <= o["tau_hi"], (g["tau"][r], o["tau_lo"], o["tau_hi"])
        ys.append(o["y"])
        fcs.append(o["f_ckpt"])
    ys = np.array(ys)
    assert st.R == R and st.T == T
    assert close(st.mean, ys.mean(), 1e-10, 1e-14)
    if R > 1:   # identical outcomes leave a variance at the level of double rounding of mean^2
        assert close(st.var, ys.var(ddof=1), 1e-8, 1e-15 * ys.mean() ** 2)
    assert st.min == g["y"].min() and st.max == g["y"].max()
    assert close(st.min, ys.min(), 1e-11, 1e-14) and close(st.max, ys.max(), 1e-11, 1e-14)
    assert st.decision_total[0] == int(g["cnt"][:, 0].sum())
    assert int(g["cnt"].sum()) == R * T
    for c in range(len(p.checkpoints)):
        assert close(st.f_mean[c], np.mean([f[c] for f in fcs]), 1e-10, 1e-14)
    say(f"[wide] ok, replayed ambiguous decisions: {replayed} of {R * T}; {st.kernel_ms:.2f} ms")
    return st, g


@pytest.mark.parametrize("case", [
    dict(d=4, N=2, T=80, R=3, ckpt=(1, 80)),
    dict(d=128, N=25, T=200, R=2, ckpt=(50, 100, 200)),
    dict(d=500, N=25, T=150, R=3, ckpt=(150,)),                 # 125 quads: a ragged last workgroup
    dict(d=1000, N=7, M=3, T=120, R=2, w0=True, lam=1.0, ckpt=(7, 120)),
    dict(d=4096, N=50, T=60, R=1, ckpt=(60,), regime="unit"),
    dict(d=10_000, N=25, T=1500, R=1, ckpt=(50, 100, 500, 1000, 1500)),   # Section 4.1, d = 1e4: the full run
])
def test_wide_against_oracle(ctx, case):
    c = dict(case)
    R, T = c.pop("R"), c.pop("T")
    d, N = c.pop("d"), c.pop("N")
    p = problem(d, N, M=c.pop("M", 1), w0=c.pop("w0", False), ckpt=c.pop("ckpt", ()), lam=c.pop("lam", 0.5),
                regime=c.pop("regime", "paper"))
    run_and_compare(ctx, p, R, T, seed=11)


def test_wide_deterministic(ctx):
    """Every sum runs in a fixed order: two runs give the same bits."""
    p = problem(2000, 25, ckpt=(100,))
    ctx.run_wide(p, 2, 100, 5)
    a = ctx.wide_paths()
    ctx.run_wide(p, 2, 100, 5)
    b = ctx.wide_paths()
    assert np.array_equal(a["decisions"], b["decisions"])
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["f_ckpt"], b["f_ckpt"])


def test_wide_zero_noise(ctx):
    """sigma = 0: the gradient is -mu at every step, so every decision is the asset of largest mean and
    f(w_T) = -max(mu) (closed form, no oracle)."""
    d = 3000
    mu, _ = workloads.diag_instance(2, 0, d, "paper")
    p = sim.Problem(mu=mu, sigma=np.zeros(d), N=25)
    ctx.run_wide(p, 1, 50, 1)
    g = ctx.wide_paths()
    assert (g["decisions"] == int(np.argmax(mu)) + 1).all()
    assert g["y"][0] == pytest.approx(-mu.max(), abs=1e-15)


def test_wide_errors(ctx):
    p = problem(102, 25)                       # not a multiple of 4
    with pytest.raises(sim.SimError):
        ctx.run_wide(p, 1, 10, 0)
    p = problem(128, 25)
    with pytest.raises(sim.SimError):
        ctx.run_wide(p, 65, 10, 0)              # above SIM_WIDE_MAX_R


def test_paper_shape_sampled(ctx):
    """Section 4.1's largest run: d = 1e5 assets, N = 50, K = 1500 iterations, mu ~ U(-1,1),
    sigma ~ U(0, 0.025), one replication. At sampled iterations the oracle recomputes the gradient at
    the device's iterate (rebuilt exactly from the device's decisions) and checks the vertex the device
    took: the oracle's own unless the margin is within its binary32 rounding bound, and then within
    the bound of the best. The final f(w_T) against the oracle's objective at the device's iterate."""
    d, N, T, seed = 100_000, 50, 1500, 0
    p = problem(d, N, ckpt=(50, 100, 500, 1000, 1500))
    say(f"[wide] paper shape d={d} N={N} T={T}")
    ctx.run_wide(p, 1, T, seed)
    st = ctx.wide_stats()
    g = ctx.wide_paths()
    say(f"[wide] paper shape: {st.kernel_ms:.1f} ms for {T} iterations, Y = {g['y'][0]:.9f}")
    dec = g["decisions"][0].astype(np.int64)
    assert int(g["cnt"].sum()) == T
    W = wide_oracle(p, seed)
    S = np.zeros(d, dtype=np.float64)
    samples = {0, 1, 2, 10, 100, 777, 1499}
    for t in range(T):
        if t in samples:
            w = np.zeros(d) if t == 0 else S * (2.0 / (t * (t + 1.0)))
            grad, bound = W.gradient(0, t, w, uroff=oracle.U32)
            a = int(dec[t])
            best = min(float(grad.min()), 0.0)
            chosen = 0.0 if a == 0 else float(grad[a - 1])
            assert chosen <= best + 2 * bound, (t, a, chosen, best, bound)
            own = int(np.argmin(grad)) + 1 if grad.min() < 0 else 0
            second = np.partition(np.append(grad, 0.0), 1)[1]
            if second - best > 2 * bound:
                assert a == own, (t, a, own)
            say(f"[wide] t={t}: vertex {a}, oracle {own}, margin {second - best:.3e}, bound {bound:.3e}")
        if dec[t] > 0:
            S[dec[t] - 1] += t + 1
    assert np.array_equal(g["wsum"][0].astype(np.float64), S)
    wT = S * (2.0 / (T * (T + 1.0)))
    assert close(g["y"][0], W.objective(wT), 1e-11, 1e-14)
    assert close(g["f_ckpt"][-1, 0], g["y"][0], 1e-15, 0.0)


@pytest.mark.parametrize("case", [
    dict(d=64, N=10, M=1, T=120, R=2, sched="grow"),        # N_k = 2 + k / 4: 2 .. 31
    dict(d=500, N=25, M=3, T=150, R=2, sched="geom"),       # N_k = ceil(4 * 1.1^k) capped at 300, M = 3
    dict(d=1000, N=25, M=1, T=80, R=1, sched="same"),       # a constant schedule equal to N
])
def test_wide_sample_size_schedule(ctx, case):
    """Algorithm 1 with per-epoch sample sizes N_k (the adaptive N_k its resampling step allows): the
    same replay protocol against the oracle run with the same schedule; a constant schedule equal to
    N reproduces the plain run bit for bit."""
    d, N, M, T, R = case["d"], case["N"], case["M"], case["T"], case["R"]
    E = (T + M - 1) // M
    if case["sched"] == "grow":
        sch = [2 + k // 4 for k in range(E)]
    elif case["sched"] == "geom":
        sch = [min(300, int(np.ceil(4 * 1.1 ** k))) for k in range(E)]
    else:
        sch = [N] * E
    base = problem(d, N, M=M, seed=5, ckpt=(T // 2, T))
    p = sim.Problem(**{**base.__dict__, "n_schedule": tuple(sch)})
    st, g = run_and_compare(ctx, p, R, T, 17)
    if case["sched"] == "same":
        ctx.run_wide(base, R, T, 17)
        plain = ctx.wide_paths()
        assert np.array_equal(plain["decisions"], g["decisions"]) and np.array_equal(plain["y"], g["y"])
