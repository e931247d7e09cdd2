"""HIP path vs the CPU oracle through the C ABI (needs an MI355X).

Tolerances (the decision protocol is in tests/parity.py):
  * decisions, decision counts, signatures: bit-exact outside the rounding bound of the kernel's
    arithmetic; hitting times inside the range that bound allows;
  * Y = f(w_T) and f(w_c): 1e-11 relative (both sides evaluate Eq. (3) in FP64 on the same
    signature; the oracle's recurrence drifts by at most ~T ulp);
  * statistics: 1e-10 relative on means, 1e-8 on variances (double-double sums on the GPU,
    Neumaier two-pass on the CPU) -- tighter than the required 1e-5.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import sim, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    s = sim.Sim(0)
    yield s
    s.close()


def run_and_compare(ctx, p, R, T, seed, check_all=True, stats=True):
    say(f"[parity] d={len(p.mu)} N={p.N} M={p.M} lam={p.lam} noise={p.noise} prec={p.precision} "
        f"R={R} T={T} seed={seed}")
    p.keep_paths = True
    p.log_reps = (0, R)
    ctx.run(p, R, T, seed)
    st = ctx.stats()
    g = ctx.paths()
    P = parity.oracle_problem(p, seed)
    u = parity.uroff(p)
    outs = (oracle.PathOut * R)()
    amb = 0
    for r in range(R):
        o = parity.check_rep(P, g, r, T, u, decisions=g["decisions"][:, r])
        outs[r] = o
        amb += o.n_replayed
    if stats:
        ost = P.reduce(outs, T)
        parity.check_stats(st, ost, len(p.checkpoints), len(p.mu), g["tau"])
    assert int(g["cnt"].sum()) == R * T
    return st, g, amb


def test_tiny_fp64_full(ctx):
    """The tiny workload in full: R=1000, T=100, d=2, N=2, FP64, parameters from seed 0."""
    w = workloads.WORKLOADS["tiny"]
    mu, sigma = workloads.diag_instance(w["seed"], 0, w["d"])
    p = sim.Problem(mu=mu, sigma=sigma, N=w["N"], precision=sim.FP64, checkpoints=w["checkpoints"])
    st, g, amb = run_and_compare(ctx, p, w["R"], w["T"], w["seed"])
    assert amb == 0                    # binary64: no decision within the rounding bound
    assert st.R == 1000 and st.T == 100


@pytest.mark.parametrize("case", [
    dict(d=10, N=10, T=600, R=700, precision=sim.FP32, ckpt=(50, 100, 500, 600)),
    dict(d=1, N=3, T=300, R=300, precision=sim.FP32, ckpt=(1, 300)),
    dict(d=3, N=5, M=3, T=200, R=300, precision=sim.FP64, w0=True, ckpt=(7, 100)),
    dict(d=5, N=7, T=200, R=300, precision=sim.FP32, lam=1.0, ckpt=(50,)),
    dict(d=7, N=4, T=200, R=300, precision=sim.FP32, ckpt=(100, 200)),
    dict(d=12, N=3, T=150, R=260, precision=sim.FP64, ckpt=(150,)),
    dict(d=16, N=3, T=150, R=300, precision=sim.FP32, ckpt=(10,)),
    dict(d=20, N=2, T=150, R=300, precision=sim.FP32, M=2, ckpt=()),
    dict(d=32, N=5, T=100, R=257, precision=sim.FP32, ckpt=(100,)),
    dict(d=6, N=8, T=150, R=300, precision=sim.FP32, noise=sim.NOISE_T, nu=3, ckpt=(50, 150)),
    dict(d=4, N=5, T=150, R=300, precision=sim.FP64, noise=sim.NOISE_T, nu=5, ckpt=(150,)),
    dict(d=24, N=4, T=100, R=200, precision=sim.FP32, noise=sim.NOISE_T, nu=4, ckpt=(100,)),
], ids=lambda c: f"d{c['d']}N{c['N']}{'t' if c.get('noise') else 'g'}{'64' if c['precision'] else '32'}")
def test_shapes(ctx, case):
    d = case["d"]
    mu, sigma = workloads.diag_instance(5, d, d)
    w0 = None
    if case.get("w0"):
        w0 = np.linspace(0.05, 0.2, d)
        w0 = w0 / w0.sum() * 0.9
    p = sim.Problem(mu=mu, sigma=sigma, N=case["N"], M=case.get("M", 1), lam=case.get("lam", 0.5),
                    w0=w0, noise=case.get("noise", sim.NOISE_GAUSS), nu=case.get("nu", 3),
                    precision=case["precision"], checkpoints=case["ckpt"], gap_eps=0.05,
                    instance_id=d)
    st, g, amb = run_and_compare(ctx, p, case["R"], case["T"], seed=1234 + d)
    say(f"[parity] replayed ambiguous decisions: {amb}")


def test_zero_noise_exact(ctx):
    mu = np.array([0.2, 0.9, 0.9, 0.1])
    p = sim.Problem(mu=mu, sigma=np.zeros(4), N=3, checkpoints=(10,), keep_paths=True)
    ctx.run(p, 300, 64, 7)
    st = ctx.stats()
    g = ctx.paths()
    assert np.all(g["y"] == -0.9)
    assert np.all(g["cnt"][2] == 64)
    assert st.mean == -0.9 and st.var == 0.0
    p = sim.Problem(mu=-mu, sigma=np.full(4, 1e-3), N=3, checkpoints=(10,), keep_paths=True)
    ctx.run(p, 300, 64, 7)
    st = ctx.stats()
    assert st.mean == 0.0 and st.decision_total[0] == 300 * 64 and st.rse_undefined[0] == 300


def test_single_path_single_step(ctx):
    mu, sigma = workloads.diag_instance(0, 0, 3)
    p = sim.Problem(mu=mu, sigma=sigma, N=2, checkpoints=(1,))
    run_and_compare(ctx, p, 1, 1, 11)


def test_wide_horizon(ctx):
    """T above 92681 switches the signature to 64 bits."""
    mu, sigma = workloads.diag_instance(0, 3, 2)
    p = sim.Problem(mu=mu, sigma=sigma, N=2, checkpoints=(92681, 100000))
    run_and_compare(ctx, p, 20, 100_000, 3)


def test_deterministic_and_seed_sensitive(ctx):
    mu, sigma = workloads.diag_instance(0, 1, 10)
    p = sim.Problem(mu=mu, sigma=sigma, N=10, checkpoints=(50,), keep_paths=True)
    ctx.run(p, 5000, 300, 42)
    a = ctx.stats()
    ya = ctx.paths()["y"]
    ctx.run(p, 5000, 300, 42)
    b = ctx.stats()
    yb = ctx.paths()["y"]
    assert np.array_equal(ya, yb)
    assert a.mean == b.mean and a.var == b.var and list(a.decision_total) == list(b.decision_total)
    ctx.run(p, 5000, 300, 43)
    c = ctx.stats()
    assert c.mean != a.mean
    # a replication's path does not depend on R
    ctx.run(p, 777, 300, 42)
    yc = ctx.paths()["y"]
    assert np.array_equal(yc, ya[:777])


def test_errors_on_device(ctx):
    with pytest.raises(sim.SimError) as e:
        ctx.run(sim.Problem(mu=np.zeros(3), sigma=np.ones(3), N=1), 10, 10, 0)
    assert e.value.code == -1
    fresh = sim.Sim(0)
    with pytest.raises(sim.SimError) as e:
        fresh.stats()
    assert e.value.code == -4
    fresh.close()


def test_paper_scale_full_size(ctx):
    """The paper-scale workload at full size (R=1e6, T=1e4, d=10, N=10, FP32) in the launch the
    benchmark times: replications of the first workgroup, a middle one and the ragged last one
    are checked against the oracle with their logged decisions, and exact properties are checked
    over all replications."""
    w = workloads.WORKLOADS["paper_scale"]
    R, T, seed = w["R"], w["T"], w["seed"]
    mu, sigma = workloads.diag_instance(seed, 0, w["d"])
    n_log = 32
    P = None
    replayed = 0
    for begin in (0, R // 2 - 7, R - n_log):
        p = sim.Problem(mu=mu, sigma=sigma, N=w["N"], checkpoints=w["checkpoints"], keep_paths=True,
                        log_reps=(begin, n_log))
        say(f"[parity] paper_scale R={R} T={T} logged [{begin}, {begin + n_log})")
        ctx.run(p, R, T, seed)
        st = ctx.stats()
        g = ctx.paths()
        say(f"[parity] kernel {st.kernel_ms:.1f} ms, {st.path_steps_per_s:.3e} path-steps/s")
        P = P or parity.oracle_problem(p, seed)
        for k in range(n_log):
            o = parity.check_rep(P, g, begin + k, T, oracle.U32, decisions=g["decisions"][:, k])
            replayed += o.n_replayed
    say(f"[parity] replayed ambiguous decisions over {3 * n_log} paths: {replayed}")
    # exact properties over all replications (the last run)
    Y = g["y"]
    assert np.all(g["cnt"].sum(axis=0) == T)
    assert math.isclose(st.mean, math.fsum(Y) / R, rel_tol=1e-14)
    m = math.fsum(Y) / R
    var = math.fsum((Y - m) ** 2) / (R - 1)
    assert math.isclose(st.var, var, rel_tol=1e-10)
    assert st.min == Y.min() and st.max == Y.max()
    assert list(st.decision_total)[: w["d"] + 1] == [int(x) for x in g["cnt"].sum(axis=1, dtype=np.uint64)]
    assert np.all(Y >= st.f_star - 1e-12)
    F = g["f_ckpt"]
    assert np.array_equal(F[-1], Y)                    # last checkpoint is T
    for c in range(len(w["checkpoints"])):
        assert math.isclose(st.f_mean[c], math.fsum(F[c]) / R, rel_tol=1e-13)
        ok = F[c] != 0
        rse = ((F[c][ok] - Y[ok]) / F[c][ok]) ** 2
        assert st.rse_undefined[c] == int((~ok).sum())
        if len(rse):
            assert math.isclose(st.rse_mean[c], math.fsum(rse) / len(rse), rel_tol=1e-12, abs_tol=1e-300)
    hit = g["tau"] != sim.TAU_NONE
    assert st.tau_count == int(hit.sum())


@pytest.mark.parametrize("kind,d,M,noise,precision", [
    ("growing", 10, 1, sim.NOISE_GAUSS, sim.FP32),
    ("geometric", 7, 2, sim.NOISE_GAUSS, sim.FP32),
    ("growing", 5, 1, sim.NOISE_T, sim.FP32),
    ("geometric", 12, 3, sim.NOISE_GAUSS, sim.FP64),
])
def test_sample_size_schedule_matches_oracle(ctx, kind, d, M, noise, precision):
    """Per-epoch sample sizes N_k (the remark on Algorithm 1's resampling step) on the per-lane
    kernel: every replication against the oracle with the same schedule."""
    T, R = 240, 300
    E = -(-T // M)
    sched = [2 + k // 2 for k in range(E)] if kind == "growing" else [min(200, int(3 * 1.06 ** k)) for k in range(E)]
    mu, sigma = workloads.diag_instance(31, d, d)
    p = sim.Problem(mu=mu, sigma=sigma, N=sched[0], M=M, noise=noise, nu=4, precision=precision,
                    checkpoints=(60, T), gap_eps=0.05, n_schedule=tuple(sched))
    st, g, amb = run_and_compare(ctx, p, R, T, 13)
    say(f"[parity] schedule {kind}: N from {sched[0]} to {sched[-1]}, replayed {amb}")


@pytest.mark.parametrize("d,noise", [(10, sim.NOISE_GAUSS), (3, sim.NOISE_GAUSS), (20, sim.NOISE_T)])
def test_constant_schedule_is_the_plain_run(ctx, d, noise):
    """A schedule with N in every epoch gives the plain run's bits (its kernel takes the per-epoch
    coefficients from the table, rounded as the plain run's are)."""
    T, R, N = 150, 500, 9
    mu, sigma = workloads.diag_instance(32, d, d)
    base = dict(mu=mu, sigma=sigma, N=N, noise=noise, nu=3, checkpoints=(50, T), keep_paths=True)
    ctx.run(sim.Problem(**base), R, T, 21)
    a, sa = ctx.paths(), ctx.stats()
    ctx.run(sim.Problem(**base, n_schedule=tuple([N] * T)), R, T, 21)
    b, sb = ctx.paths(), ctx.stats()
    for k in ("y", "cnt", "wsum", "tau", "f_ckpt"):
        assert np.array_equal(a[k], b[k]), k
    assert sa.mean == sb.mean and sa.var == sb.var
