"""Dense correlated returns (R_i = mu + L y_i, L lower triangular, d = 32 or 64) on the matrix-core
path vs the CPU oracle through the C ABI (needs an MI355X).

Same protocol and tolerances as test_gpu_parity.py: decisions, counts and signatures bit-exact
outside the oracle's rounding bound (which follows the gradient through the noise coordinates,
so it covers the kernel's order of evaluation: v = L'w and g = L h on the matrix cores), Y and
f(w_c) to 1e-11 relative, statistics to 1e-10 / 1e-8.
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


def run_and_compare(ctx, p, R, T, seed):
    say(f"[dense] d={len(p.mu)} N={p.N} M={p.M} lam={p.lam} noise={p.noise} nu={p.nu} R={R} T={T} seed={seed}")
    p.keep_paths = True
    p.log_reps = (0, R)
    ctx.run(p, R, T, seed)
    st = ctx.stats()
    g = ctx.paths()
    P = parity.oracle_problem(p, seed)
    outs = (oracle.PathOut * R)()
    amb = 0
    for r in range(R):
        o = parity.check_rep(P, g, r, T, oracle.U32, decisions=g["decisions"][:, r])
        outs[r] = o
        amb += o.n_replayed
    parity.check_stats(st, P.reduce(outs, T), len(p.checkpoints), len(p.mu), g["tau"])
    assert int(g["cnt"].sum()) == R * T
    assert math.isnan(st.f_star)
    say(f"[dense] ok, replayed ambiguous decisions: {amb}")
    return st, g


@pytest.mark.parametrize("case", [
    dict(d=32, N=10, T=200, R=300, ckpt=(1, 50, 200)),
    dict(d=64, N=8, T=150, R=200, ckpt=(150,)),
    dict(d=64, N=12, T=120, R=130, noise=sim.NOISE_T, nu=3, ckpt=(60, 120)),
    dict(d=32, N=6, T=150, R=129, M=3, lam=1.0, w0=True, noise=sim.NOISE_T, nu=5, ckpt=(7, 150)),
    dict(d=64, N=2, T=100, R=1, ckpt=(100,)),
], ids=lambda c: f"d{c['d']}N{c['N']}R{c['R']}{'t' if c.get('noise') else 'g'}")
def test_dense_shapes(ctx, case):
    d = case["d"]
    mu, L = workloads.dense_instance(11, d, d)
    w0 = None
    if case.get("w0"):
        w0 = np.linspace(0.05, 0.2, d)
        w0 = w0 / w0.sum() * 0.9
    p = sim.Problem(mu=mu, chol=L, N=case["N"], M=case.get("M", 1), lam=case.get("lam", 0.5), w0=w0,
                    noise=case.get("noise", sim.NOISE_GAUSS), nu=case.get("nu", 3),
                    checkpoints=case["ckpt"], gap_eps=0.05, instance_id=100 + d)
    run_and_compare(ctx, p, case["R"], case["T"], seed=4321 + d)


def test_dense_zero_factor_is_exact(ctx):
    """L = 0: every sample equals mu, the gradient is -mu, and every step goes to the asset with
    the largest mean (lowest index among equal ones): f(w_T) = -max mu exactly."""
    d = 32
    mu = np.linspace(-0.2, 0.3, d)
    mu[20] = mu[25] = 0.5
    p = sim.Problem(mu=mu, chol=np.zeros((d, d)), N=4, checkpoints=(5,), keep_paths=True)
    ctx.run(p, 200, 64, 9)
    st = ctx.stats()
    g = ctx.paths()
    assert np.all(g["y"] == -0.5)
    assert np.all(g["cnt"][21] == 64)
    assert st.mean == -0.5 and st.var == 0.0


def test_dense_diagonal_factor_matches_diagonal_statistics(ctx):
    """A diagonal L run on the dense kernel and the same sigma on the diagonal kernel draw the same
    normals and solve the same problem; their Monte Carlo means agree far inside the CI."""
    d = 32
    mu, sigma = workloads.diag_instance(3, 7, d)
    R, T = 20000, 200
    a = sim.Problem(mu=mu, sigma=sigma, N=10, checkpoints=(T,))
    ctx.run(a, R, T, 5)
    sa = ctx.stats()
    b = sim.Problem(mu=mu, chol=np.diag(sigma), N=10, checkpoints=(T,))
    ctx.run(b, R, T, 5)
    sb = ctx.stats()
    say(f"[dense] diagonal: {sa.mean:.9f} vs {sb.mean:.9f}, ci {sa.ci95_halfwidth:.2e}")
    assert abs(sa.mean - sb.mean) <= 0.05 * sa.ci95_halfwidth
    assert sum(sa.decision_total) == sum(sb.decision_total) == R * T


def test_dense_errors(ctx):
    mu, L = workloads.dense_instance(0, 0, 32)
    with pytest.raises(sim.SimError) as e:
        ctx.run(sim.Problem(mu=mu, chol=L, N=4), 10, 70000, 1)
    assert e.value.code == -5
    with pytest.raises(sim.SimError) as e:
        ctx.run(sim.Problem(mu=mu, chol=L, N=4, precision=sim.FP64), 10, 10, 1)
    assert e.value.code == -5


def test_stress_reduced(ctx):
    """The stress workload (d=64 dense L, N=100, t(3) noise, T=1000) at R = 4096: logged
    replications at both ends are checked against the oracle, every one by exact properties."""
    w = workloads.WORKLOADS["stress"]
    mu, L = workloads.dense_instance(w["seed"], 0, w["d"], "unit")
    R, T = 4096, w["T"]
    p = sim.Problem(mu=mu, chol=L, N=w["N"], noise=sim.NOISE_T, nu=w["nu"], checkpoints=w["checkpoints"],
                    keep_paths=True, log_reps=(R - 130, 130))
    say(f"[dense] stress reduced R={R} T={T}")
    ctx.run(p, R, T, w["seed"])
    st = ctx.stats()
    g = ctx.paths()
    say(f"[dense] stress: {st.kernel_ms:.1f} ms, {st.path_steps_per_s:.3e} path-steps/s")
    assert np.all(g["cnt"].sum(axis=0) == T)
    assert np.array_equal(g["f_ckpt"][-1], g["y"])
    assert math.isclose(st.mean, math.fsum(g["y"]) / R, rel_tol=1e-13)
    P = parity.oracle_problem(p, w["seed"])
    for r in (R - 130, R - 129, R - 2, R - 1):
        parity.check_rep(P, g, r, T, oracle.U32, decisions=g["decisions"][:, r - (R - 130)])
        say(f"[dense] stress rep {r} matches the oracle")


@pytest.mark.timeout(600)
def test_stress_full_size(ctx):
    """The stress workload at full size (R = 1e7, one launch): the decisions of the last 40
    replications (the end of the last workgroup) are logged and replayed by the oracle for a few
    of them, with their checkpoint values; every replication by exact properties of the totals."""
    w = workloads.WORKLOADS["stress"]
    mu, L = workloads.dense_instance(w["seed"], 0, w["d"], "unit")
    R, T = w["R"], w["T"]
    p = sim.Problem(mu=mu, chol=L, N=w["N"], noise=sim.NOISE_T, nu=w["nu"], checkpoints=w["checkpoints"],
                    log_reps=(R - 40, 40))
    say(f"[dense] stress full size R={R} T={T}")
    ctx.run(p, R, T, w["seed"])
    st = ctx.stats()
    say(f"[dense] stress full: {st.kernel_ms:.1f} ms, {st.path_steps_per_s:.3e} path-steps/s")
    g = ctx.paths()
    assert st.R == R and sum(st.decision_total) == R * T
    y = g["f_ckpt"][-1]                      # the last checkpoint is T: Y of every replication
    assert math.isclose(st.mean, math.fsum(y) / R, rel_tol=1e-12)
    assert st.min == y.min() and st.max == y.max()
    P = parity.oracle_problem(p, w["seed"])
    for r in (R - 40, R - 25, R - 1):
        o = P.path(r, T, replay=g["decisions"][:, r - (R - 40)], uroff=oracle.U32)
        assert o.n_mismatch == 0, f"rep {r}: first mismatch at {o.first_mismatch}"
        for c in range(len(w["checkpoints"])):
            assert abs(g["f_ckpt"][c, r] - o.f_ckpt[c]) <= parity.Y_RTOL * abs(o.f_ckpt[c]) + parity.Y_ATOL
        say(f"[dense] stress rep {r} matches the oracle ({o.n_replayed} replayed)")
