"""Batched runs of uneven instances vs the CPU oracle (Algorithm 1, Section 3.1, over instances
of uneven horizon and size)."""
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


def make(i, d, N, noise=sim.NOISE_GAUSS, nu=3, ckpt=(), w0=None, log=None):
    mu, sigma = workloads.diag_instance(77, i, d)
    return sim.Problem(mu=mu, sigma=sigma, N=N, noise=noise, nu=nu, checkpoints=ckpt, gap_eps=0.05,
                       w0=w0, instance_id=i, log_reps=log)


SMALL = [  # (d, N, T, R, P, noise)
    (2, 2, 300, 130, 1, 0),
    (3, 5, 200, 70, 2, 0),
    (5, 7, 150, 100, 4, 0),
    (8, 4, 120, 64, 8, 0),
    (13, 9, 100, 40, 16, 0),
    (20, 11, 80, 33, 64, 0),
    (32, 6, 60, 65, 8, 0),
    (4, 6, 100, 50, 4, 1),
    (17, 5, 60, 30, 4, 1),
    (7, 3, 150, 90, 0, 0),     # 0: the cost model chooses
]


def test_small_batch_parity(ctx):
    probs, R, T, P = [], [], [], []
    for i, (d, N, t, r, p, noise) in enumerate(SMALL):
        w0 = np.full(d, 0.5 / d) if i == 2 else None
        probs.append(make(i, d, N, noise=noise, nu=4 if noise else 3, ckpt=(10, t), w0=w0, log=(0, r)))
        R.append(r)
        T.append(t)
        P.append(p)
    say(f"[batch] small batch {len(probs)} instances")
    ctx.run_batch(probs, R, T, seed=99, lanes_per_rep=P, keep_paths=True)
    for i, p in enumerate(probs):
        st = ctx.batch_stats(i)
        g = ctx.batch_paths(i)
        if P[i]:
            assert g["lanes_per_rep"] == P[i]
        op = parity.oracle_problem(p, 99)
        outs = (oracle.PathOut * R[i])()
        for r in range(R[i]):
            outs[r] = parity.check_rep(op, g, r, T[i], oracle.U32, decisions=g["decisions"][:, r])
        parity.check_stats(st, op.reduce(outs, T[i]), len(p.checkpoints), len(p.mu), g["tau"])
        say(f"[batch] instance {i} d={len(p.mu)} P={g['lanes_per_rep']} ok")


def test_batch_equals_single_run_at_one_lane(ctx):
    """One lane per replication (d <= 8) runs the same arithmetic in the same order as sim_run:
    identical bits."""
    d, N, T, R = 8, 10, 400, 300
    p = make(3, d, N, ckpt=(100, 400))
    p.keep_paths = True
    ctx.run(p, R, T, 5)
    a = ctx.paths()
    sa = ctx.stats()
    other = make(4, 6, 3, ckpt=(50,))
    ctx.run_batch([other, p], [100, R], [200, T], seed=5, lanes_per_rep=[2, 1], keep_paths=True)
    b = ctx.batch_paths(1)
    sb = ctx.batch_stats(1)
    assert np.array_equal(a["y"], b["y"])
    assert np.array_equal(a["cnt"], b["cnt"]) and np.array_equal(a["wsum"], b["wsum"])
    assert np.array_equal(a["tau"], b["tau"]) and np.array_equal(a["f_ckpt"], b["f_ckpt"])
    assert sa.mean == sb.mean and sa.var == sb.var


def test_batch_composition_invariance(ctx):
    """An instance's paths do not depend on the other instances, their order or the tiling."""
    A = make(10, 12, 8, ckpt=(30,))
    Bp = make(11, 5, 20, ckpt=(30,))
    Cp = make(12, 30, 4, ckpt=(30,))
    ctx.run_batch([A, Bp, Cp], [200, 100, 150], [120, 300, 60], seed=7, lanes_per_rep=[4, 2, 8], keep_paths=True)
    ya = ctx.batch_paths(0)["y"].copy()
    sa = ctx.batch_stats(0)
    ctx.run_batch([Cp, A], [150, 200], [60, 120], seed=7, lanes_per_rep=[4, 4], keep_paths=True)
    yb = ctx.batch_paths(1)["y"]
    sb = ctx.batch_stats(1)
    assert np.array_equal(ya, yb)
    assert sa.mean == sb.mean and sa.var == sb.var and list(sa.decision_total) == list(sb.decision_total)


def test_batch_errors(ctx):
    p = make(0, 40, 4)
    with pytest.raises(sim.SimError) as e:
        ctx.run_batch([p], [10], [10], seed=1)
    assert e.value.code == -5
    q = make(0, 4, 4)
    q.precision = sim.FP64
    with pytest.raises(sim.SimError) as e:
        ctx.run_batch([q], [10], [10], seed=1)
    assert e.value.code == -5
    with pytest.raises(sim.SimError) as e:
        ctx.run_batch([make(0, 4, 4)], [10], [10], seed=1, lanes_per_rep=[3])
    assert e.value.code == -1


def test_batch_maximum_horizon(ctx):
    """T = 131071, the longest horizon the batched kernels hold (the signature's 33rd bit): a zero-noise
    instance whose one chosen asset reaches S = T (T+1)/2 > 2^32 (closed form), and a noisy one at 2 and
    4 lanes per replication against the oracle's replay."""
    T = 131_071
    mu, _ = workloads.diag_instance(5, 0, 2)
    z = sim.Problem(mu=mu, sigma=np.zeros(2), N=2, checkpoints=(T,), instance_id=0)
    noisy = make(1, 6, 3, ckpt=(1000, T), log=(0, 4))
    wide = make(2, 12, 2, ckpt=(T,), log=(0, 2))
    say(f"[batch] maximum horizon T={T}")
    ctx.run_batch([z, noisy, wide], [64, 16, 8], [T, T, T], seed=4, lanes_per_rep=[1, 2, 4], keep_paths=True)
    g = ctx.batch_paths(0)
    best = int(np.argmax(mu))
    assert np.all(g["cnt"][best + 1] == T) and np.all(g["wsum"][best] == T * (T + 1) // 2)
    assert T * (T + 1) // 2 > 2 ** 32
    assert np.allclose(g["y"], -mu[best], rtol=0, atol=1e-15)
    for i, (p, n_log) in enumerate([(noisy, 4), (wide, 2)], start=1):
        g = ctx.batch_paths(i)
        op = parity.oracle_problem(p, 4)
        for r in range(n_log):
            parity.check_rep(op, g, r, T, oracle.U32, decisions=g["decisions"][:, r])
        say(f"[batch] instance {i} (d={len(p.mu)}, P={g['lanes_per_rep']}) matches the oracle at T={T}")


def test_uneven_full_size(ctx):
    """The uneven workload at full size: 256 instances x 4,096 replications, T log-uniform on
    [100, 1e5]; replications of several instances are checked
    against the oracle with their decision logs, every instance by exact properties."""
    w = workloads.WORKLOADS["uneven"]
    batch = workloads.uneven_batch(w["seed"], w["n_instances"], w["R"], w["d_range"], w["n_range"], w["t_range"])
    costs = np.array([b.T * b.N * b.d for b in batch], dtype=float)
    order = np.argsort(costs)
    checked = [int(order[0]), int(order[40]), int(order[128]), int(order[200])]
    probs = []
    for b in batch:
        log = (b.R - 3, 3) if b.instance in checked else None
        probs.append(sim.Problem(mu=b.mu, sigma=b.sigma, N=b.N, checkpoints=(min(50, b.T), b.T),
                                 instance_id=b.instance, log_reps=log))
    steps = sum(b.R * b.T for b in batch)
    say(f"[batch] uneven: {len(batch)} instances, {steps:.3e} path-steps")
    ctx.run_batch(probs, [b.R for b in batch], [b.T for b in batch], seed=w["seed"], keep_paths=True)
    st0 = ctx.batch_stats(0)
    say(f"[batch] uneven: {st0.kernel_ms:.1f} ms, {st0.path_steps_per_s:.3e} path-steps/s")
    for i, b in enumerate(batch):
        st = ctx.batch_stats(i)
        g = ctx.batch_paths(i)
        assert np.all(g["cnt"].sum(axis=0) == b.T)
        assert math.isclose(st.mean, math.fsum(g["y"]) / b.R, rel_tol=1e-13)
        assert st.min == g["y"].min() and st.max == g["y"].max()
        assert np.all(g["y"] >= st.f_star - 1e-12)
        assert np.array_equal(g["f_ckpt"][-1], g["y"])
        if i in checked:
            op = parity.oracle_problem(probs[i], w["seed"])
            for k in range(3):
                parity.check_rep(op, g, b.R - 3 + k, b.T, oracle.U32, decisions=g["decisions"][:, k])
            say(f"[batch] instance {i} (d={b.d} N={b.N} T={b.T} P={g['lanes_per_rep']}) matches the oracle")


def test_tuner_measures_and_caches(ctx, tmp_path):
    """sim_tune_batch times every theta candidate on reduced horizons, returns the fastest, writes
    it to the cache, and a second call with the same instances reads the cache without running."""
    probs = [make(i, d, N) for i, (d, N) in enumerate([(3, 5), (12, 40), (30, 20), (7, 2)])]
    R, T = [512, 256, 256, 1024], [400, 3000, 2000, 200]
    cache = str(tmp_path / "tune.json")
    a = ctx.tune_batch(probs, R, T, seed=3, t_scale=4, cache=cache)
    say(f"[batch] tuner: theta {a['heavy_factor']} from {a['candidates']}")
    assert not a["from_cache"] and len(a["candidates"]) >= 4
    assert all(ms > 0 for _, ms in a["candidates"])
    assert a["heavy_factor"] == min(a["candidates"], key=lambda c: c[1])[0]
    b = ctx.tune_batch(probs, R, T, seed=3, t_scale=4, cache=cache)
    assert b["from_cache"] and b["heavy_factor"] == a["heavy_factor"] and b["key"] == a["key"]
    c = ctx.tune_batch(probs, R, [t + 1 for t in T], seed=3, t_scale=4, cache=cache)
    assert not c["from_cache"] and c["key"] != a["key"]
    # the tuned plan runs and matches the oracle on a logged replication of the heaviest instance
    p = make(1, 12, 40, ckpt=(100, 3000), log=(0, 2))
    probs[1] = p
    ctx.run_batch(probs, R, T, seed=3, heavy_factor=a["heavy_factor"], keep_paths=True)
    g = ctx.batch_paths(1)
    op = parity.oracle_problem(p, 3)
    for k in range(2):
        parity.check_rep(op, g, k, T[1], oracle.U32, decisions=g["decisions"][:, k])


def test_graph_launch_replays_match_eager(ctx):
    """SIM_BATCH_GRAPH: the captured launch, replayed several times with other eager work and
    synchronisations between the replays, gives the eager run's bits every time; a new seed
    travels in the descriptors of the same graph."""
    probs = [make(20 + i, d, N, ckpt=(20, t)) for i, (d, N, t) in enumerate([(4, 6, 150), (11, 9, 90), (25, 5, 60)])]
    R, T = [200, 130, 70], [150, 90, 60]

    def snap():
        out = []
        for i in range(len(probs)):
            st = ctx.batch_stats(i)
            g = ctx.batch_paths(i)
            out.append((st.mean, st.var, tuple(st.decision_total), g["y"].copy(), g["cnt"].copy()))
        return out

    def same(a, b):
        for x, y in zip(a, b):
            assert x[0] == y[0] and x[1] == y[1] and x[2] == y[2]
            assert np.array_equal(x[3], y[3]) and np.array_equal(x[4], y[4])

    ctx.run_batch(probs, R, T, seed=41, keep_paths=True)
    eager = snap()
    ctx.run_batch(probs, R, T, seed=42, keep_paths=True)
    eager42 = snap()
    other = make(30, 6, 4)
    for k in range(3):
        say(f"[batch] graph replay {k}")
        ctx.run_batch(probs, R, T, seed=41, keep_paths=True, graph=True)
        same(snap(), eager)
        ctx.run(other, 500, 80, 9 + k)         # eager work between replays
        ctx.stats()
    ctx.run_batch(probs, R, T, seed=42, keep_paths=True, graph=True)
    same(snap(), eager42)


WAVE = [  # (d, N, T, R, M): every instance at 64 lanes per replication, Gaussian noise
    (10, 10, 400, 40, 1),
    (2, 100, 200, 20, 2),      # N > 64
    (32, 65, 100, 12, 1),      # d = 32, N d + 3 = 2083 of the 2112 staged floats
    (7, 9, 300, 30, 3),        # Philox blocks span samples
]


def test_wave_kernel_parity(ctx):
    """The one-wavefront form (fw_wave_kernel), which the batch takes when every instance asks for 64
    lanes per replication with Gaussian noise and N d within the staging area, against the oracle
    under the replay protocol; then the paper-scale instance (d = N = 10) over its full horizon
    T = 1e4, as the control-variate leg's plain stage runs it."""
    probs, R, T = [], [], []
    for i, (d, N, t, r, M) in enumerate(WAVE):
        mu, sigma = workloads.diag_instance(78, i, d)
        w0 = np.full(d, 0.5 / d) if i == 3 else None
        probs.append(sim.Problem(mu=mu, sigma=sigma, N=N, M=M, checkpoints=(10, t), gap_eps=0.05, w0=w0,
                                 instance_id=20 + i, log_reps=(0, r)))
        R.append(r)
        T.append(t)
    say(f"[batch] wave form, {len(probs)} instances")
    ctx.run_batch(probs, R, T, seed=41, lanes_per_rep=[64] * len(probs), keep_paths=True)
    for i, p in enumerate(probs):
        st = ctx.batch_stats(i)
        g = ctx.batch_paths(i)
        assert g["lanes_per_rep"] == 64
        op = parity.oracle_problem(p, 41)
        outs = (oracle.PathOut * R[i])()
        for r in range(R[i]):
            outs[r] = parity.check_rep(op, g, r, T[i], oracle.U32, decisions=g["decisions"][:, r])
        parity.check_stats(st, op.reduce(outs, T[i]), len(p.checkpoints), len(p.mu), g["tau"])
        say(f"[batch] wave instance {i} d={len(p.mu)} N={p.N} ok")
    w = workloads.WORKLOADS["paper_scale"]
    mu, sigma = workloads.diag_instance(w["seed"], 0, w["d"])
    p = sim.Problem(mu=mu, sigma=sigma, N=w["N"], checkpoints=(5000, w["T"]), log_reps=(0, 8))
    ctx.run_batch([p], [8], [w["T"]], seed=3, lanes_per_rep=[64], keep_paths=True)
    st = ctx.batch_stats(0)
    g = ctx.batch_paths(0)
    op = parity.oracle_problem(p, 3)
    outs = (oracle.PathOut * 8)()
    for r in range(8):
        outs[r] = parity.check_rep(op, g, r, w["T"], oracle.U32, decisions=g["decisions"][:, r])
    parity.check_stats(st, op.reduce(outs, w["T"]), len(p.checkpoints), len(p.mu), g["tau"])
    say(f"[batch] wave form at the paper-scale instance, T = {w['T']}: ok ({st.kernel_ms:.1f} ms)")
