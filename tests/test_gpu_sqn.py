"""Algorithms 3-4, stochastic quasi-Newton classification (sim_run_sqn), vs the CPU oracle through the
C ABI (needs an MI355X).

There are no discrete decisions besides the sampled rows, which both sides draw from the same Philox
counters (bit-exact). The iterates differ only by rounding: the device sums dot products in a tree,
and applies H_t through the compact representation instead of Algorithm 4's explicit chain (the
oracle's pins show the two are the same matrix). Tolerances, in FP64: w^{K+1} and the checkpoint
iterates to 1e-9 relative in the 2-norm, F to 1e-10 relative; the loss kernel alone (F at the
device's own iterate) to 1e-12. Pair counts exact. At Section 4.1's largest shape (n = 5000,
N = 30 n, b_H = 600, K = 2000) the oracle checks the first iterations exactly that way and the full
run through properties: the loss at every checkpoint recomputed by the oracle at the device's iterate,
a decreasing loss, the pair count.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import sim, workloads

pytestmark = pytest.mark.gpu

W_RTOL = 1e-9
F_RTOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    s = sim.Sim(0)
    yield s
    s.close()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_and_compare(ctx, X, z, R, K, seed, L=10, M=25, b=50, bH=300, beta=2.0, ckpt=(), instance=0, load=True,
                    pairs_fp32=False, split=False):
    N, n = X.shape
    say(f"[sqn] n={n} N={N} R={R} K={K} L={L} M={M} b={b} bH={bH} seed={seed} ckpt={ckpt} fp32 pairs={pairs_fp32}"
        f"{' split' if split else ''}")
    if load:
        ctx.sqn_load(X, z)
    ctx.run_sqn(R, K, seed, L=L, M=M, b=b, bH=bH, beta=beta, checkpoints=ckpt, instance_id=instance,
                pairs_fp32=pairs_fp32, split=split)
    st = ctx.sqn_stats()
    g = ctx.sqn_paths()
    assert np.all(g["w_pad"] == 0.0)
    O = oracle.SqnOracle(X, z, L=L, M=M, b=b, bH=bH, beta=beta, seed=seed, instance=instance, ckpt=ckpt,
                         pairs_fp32=pairs_fp32)
    # binary32 pairs: both sides round at the same points, but a value within 1e-15 of a binary32
    # rounding boundary may round differently on the two sides (one ulp, 6e-8 of one entry)
    w_rtol, f_rtol = (1e-7, 1e-9) if pairs_fp32 else (W_RTOL, F_RTOL)
    Fs, worst_w, worst_f = [], 0.0, 0.0
    for r in range(R):
        o = O.run(r, K)
        assert int(g["pairs"][r]) == o["pairs"]
        ew = rel(g["w"][r], o["w"])
        ef = abs(g["F"][r] - o["F"]) / o["F"]
        worst_w, worst_f = max(worst_w, ew), max(worst_f, ef)
        assert ew <= w_rtol, (r, ew)
        assert ef <= f_rtol, (r, g["F"][r], o["F"])
        assert abs(g["F"][r] - O.loss(g["w"][r])) <= 1e-12 * o["F"]
        for c in range(len(ckpt)):
            assert abs(g["F_ckpt"][c, r] - o["F_ckpt"][c]) <= f_rtol * o["F_ckpt"][c]
            assert abs(g["F_ckpt"][c, r] - O.loss(g["w_ckpt"][c, r])) <= 1e-12 * o["F_ckpt"][c]
        Fs.append(o["F"])
    Fs = np.array(Fs)
    assert abs(st.mean - Fs.mean()) <= 1e-10 * Fs.mean()
    if R > 1:
        assert abs(st.var - Fs.var(ddof=1)) <= 1e-6 * Fs.var(ddof=1) + 1e-20
    assert st.min == g["F"].min() and st.max == g["F"].max()
    assert st.T == K and st.R == R
    say(f"[sqn] ok: max rel err w {worst_w:.2e}, F {worst_f:.2e}; {st.kernel_ms:.2f} ms")
    return st, g


@pytest.mark.parametrize("case", [
    dict(n=50, R=3, K=200, ckpt=(50, 100, 200)),                              # 19 pairs, ring not full
    dict(n=50, R=2, K=400, M=5, ckpt=(400,)),                                 # the ring wraps 34 times
    dict(n=37, N=1110, R=2, K=120, L=5, M=4, b=17, bH=33, ckpt=(7, 60)),      # ragged quads and chunks
    dict(n=24, N=700, R=2, K=60, L=1, M=1, b=9, bH=5),                        # a pair every iteration
    dict(n=1000, N=30000, R=2, K=60, M=3, bH=600, ckpt=(30,)),                # 256 threads
    dict(n=4100, N=5000, R=1, K=40, M=3, ckpt=(25,)),                         # two quads per thread
])
def test_sqn_against_oracle(ctx, case):
    c = dict(case)
    n = c.pop("n")
    X, z = workloads.sqn_dataset(11, n, c.pop("N", None))
    run_and_compare(ctx, X, z, c.pop("R"), c.pop("K"), 21, **c)


@pytest.mark.parametrize("case", [
    dict(n=9, N=1, R=2, K=40, L=4, M=3, b=3, bH=2),            # one row: every sample is that row
    dict(n=16, N=200, R=2, K=1),                                # a single gradient step
    dict(n=16, N=200, R=2, K=25, L=30),                         # no window closes: plain SGD, no pair
    dict(n=20, N=600, R=1, K=400, L=2, M=32, b=1024, bH=1024),  # largest M, b and b_H
    dict(n=8192, N=300, R=1, K=25, L=5, M=3, b=40, bH=60),      # largest n: two quads in every thread
])
def test_sqn_edge_cases(ctx, case):
    c = dict(case)
    n = c.pop("n")
    X, z = workloads.sqn_dataset(30, n, c.pop("N"))
    st, g = run_and_compare(ctx, X, z, c.pop("R"), c.pop("K"), 2, **c)
    if case.get("L", 10) * 2 >= case["K"]:
        assert np.all(g["pairs"] <= 1)


@pytest.mark.parametrize("split", [False, True], ids=["one_workgroup", "split"])
def test_sqn_single_feature(ctx, split):
    """One feature: a window whose Hessian rows all have x = 0 gives y = 0, so gamma = s'y / y'y is
    0/0 and the method (which uses every pair as formed) breaks down; the device must break down in
    the same replication as the oracle, with the same pair count, and agree where it does not (on
    both paths)."""
    X, z = workloads.sqn_dataset(30, 1, 40)
    ctx.sqn_load(X, z)
    O = oracle.SqnOracle(X, z, L=3, M=2, b=5, bH=7, seed=2)
    ctx.run_sqn(2, 50, 2, L=3, M=2, b=5, bH=7, split=split)
    g = ctx.sqn_paths()
    for r in range(2):
        o = O.run(r, 50)
        assert int(g["pairs"][r]) == o["pairs"]
        if np.isnan(o["F"]):
            assert np.isnan(g["F"][r])
        else:
            assert rel(g["w"][r], o["w"]) <= W_RTOL


@pytest.mark.parametrize("case", [
    dict(n=50, R=2, K=400, M=5, ckpt=(200, 400)),
    dict(n=37, N=1110, R=2, K=120, L=5, M=4, b=17, bH=33),
    dict(n=1000, N=30000, R=2, K=60, M=3, bH=600, ckpt=(30,)),
    dict(n=4100, N=5000, R=1, K=40, M=3),
])
def test_sqn_binary32_pairs(ctx, case):
    """The pairs kept in binary32 (pairs_fp32): against the oracle run with the same rounding points;
    against the binary64 method (the oracle with its pairs in binary64), which rounding the pairs
    perturbs by at most 1e-5 of the iterate and 1e-6 of the loss on these runs (the oracle's own
    two modes differ by up to 3.6e-6 and 3.4e-7 here); Algorithm 4's matrix from the float pairs
    against the oracle's chain over the same pairs."""
    c = dict(case)
    n = c.pop("n")
    X, z = workloads.sqn_dataset(18, n, c.pop("N", None))
    R, K = c.pop("R"), c.pop("K")
    st, g = run_and_compare(ctx, X, z, R, K, 23, pairs_fp32=True, **c)
    kw = dict(L=c.get("L", 10), M=c.get("M", 25), b=c.get("b", 50), bH=c.get("bH", 300), seed=23,
              ckpt=c.get("ckpt", ()))
    O64 = oracle.SqnOracle(X, z, **kw)
    for r in range(R):
        o = O64.run(r, K)
        assert int(g["pairs"][r]) == o["pairs"]
        assert rel(g["w"][r], o["w"]) <= 1e-5, (r, rel(g["w"][r], o["w"]))
        assert abs(g["F"][r] - o["F"]) <= 1e-6 * o["F"], (r, g["F"][r], o["F"])
    S, Y = g["S"][0], g["Y"][0]
    assert np.array_equal(S, S.astype(np.float32).astype(np.float64))
    h = ctx.sqn_hessian(0)
    ref = oracle.SqnOracle.hessian_approx(S, Y)
    assert np.linalg.norm(h["H"] - ref) <= 1e-10 * np.linalg.norm(ref)


def test_sqn_many_replications(ctx):
    """140 stored iterates (70 replications, one checkpoint) take the loss kernel with a lane per
    iterate: every F against the oracle's loss at the device's iterate, three replications against the
    oracle's run, the statistics against those F."""
    X, z = workloads.sqn_dataset(16, 52)
    R, K = 70, 60
    say(f"[sqn] many replications R={R}")
    ctx.sqn_load(X, z)
    ctx.run_sqn(R, K, 9, M=4, checkpoints=(30,))
    st = ctx.sqn_stats()
    g = ctx.sqn_paths()
    O = oracle.SqnOracle(X, z, M=4, seed=9, ckpt=(30,))
    for r in range(R):
        f = O.loss(g["w"][r])
        assert abs(g["F"][r] - f) <= 1e-12 * f, (r, g["F"][r], f)
        fc = O.loss(g["w_ckpt"][0, r])
        assert abs(g["F_ckpt"][0, r] - fc) <= 1e-12 * fc
    for r in (0, 33, R - 1):
        o = O.run(r, K)
        assert rel(g["w"][r], o["w"]) <= W_RTOL and abs(g["F"][r] - o["F"]) <= F_RTOL * o["F"]
    assert abs(st.mean - g["F"].mean()) <= 1e-13 * g["F"].mean()
    assert abs(st.f_mean[0] - g["F_ckpt"][0].mean()) <= 1e-13 * g["F_ckpt"][0].mean()


@pytest.mark.parametrize("n,M,K", [(37, 4, 120), (300, 25, 200), (1000, 7, 150), (4100, 3, 60), (700, 32, 360)])
def test_sqn_explicit_hessian(ctx, n, M, K):
    """Algorithm 4's matrix formed on the device (sim_sqn_hessian) from the pairs each replication
    holds, against the oracle's explicit chain of BFGS updates over the same pairs (read back from
    the device's ring, oldest first): Frobenius-relative 1e-10, gamma of the newest pair, the secant
    equation H y_t = s_t, symmetry. M = 32 with 35 pairs computed fills the ring: the product kernel's
    largest operand blocks (k = 64)."""
    X, z = workloads.sqn_dataset(17, n, min(30 * n, 6000))
    say(f"[sqn] explicit H n={n} M={M} K={K}")
    ctx.sqn_load(X, z)
    ctx.run_sqn(2, K, 3, M=M)
    g = ctx.sqn_paths()
    for r in range(2):
        h = ctx.sqn_hessian(r)
        S, Y = g["S"][r], g["Y"][r]
        assert h["m"] == len(S) == min(int(g["pairs"][r]), M) and h["n"] == n
        ref = oracle.SqnOracle.hessian_approx(S, Y)
        err = np.linalg.norm(h["H"] - ref) / np.linalg.norm(ref)
        say(f"[sqn] rep {r}: m={h['m']} rel err {err:.2e}, {h['device_ms']:.3f} ms")
        assert err <= 1e-10
        gam = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
        assert abs(h["gamma"] - gam) <= 1e-12 * abs(gam)
        assert np.linalg.norm(h["H"] @ Y[-1] - S[-1]) <= 1e-8 * np.linalg.norm(S[-1])
        assert np.allclose(h["H"], h["H"].T, rtol=0, atol=1e-12 * np.abs(h["H"]).max())
    with pytest.raises(sim.SimError):
        ctx.sqn_hessian(2)
    ctx.run_sqn(1, 15, 3, M=M)                     # k = 15 < 2L: no pair yet
    with pytest.raises(sim.SimError):
        ctx.sqn_hessian(0)


def test_sqn_instance_and_seed_streams(ctx):
    X, z = workloads.sqn_dataset(12, 40)
    run_and_compare(ctx, X, z, 2, 90, 0x1234_5678_9ABC, M=6, ckpt=(45,), instance=77)


def test_sqn_deterministic_and_reload(ctx):
    X, z = workloads.sqn_dataset(13, 64)
    ctx.sqn_load(X, z)
    ctx.run_sqn(3, 150, 5, checkpoints=(100,))
    a = ctx.sqn_paths()
    ctx.run_sqn(3, 150, 5, checkpoints=(100,))
    b = ctx.sqn_paths()
    assert np.array_equal(a["w"], b["w"]) and np.array_equal(a["F"], b["F"])
    # another data set replaces the first one; the first one again gives the first results
    X2, z2 = workloads.sqn_dataset(14, 30)
    ctx.sqn_load(X2, z2)
    ctx.run_sqn(1, 20, 5)
    assert ctx.sqn_paths()["w"].shape == (1, 30)
    ctx.sqn_load(X, z)
    ctx.run_sqn(3, 150, 5, checkpoints=(100,))
    assert np.array_equal(ctx.sqn_paths()["w"], a["w"])


def test_sqn_rejects_bad_data(ctx):
    X, z = workloads.sqn_dataset(15, 8)
    bad = X.copy()
    bad[3, 2] = 2
    with pytest.raises(sim.SimError):
        ctx.sqn_load(bad, z)
    zb = z.copy()
    zb[0] = 7
    with pytest.raises(sim.SimError):
        ctx.sqn_load(X, zb)


def test_paper_shape_sampled(ctx):
    """Section 4.1's largest Task 3 run: n = 5000, N = 30 n, b = 50, b_H = 600, M = 25, L = 10, beta = 2,
    K = 2000. The first 35 iterations (three pairs) against the oracle; the full run through the loss
    at every checkpoint recomputed by the oracle at the device's iterate, its decrease and the pair
    count."""
    n = 5000
    X, z = workloads.sqn_dataset(0, n)
    say(f"[sqn] paper shape n={n} N={X.shape[0]}")
    ctx.sqn_load(X, z)
    run_and_compare(ctx, X, z, 1, 35, 0, bH=600, ckpt=(20,), load=False)
    ck = (50, 100, 500, 1000, 2000)
    ctx.run_sqn(1, 2000, 0, bH=600, checkpoints=ck)
    st = ctx.sqn_stats()
    g = ctx.sqn_paths()
    say(f"[sqn] paper shape: {st.kernel_ms:.1f} ms for 2000 iterations, F = {g['F'][0]:.6f}")
    assert int(g["pairs"][0]) == 199
    O = oracle.SqnOracle(X, z)
    for c, k in enumerate(ck):
        f = O.loss(g["w_ckpt"][c, 0])
        assert abs(g["F_ckpt"][c, 0] - f) <= 1e-12 * f, (k, g["F_ckpt"][c, 0], f)
    assert g["F_ckpt"][-1, 0] == g["F"][0]
    assert np.all(np.diff(g["F_ckpt"][1:, 0]) < 0) and g["F"][0] < np.log(2.0)
    h = ctx.sqn_hessian(0, copy=False)
    say(f"[sqn] paper shape: H_t with m={h['m']} pairs formed in {h['device_ms']:.3f} ms")
    assert h["m"] == 25


# ---- the split path (sim_run_sqn_split): each replication over many one-wavefront workgroups ----

SPLIT_CASES = [
    dict(n=50, R=3, K=200, ckpt=(50, 100, 200)),                              # one slice, ring not full
    dict(n=50, R=2, K=400, M=5, ckpt=(400,)),                                 # the ring wraps
    dict(n=37, N=1110, R=2, K=120, L=5, M=4, b=17, bH=33, ckpt=(7, 60)),      # ragged quads
    dict(n=24, N=700, R=2, K=60, L=1, M=1, b=9, bH=5),                        # a pair every iteration
    dict(n=1000, N=30000, R=2, K=60, M=3, bH=600, ckpt=(30,)),                # four slices, the last ragged
    dict(n=4100, N=5000, R=1, K=40, M=3, ckpt=(25,)),                         # 17 slices
    dict(n=9, N=1, R=2, K=40, L=4, M=3, b=3, bH=2),                           # one row
    dict(n=16, N=200, R=2, K=1),                                              # a single gradient step
    dict(n=20, N=600, R=1, K=400, L=2, M=32, b=1024, bH=1024),                # largest M, b and b_H
    dict(n=8192, N=300, R=1, K=25, L=5, M=3, b=40, bH=60),                    # largest n: 32 slices
    dict(n=1000, N=30000, R=2, K=60, M=3, bH=600, ckpt=(30,), pairs_fp32=True),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[f"n{c['n']}_R{c['R']}_K{c['K']}" + ("_f32" if c.get("pairs_fp32")
                                                                                    else "") for c in SPLIT_CASES])
def test_sqn_split_against_oracle(ctx, case):
    c = dict(case)
    n = c.pop("n")
    X, z = workloads.sqn_dataset(11, n, c.pop("N", None))
    run_and_compare(ctx, X, z, c.pop("R"), c.pop("K"), 21, split=True, **c)


def test_sqn_split_matches_one_workgroup(ctx):
    """Both paths on the same data and seed: the same pair counts, iterates within 1e-11 (they differ
    only in the order of the dot products' sums), and the split run's pairs give Algorithm 4's
    matrix like the oracle's chain."""
    X, z = workloads.sqn_dataset(19, 700, 21000)
    ctx.sqn_load(X, z)
    kw = dict(M=6, bH=400, checkpoints=(90,))
    ctx.run_sqn(2, 180, 4, **kw)
    a = ctx.sqn_paths()
    ctx.run_sqn(2, 180, 4, split=True, **kw)
    b = ctx.sqn_paths()
    assert np.array_equal(a["pairs"], b["pairs"])
    for r in range(2):
        assert rel(b["w"][r], a["w"][r]) <= 1e-11, (r, rel(b["w"][r], a["w"][r]))
        assert abs(b["F"][r] - a["F"][r]) <= 1e-12 * a["F"][r]
    assert np.all(b["w_pad"] == 0.0)
    h = ctx.sqn_hessian(1)
    ref = oracle.SqnOracle.hessian_approx(b["S"][1], b["Y"][1])
    assert np.linalg.norm(h["H"] - ref) <= 1e-10 * np.linalg.norm(ref)


def test_sqn_split_rejects(ctx):
    X, z = workloads.sqn_dataset(20, 40)
    ctx.sqn_load(X, z)
    with pytest.raises(sim.SimError) as e:
        ctx.run_sqn(sim.SQN_SPLIT_MAX_R + 1, 10, 1, split=True)
    assert e.value.code == -1
    with pytest.raises(sim.SimError):
        ctx.run_sqn(1, 10, 1, split=True, L=0)


def test_paper_shape_split(ctx):
    """Section 4.1's largest Task 3 run on the split path: the first 35 iterations against the oracle;
    the full K = 2000 run through the loss at every checkpoint recomputed by the oracle at the
    device's iterate, its decrease, the pair count, and the final loss against the one-workgroup
    path's (1e-8: the two sum in different orders over 2000 iterations)."""
    n = 5000
    X, z = workloads.sqn_dataset(0, n)
    say(f"[sqn] paper shape split n={n} N={X.shape[0]}")
    ctx.sqn_load(X, z)
    run_and_compare(ctx, X, z, 1, 35, 0, bH=600, ckpt=(20,), load=False, split=True)
    ck = (50, 100, 500, 1000, 2000)
    ctx.run_sqn(1, 2000, 0, bH=600, checkpoints=ck, split=True)
    st = ctx.sqn_stats()
    g = ctx.sqn_paths()
    say(f"[sqn] paper shape split: {st.kernel_ms:.1f} ms for 2000 iterations, F = {g['F'][0]:.6f}")
    assert int(g["pairs"][0]) == 199
    O = oracle.SqnOracle(X, z)
    for c, k in enumerate(ck):
        f = O.loss(g["w_ckpt"][c, 0])
        assert abs(g["F_ckpt"][c, 0] - f) <= 1e-12 * f, (k, g["F_ckpt"][c, 0], f)
    assert np.all(np.diff(g["F_ckpt"][1:, 0]) < 0) and g["F"][0] < np.log(2.0)
    ctx.run_sqn(1, 2000, 0, bH=600, checkpoints=ck)
    one = ctx.sqn_paths()
    say(f"[sqn] paper shape: split vs one workgroup, w rel {rel(g['w'][0], one['w'][0]):.2e}, "
        f"F rel {abs(g['F'][0] - one['F'][0]) / one['F'][0]:.2e}")
    assert abs(g["F"][0] - one["F"][0]) <= 1e-8 * one["F"][0]
