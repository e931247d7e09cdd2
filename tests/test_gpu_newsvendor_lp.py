"""Algorithm 2 over Eq. (7)'s general constraint set X = {A x <= C, x >= 0} (sim_run_newsvendor_lp,
M resource rows, the linear subproblem solved on the device) vs the oracle through the C ABI (needs
an MI355X).

Protocol (oracle.NvLpOracle): at every iteration the device's recorded vertex must be feasible. Its
value under the oracle's FP64 gradient must be within the bound of the LP optimum (HiGHS): the
gradient's binary32 uncertainty over the vertex and the optimiser, plus 1e-9 of the values. The
oracle then follows the device's vertex, so the iterates must be equal bit for bit. f(x_T) and
f(x_c) must match to 1e-11, tau must lie in the bound's range, and the statistics must match the
per-path values.
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


def run_and_compare(ctx, n, m, S, Mr, T, R, seed, x0=False, ckpt=()):
    inst = workloads.newsvendor_instance(5, 0, n)
    A, C = workloads.newsvendor_constraints(5, 0, n, m)
    x0v = np.full(n, 0.25 * float(np.min(C / A.sum(axis=1)))) if x0 else None
    say(f"[nvlp] n={n} M={m} S={S} resample={Mr} T={T} R={R} x0={x0}")
    ctx.run_newsvendor_lp(inst, A, C, R, T, seed, S=S, M=Mr, x0=x0v, checkpoints=ckpt)
    st = ctx.nv_lp_stats()
    g = ctx.nv_lp_paths()
    assert np.all(g["pivots"] <= sim.NV_LP_MAX_PIVOTS), "a subproblem was left unsolved"
    O = oracle.NvLpOracle(inst, A, C, S=S, M=Mr, x0=x0v, seed=seed, ckpt=ckpt)
    ys = []
    for r in range(R):
        o = O.path(r, T, replay=(g["basis"][r], g["value"][r]), uroff=oracle.U32)
        assert o["n_mismatch"] == 0, (r, o["first_mismatch"], o["worst_excess"])
        assert np.array_equal(g["x"][r], o["x"]), (r, float(np.abs(g["x"][r] - o["x"]).max()))
        assert g["y"][r] == pytest.approx(o["y"], rel=1e-11)
        for c in range(len(ckpt)):
            assert g["f_ckpt"][c, r] == pytest.approx(o["f_ckpt"][c], rel=1e-11)
        assert o["tau_lo"] <= int(g["tau"][r]) <= o["tau_hi"], (g["tau"][r], o["tau_lo"], o["tau_hi"])
        assert np.all(A @ g["x"][r] <= C * (1 + 1e-12)) and np.all(g["x"][r] >= 0)
        ys.append(o["y"])
    ys = np.array(ys)
    assert st.R == R and st.T == T
    assert st.mean == pytest.approx(ys.mean(), rel=1e-10)
    if R > 1:
        assert st.var == pytest.approx(ys.var(ddof=1), rel=1e-8, abs=1e-15 * ys.mean() ** 2)
    assert st.min == g["y"].min() and st.max == g["y"].max()
    say(f"[nvlp] ok: pivots per iteration mean {g['pivots'].mean():.2f} max {int(g['pivots'].max())}; "
        f"{st.kernel_ms:.2f} ms")
    return st, g


@pytest.mark.parametrize("case", [
    dict(n=8, m=2, S=25, Mr=1, T=200, R=3, ckpt=(50, 200)),
    dict(n=100, m=3, S=25, Mr=1, T=300, R=2, ckpt=(100, 300)),
    dict(n=1000, m=4, S=7, Mr=3, T=150, R=2, ckpt=(150,), x0=True),
    dict(n=4096, m=8, S=50, Mr=1, T=100, R=1, ckpt=(100,)),
    dict(n=64, m=1, S=25, Mr=2, T=200, R=2, ckpt=(200,)),
    dict(n=10_000, m=3, S=25, Mr=1, T=400, R=1, ckpt=(100, 400)),
])
def test_newsvendor_lp_against_oracle(ctx, case):
    c = dict(case)
    run_and_compare(ctx, c.pop("n"), c.pop("m"), c.pop("S"), c.pop("Mr"), c.pop("T"), c.pop("R"), 19,
                    x0=c.pop("x0", False), ckpt=c.pop("ckpt", ()))


def test_newsvendor_lp_one_row_matches_the_ratio_rule(ctx):
    """With A = c (one row) the device's vertex each iteration is the ratio rule's: the general path
    and sim_run_newsvendor take the same decisions where the latter's are unambiguous, and reach the
    same cost."""
    n, T, seed = 64, 200, 7
    inst = workloads.newsvendor_instance(8, 0, n)
    ctx.run_newsvendor(inst, 1, T, seed, S=25)
    single = ctx.nv_paths()
    ctx.run_newsvendor_lp(inst, inst["c"][None, :], [inst["C"]], 1, T, seed, S=25)
    g = ctx.nv_lp_paths()
    dec = np.zeros(T, dtype=np.int64)
    for t in range(T):
        prods = [int(b) for b, v in zip(g["basis"][0, t], g["value"][0, t]) if b < n and v > 0]
        dec[t] = prods[0] + 1 if prods else 0
    agree = float(np.mean(dec == single["decisions"][0]))
    say(f"[nvlp] one row: decisions agree on {agree:.3f} of the iterations")
    assert agree > 0.95
    assert g["y"][0] == pytest.approx(single["y"][0], rel=1e-3)


def test_newsvendor_lp_errors(ctx):
    n = 16
    inst = workloads.newsvendor_instance(1, 0, n)
    A, C = workloads.newsvendor_constraints(1, 0, n, 2)
    A0 = A.copy()
    A0[:, 3] = 0.0
    with pytest.raises(sim.SimError):
        ctx.run_newsvendor_lp(inst, A0, C, 1, 10, 0, S=5)     # a product using no resource
    with pytest.raises(sim.SimError):
        ctx.run_newsvendor_lp(inst, A, -C, 1, 10, 0, S=5)


def test_newsvendor_lp_lane_split_invariance(ctx):
    """The gradient launch splits each quad's S samples over P lanes (16 at R = 1 and 4 at R = 8 for
    1e4 products); the integer counts make replication 0's gradients, hence its bases, basic values,
    pivots and iterate, the same bits either way."""
    n, m = 10_000, 3
    inst = workloads.newsvendor_instance(7, 0, n)
    A, C = workloads.newsvendor_constraints(7, 0, n, m)
    ctx.run_newsvendor_lp(inst, A, C, 1, 60, 5, S=25, checkpoints=(60,))
    a = ctx.nv_lp_paths()
    ctx.run_newsvendor_lp(inst, A, C, 8, 60, 5, S=25, checkpoints=(60,))
    b = ctx.nv_lp_paths()
    assert np.array_equal(a["basis"][0], b["basis"][0]) and np.array_equal(a["value"][0], b["value"][0])
    assert np.array_equal(a["pivots"][0], b["pivots"][0]) and np.array_equal(a["x"][0], b["x"][0])
    assert a["y"][0] == b["y"][0]
