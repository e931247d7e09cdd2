"""The context-level boundary calls that the plain run does not cover (needs an MI355X):
sim_run_into (results in caller device memory) against sim_run on the same inputs, bit for bit;
sim_create_ex's workspace cap (a run past it is refused before any launch and the context stays
usable); a run on parameters drawn by sim_param_gen against the oracle's replay."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import sim, workloads
from tests import parity
from tests.hipmem import Hip

pytestmark = pytest.mark.gpu

FIELDS = ("R", "T", "mean", "var", "ci95_halfwidth", "min", "max", "n_checkpoints", "tau_count", "tau_mean")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b, d, nc):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), f
    for c in range(nc):
        for f in ("f_mean", "f_sd", "rse_mean", "rse_sd", "rse_undefined"):
            assert getattr(a, f)[c] == getattr(b, f)[c], (f, c)
    assert list(a.decision_total)[: d + 1] == list(b.decision_total)[: d + 1]


@pytest.mark.parametrize("dense", [False, True])
def test_run_into_matches_run(dense):
    ctx = sim.Sim(0)
    hip = Hip()
    try:
        d, N, R, T, ck, seed = (32, 6, 20_000, 200, (20, 200), 5) if dense else (10, 10, 300_000, 250, (50, 250), 4)
        if dense:
            mu, L = workloads.dense_instance(seed, 0, d)
            p = sim.Problem(mu=mu, chol=L, N=N, checkpoints=ck, gap_eps=0.05, keep_paths=True)
        else:
            mu, sigma = workloads.diag_instance(seed, 0, d)
            p = sim.Problem(mu=mu, sigma=sigma, N=N, checkpoints=ck, gap_eps=0.05, keep_paths=True)
        say(f"[boundary] run_into dense={dense} d={d} N={N} R={R} T={T}")
        ctx.run(p, R, T, seed)
        ref = ctx.stats()
        ref_paths = ctx.paths()
        ref_f = ref_paths["f_ckpt"].copy()
        ref_y = ref_paths["y"].copy()
        nf = sim.noalloc_stats_fields(len(ck))
        fck = hip.alloc(8 * R * len(ck))
        sf = hip.alloc(8 * nf)
        si = hip.alloc(8 * (d + 3))
        ctx.run_into(p, R, T, seed, fck, sf, si)
        got = sim.stats_from_raw(p, R, T, hip.get(sf, np.float64, nf), hip.get(si, np.uint64, d + 3))
        _same(got, ref, d, len(ck))
        assert np.array_equal(hip.get(fck, np.float64, R * len(ck)).reshape(len(ck), R), ref_f)
        g = ctx.paths()                                 # the records stay in the context
        assert g.get("f_ckpt") is None and np.array_equal(g["y"], ref_y)
        with pytest.raises(sim.SimError) as e:
            ctx.stats()
        assert e.value.code == -4                       # SIM_ESTATE until the next sim_run
        ctx.run(p, 1000, T, seed)
        assert ctx.stats().R == 1000
    finally:
        hip.close()
        ctx.close()


def test_workspace_cap():
    d, N, T, seed = 10, 10, 50, 9
    mu, sigma = workloads.diag_instance(seed, 0, d)
    p = sim.Problem(mu=mu, sigma=sigma, N=N, checkpoints=(T,), keep_paths=True)
    cap = 4 << 20
    capped = sim.Sim(0, workspace_bytes=cap)
    free = sim.Sim(0)
    try:
        say("[boundary] workspace cap 4 MiB: R = 1e6 with per-path records is refused")
        with pytest.raises(sim.SimError) as e:
            capped.run(p, 1_000_000, T, seed)
        assert e.value.code == -2                       # SIM_ENOMEM, before any launch
        assert capped.workspace_bytes() <= cap
        capped.run(p, 20_000, T, seed)
        free.run(p, 20_000, T, seed)
        _same(capped.stats(), free.stats(), d, 1)
        assert capped.workspace_bytes() <= cap
    finally:
        capped.close()
        free.close()


def test_param_gen_instance_against_oracle():
    """A run on Section 4.1's parameter regime as sim_param_gen draws it, under the replay protocol."""
    d, N, R, T, seed = 16, 8, 64, 300, 21
    mu, sigma = sim.param_gen(d, sim.REGIME_PAPER, 1234)
    p = sim.Problem(mu=mu, sigma=sigma, N=N, checkpoints=(100, 300), keep_paths=True, log_reps=(0, R))
    ctx = sim.Sim(0)
    try:
        ctx.run(p, R, T, seed)
        st = ctx.stats()
        g = ctx.paths()
        op = parity.oracle_problem(p, seed)
        outs = (oracle.PathOut * R)()
        for r in range(R):
            outs[r] = parity.check_rep(op, g, r, T, oracle.U32, decisions=g["decisions"][:, r])
        parity.check_stats(st, op.reduce(outs, T), len(p.checkpoints), d, g["tau"])
    finally:
        ctx.close()
