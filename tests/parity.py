"""Comparison protocol between the HIP path and the CPU oracle (test infrastructure).

Decisions: every logged decision of the HIP path must equal the oracle's, except at steps where
the oracle's LMO margin lies within the rounding bound of the HIP arithmetic (unit roundoff
2^-24 for binary32, 2^-53 for binary64, times the accumulation depth); there the oracle adopts
the logged decision when it is a near-optimal vertex and carries on along that path. Counts and
signatures must then agree exactly, the hitting time must lie in the range the bound allows (and
equal the oracle's when that range is one step), and the FP64 outcomes must agree to 1e-11.
"""
from __future__ import annotations

import numpy as np

import oracle

Y_RTOL = 1e-11
Y_ATOL = 1e-13


def oracle_problem(p, seed):
    """The oracle's view of a sim.Problem."""
    chol = p.chol if p.chol is not None else np.diag(np.asarray(p.sigma, dtype=np.float64))
    return oracle.OracleProblem(p.mu, chol=chol, N=p.N, M=p.M, lam=p.lam, w0=p.w0, noise=p.noise,
                                nu=p.nu, seed=seed, instance=p.instance_id,
                                ckpt=p.checkpoints, gap_eps=p.gap_eps, cv_ref=p.cv_ref,
                                n_sched=p.n_schedule)


def uroff(p):
    from paper_2404_11631_amd import sim
    return oracle.U64 if p.precision == sim.FP64 else oracle.U32


def check_rep(P, gpu, r, T, u, decisions=None, require_unambiguous=False):
    """Compares replication r; returns the oracle's path record."""
    d = P.d
    o = P.path(r, T, replay=decisions, uroff=u)
    if decisions is None and require_unambiguous and o.n_ambiguous:
        return None
    assert o.n_mismatch == 0, f"rep {r}: {o.n_mismatch} unambiguous decision mismatches, first at {o.first_mismatch}"
    assert np.array_equal(gpu["cnt"][:, r].astype(np.uint64), np.array(o.cnt[: d + 1], dtype=np.uint64)), f"rep {r} cnt"
    assert np.array_equal(gpu["wsum"][:, r], np.array(o.wsum[:d], dtype=np.uint64)), f"rep {r} wsum"
    tg = int(gpu["tau"][r])
    lo, hi = o.tau_lo, o.tau_hi
    assert lo <= tg <= hi, f"rep {r}: tau {tg} outside [{lo}, {hi}] (oracle {o.tau})"
    if lo == hi:
        assert tg == o.tau, f"rep {r}: tau {tg} != {o.tau}"
    assert abs(gpu["y"][r] - o.y) <= Y_RTOL * abs(o.y) + Y_ATOL, f"rep {r}: Y {gpu['y'][r]!r} vs {o.y!r}"
    for c in range(len(P.ckpt)):
        f = gpu["f_ckpt"][c, r]
        assert abs(f - o.f_ckpt[c]) <= Y_RTOL * abs(o.f_ckpt[c]) + Y_ATOL, f"rep {r} ckpt {c}"
    return o


def close(a, b, rtol, atol=0.0):
    return abs(a - b) <= rtol * max(abs(a), abs(b)) + atol


def check_stats(st, ost, n_ckpt, d, gpu_tau, rtol=1e-10):
    """GPU statistics vs the oracle's reduction of the same (replayed) paths; the hitting-time
    totals against the GPU's own per-path hitting times (checked per path by check_rep)."""
    assert st.R == ost.R
    assert close(st.mean, ost.mean, rtol, 1e-14), (st.mean, ost.mean)
    assert close(st.var, ost.var, 1e-8, 1e-20), (st.var, ost.var)
    assert close(st.ci95_halfwidth, ost.ci95, 1e-8, 1e-20)
    assert close(st.min, ost.ymin, rtol, 1e-14) and close(st.max, ost.ymax, rtol, 1e-14)
    for c in range(n_ckpt):
        assert close(st.f_mean[c], ost.f_mean[c], rtol, 1e-14)
        assert close(st.f_sd[c], ost.f_sd[c], 1e-7, 1e-12)
        assert st.rse_undefined[c] == ost.rse_undef[c]
        assert close(st.rse_mean[c], ost.rse_mean[c], 1e-8, 1e-13)
        assert close(st.rse_sd[c], ost.rse_sd[c], 1e-6, 1e-12)
    assert list(st.decision_total)[: d + 1] == list(ost.decision_total)[: d + 1]
    hit = gpu_tau != oracle.TAU_NONE
    assert st.tau_count == int(hit.sum())
    if hit.any():
        assert close(st.tau_mean, float(gpu_tau[hit].astype(np.float64).mean()), 1e-14)
