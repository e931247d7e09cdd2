"""Throughput of the batched stochastic Frank-Wolfe simulation on one MI355X.

A step is one sim_run over the paper-scale workload (R = 1e6 replications of Algorithm 1,
T = 1e4 iterations, d = 10 assets, N = 10 samples per gradient, FP32 state, FP64 statistics),
fused with its cross-path reduction, followed by sim_stats; every step draws fresh noise (seed
+ step). Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--cpu-seconds 20] [--no-cpu-baseline]

The line also carries: each statistic's error against FP64 references ("stats"); the
control-variate leg ("cv", skip with --no-cv); the sweeps over the Section 4.1 shapes of Task 1
("paper_shape"), Task 2 ("newsvendor_shape"; over three resource rows, "newsvendor_lp_shape") and
Task 3 ("sqn_shape"), and Table 2's RSE
statistic over seven replications of each task ("table2"), all skipped with --no-paper-shape; the
uneven workload in one batched launch with its measured plan ("uneven", --no-uneven); the
dense-L t(3) stress workload at R = 1e7 ("stress", --no-stress); the oracle on every host core
("cpu_baseline") and on one thread per configuration, extrapolated to each full workload
("oracle_single_core"), both skipped with --no-cpu-baseline.

Other measurements (not the headline line):
    --workload stress [--reps R]   the dense-L, t(3) stress workload (d = 64, N = 100, T = 1e3)
    --workload paper_shape         Section 4.1's shape alone: one replication, d = 5e2 .. 1e5,
                                   K = 1500, on the wide path (--steps runs per size)
    --workload newsvendor_shape    Task 2 (Algorithm 2) at Section 4.1's shape: n = 1e2 .. 1e6
                                   products, K = 1500
    --workload newsvendor_lp_shape Task 2 over three resource rows (Eq. (7) in general): n = 1e2 .. 1e4
    --workload sqn_shape           Task 3 (Algorithms 3-4) at Section 4.1's settings: n = 50 .. 5000
                                   features, N = 30 n, K = 2000, b_H = 300 / 600
    --workload uneven              the 256 uneven instances on the plain path, instance by instance
                                   over four streams (the comparison without batching)
    --workload uneven_batch [--heavy-factor a,b,..] [--tune]
                                   the 256 uneven instances in one batched launch, per theta
    --copy-probe BYTES             one plain device-to-device copy of BYTES, for calibrating the
                                   FETCH_SIZE / WRITE_SIZE counters against known traffic
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "path-steps/sec and wall time to 95% CI half-width 1e-3, plain vs CV, 1 MI355X"

# ALU roofline. Algorithmic 32-bit VALU lane-operations per standard normal:
# Philox4x32-10 (10 rounds x (2 wide products + 4 xors) per 4 normals) = 15, uniform map = 2,
# Box-Muller (log2, sqrt, sin, cos, 2 products per pair) = 3, one-pass sample statistics
# (dot FMA, sum, FMA) = 3; per iteration ~15 d more for gradient, linear subproblem and update.
OPS_PER_NORMAL = 15 + 2 + 3 + 3
OPS_PER_ASSET_STEP = 15
# 256 CUs x 2.4 GHz x 128 lane-ops/clock: the FP32 vector rate 157.3 TFLOP/s at 2 flops per FMA
PEAK_OPS = 256 * 2.4e9 * 128
# HBM3E bandwidth of one MI355X, bytes/s
PEAK_HBM = 8.0e12
# dense FP64 matrix-core rate of one MI355X, flop/s
PEAK_F64 = 78.6e12
# dense FP32 matrix-core rate of one MI355X, flop/s
PEAK_F32_MFMA = 157.3e12


def ops_per_path_step(d: int, N: int) -> float:
    return OPS_PER_NORMAL * N * d + OPS_PER_ASSET_STEP * d


def ops_per_path_step_dense(d: int, N: int, nu: int) -> float:
    """Dense L with t noise: N (d + nu) normals (the chi-square normals need one FMA, not three),
    and the two d x d products v = L'w, g = L h at 2 d^2 flops each."""
    return (OPS_PER_NORMAL * N * d + (OPS_PER_NORMAL - 2) * N * nu + OPS_PER_ASSET_STEP * d
            + 2 * 2 * d * d)


# Sources whose compiled code the paper-scale step runs; a counter summary taken on other sources
# no longer describes the kernel.
KERNEL_SOURCES = ("paper_2404_11631_amd/csrc/fw_paths.hip", "paper_2404_11631_amd/csrc/device_rng.hpp",
                  "paper_2404_11631_amd/csrc/device_reduce.hpp", "paper_2404_11631_amd/csrc/sim_types.hpp")
TRAFFIC_PROFILE = "profiles/hbm_traffic_paper_scale.md"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was taken on these sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = re.search(r"kernel source hash: `([0-9a-f]+)`", text)
    val = re.search(r"HBM bytes per launch: `([0-9.eE+]+)`", text)
    if not src or not val or src.group(1) != kernel_source_hash():
        return None
    return float(val.group(1))


def copy_probe(nbytes: int):
    """One plain copy of nbytes between two device buffers (fetch nbytes, write nbytes)."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)


def host_cpus():
    """What the host offers this process: logical CPUs (nproc), the affinity set, the cgroup CPU
    quota (cores' worth of time, None when unlimited) and the CPU model."""
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = nproc
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = aff if quota is None else max(1, min(aff, int(math.floor(quota + 1e-9))))
    return {"nproc": nproc, "affinity": aff, "cgroup_quota_cpus": quota, "model": model, "usable": usable}


def cpu_baseline(w, mu, sigma, seconds: float):
    """The oracle as it stands, on every host core this process may use (one thread per core of
    the affinity set, capped by the cgroup CPU quota), over a bounded sample of replications."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    host = host_cpus()
    threads = host["usable"]
    P = oracle.OracleProblem(mu, sigma, N=w["N"], seed=w["seed"], ckpt=w["checkpoints"])
    T = w["T"]
    # calibrate: one path on one thread
    t0 = time.perf_counter()
    P.run(1, T, r0=0)
    one = time.perf_counter() - t0
    per_thread = max(1, int(seconds / one))
    n = per_thread * threads

    def work(k):
        return P.run(per_thread, T, r0=1 + k * per_thread)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(threads)))
    el = time.perf_counter() - t0
    return {"value": n * T / el, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
            "nproc": host["nproc"], "affinity": host["affinity"], "cgroup_quota_cpus": host["cgroup_quota_cpus"],
            "cpu_model": host["model"], "single_thread_path_steps_per_s": T / one,
            "sample": f"{n} replications x T={T} of the paper-scale workload "
                      f"({per_thread} per thread on {threads} threads), serial FP64 oracle, {el:.1f} s wall"}


def oracle_single_core():
    """The serial FP64 oracle on one host thread, per configuration:
    - the tiny workload (d = 2, N = 2, T = 100, R = 1,000) in full;
    - the paper-scale workload on one replication of T = 10,000;
    - the uneven workload on one replication of each of 8 instances spread over the cost order;
    - the dense-L t(3) stress workload on one replication of T = 1,000.
    Each reports path-steps/s (normals/s for the uneven sample) and the full configuration's time
    extrapolated at that rate (by path-steps; by normals for the uneven workload)."""
    import numpy as np

    import oracle
    from paper_2404_11631_amd import workloads

    out = {"threads": 1, "kind": "oracle", "precision": "fp64"}

    def timed(f):
        t0 = time.perf_counter()
        f()
        return time.perf_counter() - t0

    c1 = workloads.WORKLOADS["tiny"]
    mu, sg = workloads.diag_instance(c1["seed"], 0, c1["d"])
    P = oracle.OracleProblem(mu, sg, N=c1["N"], seed=c1["seed"], ckpt=c1["checkpoints"])
    el = timed(lambda: P.run(c1["R"], c1["T"], r0=0))
    out["tiny"] = {"path_steps_per_s": c1["R"] * c1["T"] / el, "full_s": el, "sample": "the whole workload"}

    c2 = workloads.WORKLOADS["paper_scale"]
    mu, sg = workloads.diag_instance(c2["seed"], 0, c2["d"])
    P = oracle.OracleProblem(mu, sg, N=c2["N"], seed=c2["seed"], ckpt=c2["checkpoints"])
    el = timed(lambda: P.run(1, c2["T"], r0=0))
    rate = c2["T"] / el
    out["paper_scale"] = {"path_steps_per_s": rate, "full_s": c2["R"] * c2["T"] / rate,
                          "sample": "one replication of T = 10,000"}

    c3 = workloads.WORKLOADS["uneven"]
    batch = workloads.uneven_batch(c3["seed"], c3["n_instances"], c3["R"], c3["d_range"], c3["n_range"], c3["t_range"])
    order = np.argsort([b.T * b.N * b.d for b in batch])
    pick = [batch[int(order[k])] for k in range(0, len(batch), len(batch) // 8)][:8]
    normals = sum(b.N * b.d * b.T for b in pick)
    el = 0.0
    for b in pick:
        P = oracle.OracleProblem(b.mu, b.sigma, N=b.N, seed=c3["seed"], instance=b.instance)
        el += timed(lambda: P.run(1, b.T, r0=0))
    total_normals = sum(b.R * b.N * b.d * b.T for b in batch)
    out["uneven"] = {"normals_per_s": normals / el, "full_s": total_normals / (normals / el),
                     "sample": "one replication of each of 8 instances spread over the cost order"}

    c5 = workloads.WORKLOADS["stress"]
    mu, L = workloads.dense_instance(c5["seed"], 0, c5["d"])
    P = oracle.OracleProblem(mu, chol=L, N=c5["N"], noise=oracle.NOISE_T, nu=c5["nu"], seed=c5["seed"],
                             ckpt=c5["checkpoints"])
    el = timed(lambda: P.run(1, c5["T"], r0=0))
    rate = c5["T"] / el
    out["stress"] = {"path_steps_per_s": rate, "full_s": c5["R"] * c5["T"] / rate,
                     "sample": "one replication of T = 1,000"}
    return out


def parity_leg(ctx, sim, w, mu, sigma, n_log: int = 96):
    """Each statistic's error at the paper-scale workload (Algorithm 1, Section 3.1, binary32 state)
    against binary64 references, two ways.

    (a) The FP64 oracle run without replay on n_log replications of the benchmarked launch (the
        middle of the replication range, decisions logged): per path the decisions that differ, the
        steps whose LMO margin lies within the rounding bound (ambiguous), Y's relative error; then
        mean, variance, checkpoint means and RSE means of those paths, GPU vs oracle. The replayed
        oracle (logged decision adopted at ambiguous steps) must then agree everywhere else.
    (b) The same launch with binary64 state on the device over all R replications (its decisions
        match the oracle bit for bit in the parity tests): the full-R statistics' relative change."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    R, T, N, seed, ck = w["R"], w["T"], w["N"], w["seed"], w["checkpoints"]
    begin = R // 2 - n_log // 2
    p = sim.Problem(mu=mu, sigma=sigma, N=N, M=w["M"], precision=sim.FP32, checkpoints=ck, keep_paths=True,
                    log_reps=(begin, n_log))
    ctx.run(p, R, T, seed)
    st = ctx.stats()
    g = ctx.paths()
    P = oracle.OracleProblem(mu, sigma, N=N, M=w["M"], seed=seed, ckpt=ck)

    def one(k):
        r = begin + k
        free, dec = P.path(r, T, uroff=oracle.U32, want_decisions=True)
        rep = P.path(r, T, replay=g["decisions"][:, k], uroff=oracle.U32)
        return free, dec, rep

    threads = host_cpus()["usable"]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(n_log)))
    oracle_s = time.perf_counter() - t0
    outs = (oracle.PathOut * n_log)()
    diff_steps = diff_paths = amb_steps = amb_paths = rep_mismatch = 0
    y_err = []
    for k, (free, dec, rep) in enumerate(res):
        r = begin + k
        outs[k] = free
        dsteps = int(np.count_nonzero(dec[:T] != g["decisions"][:T, k]))
        diff_steps += dsteps
        diff_paths += dsteps > 0
        amb_steps += int(free.n_ambiguous)
        amb_paths += free.n_ambiguous > 0
        rep_mismatch += int(rep.n_mismatch)
        y_err.append(abs(g["y"][r] - free.y) / abs(free.y))
    ost = P.reduce(outs, T)
    Y = g["y"][begin:begin + n_log]
    F = g["f_ckpt"][:, begin:begin + n_log]
    m = math.fsum(Y) / n_log
    var = math.fsum((Y - m) ** 2) / (n_log - 1)

    def rel(a, b):
        return abs(a - b) / abs(b) if b != 0 else abs(a - b)

    errs = {"mean": rel(m, ost.mean), "var": rel(var, ost.var)}
    for c, t in enumerate(ck):
        fm = math.fsum(F[c]) / n_log
        ok = F[c] != 0
        rse = ((F[c][ok] - Y[ok]) / F[c][ok]) ** 2
        errs[f"f_mean@{t}"] = rel(fm, ost.f_mean[c])
        errs[f"rse_mean@{t}"] = rel(math.fsum(rse) / max(1, len(rse)), ost.rse_mean[c])
    sample = {"paths": n_log, "replications": [begin, begin + n_log], "oracle_s": oracle_s, "threads": threads,
              "paths_with_differing_decisions": diff_paths, "differing_steps": diff_steps,
              "ambiguous_paths": amb_paths, "ambiguous_path_fraction": amb_paths / n_log,
              "ambiguous_steps": amb_steps, "ambiguous_step_fraction": amb_steps / (n_log * T),
              "replay_unambiguous_mismatches": rep_mismatch,
              "y_rel_err_max": max(y_err), "y_rel_err_median": float(np.median(y_err)),
              "stat_rel_err": errs, "stat_rel_err_max": max(errs.values())}

    # (b) binary64 state over all replications, same seed
    p64 = sim.Problem(mu=mu, sigma=sigma, N=N, M=w["M"], precision=sim.FP64, checkpoints=ck)
    ctx.run(p64, R, T, seed)
    s64 = ctx.stats()
    full = {"R": R, "fp64_kernel_ms": s64.kernel_ms, "mean": rel(st.mean, s64.mean), "var": rel(st.var, s64.var),
            "mean_shift_over_ci95": abs(st.mean - s64.mean) / s64.ci95_halfwidth}
    for c, t in enumerate(ck):
        full[f"f_mean@{t}"] = rel(st.f_mean[c], s64.f_mean[c])
        full[f"rse_mean@{t}"] = rel(st.rse_mean[c], s64.rse_mean[c])
    d = len(mu)
    full["decision_total_rel_diff_max"] = max(
        abs(int(a) - int(b)) / max(1, int(b)) for a, b in zip(list(st.decision_total)[:d + 1],
                                                          list(s64.decision_total)[:d + 1]))
    return {"vs_fp64_oracle_sample": sample, "vs_fp64_state_full_R": full}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="paper_scale",
                    choices=("paper_scale", "stress", "paper_shape", "newsvendor_shape", "newsvendor_lp_shape", "sqn_shape", "uneven",
                             "uneven_batch"))
    ap.add_argument("--tune", action="store_true", help="uneven_batch: take theta from the measuring tuner")
    ap.add_argument("--heavy-factor", default="0", help="uneven_batch: theta of the tile plan, or a comma "
                    "list of them (0: the library's default)")
    ap.add_argument("--no-paper-shape", action="store_true", help="skip the Section 4.1 shape sweeps")
    ap.add_argument("--reps", type=int, default=0, help="replications of the stress workload (0: the full 1e7)")
    ap.add_argument("--sqn-sizes", default="", help="feature counts of the sqn_shape workload (comma list; "
                    "default: all of Section 4.1's)")
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--no-cv", action="store_true", help="skip the control-variate leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-parity", action="store_true", help="skip the statistics-error leg")
    ap.add_argument("--no-stress", action="store_true", help="skip the stress leg")
    ap.add_argument("--cv-train-runs", type=int, default=10, help="training simulations of 1e6 paths")
    ap.add_argument("--cv-epochs", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the simulation shards replications across GPUs only by "
              f"design (see DESIGN.md); --gpus {args.gpus} is not run.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "stress":
        stress(args)
        return
    if args.workload == "uneven":
        uneven_plain(args)
        return
    if args.workload == "uneven_batch":
        import torch

        from paper_2404_11631_amd import sim

        torch.cuda.init()
        ctx = sim.Sim(0, torch.cuda.current_stream().cuda_stream)
        if args.tune:
            print(json.dumps(uneven_batch_leg(ctx, sim, tune=True)), flush=True)
        for hf in (float(x) for x in str(args.heavy_factor).split(",") if float(x) >= 0 and not args.tune):
            print(json.dumps(uneven_batch_leg(ctx, sim, hf)), flush=True)
        ctx.close()
        return
    if args.workload in ("paper_shape", "newsvendor_shape", "newsvendor_lp_shape", "sqn_shape"):
        import torch

        from paper_2404_11631_amd import sim

        torch.cuda.init()
        ctx = sim.Sim(0, torch.cuda.current_stream().cuda_stream)
        leg = {"paper_shape": paper_shape_leg, "newsvendor_shape": newsvendor_shape_leg,
               "newsvendor_lp_shape": newsvendor_lp_shape_leg, "sqn_shape": sqn_shape_leg}[args.workload]
        kw = {}
        if args.workload == "sqn_shape" and args.sqn_sizes:
            kw["sizes"] = tuple(int(x) for x in args.sqn_sizes.split(","))
        print(json.dumps(leg(ctx, sim, max(1, args.steps), args.warmup, **kw)), flush=True)
        ctx.close()
        return

    import torch

    from paper_2404_11631_amd import sim, workloads

    w = workloads.WORKLOADS["paper_scale"]
    R, T, d, N, seed = w["R"], w["T"], w["d"], w["N"], w["seed"]
    mu, sigma = workloads.diag_instance(seed, 0, d)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = sim.Sim(0, stream.cuda_stream)
    p = sim.Problem(mu=mu, sigma=sigma, N=N, M=w["M"], precision=sim.FP32,
                    checkpoints=w["checkpoints"])

    for k in range(args.warmup):
        ctx.run(p, R, T, seed + 1000 + k)
        ctx.stats()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.run(p, R, T, seed + k)
        st = ctx.stats()
        kernel_ms.append(st.kernel_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    par = {} if args.no_parity else parity_leg(ctx, sim, w, mu, sigma)
    cv = None if args.no_cv else cv_leg(ctx, sim, w, mu, sigma, args)
    shape = None if args.no_paper_shape else paper_shape_leg(ctx, sim, 2, 1)
    nv_shape = None if args.no_paper_shape else newsvendor_shape_leg(ctx, sim, 2, 1)
    nv_lp_shape = None if args.no_paper_shape else newsvendor_lp_shape_leg(ctx, sim, 2, 1)
    sqn_shape = None if args.no_paper_shape else sqn_shape_leg(ctx, sim, 2, 1)
    table2 = None if args.no_paper_shape else table2_leg(ctx, sim)
    uneven = None if args.no_uneven else uneven_batch_leg(ctx, sim, tune=True)
    stress_r = None if args.no_stress else stress_leg(ctx, sim, args.reps or workloads.WORKLOADS["stress"]["R"])
    ctx.close()

    ms_step = 1e3 * wall / args.steps
    kavg = sum(kernel_ms) / len(kernel_ms)
    alg = ops_per_path_step(d, N) * R * T
    achieved = alg / (kavg * 1e-3)
    line = {
        "metric": METRIC,
        "value": R * T * args.steps / wall,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper_scale", "R": R, "T": T, "d": d, "N": N, "M": w["M"],
                   "state": "fp32", "statistics": "fp64 double-double", "seed": seed,
                   "launch": "one fused kernel per step"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_OPS, "traffic": measured_traffic(),
                     "kernel_ms": kavg, "ops_per_path_step": ops_per_path_step(d, N)},
        "stats": {"mean": st.mean, "ci95_halfwidth": st.ci95_halfwidth, "f_star": st.f_star, **par},
    }
    if cv is not None:
        line["cv"] = cv
    if shape is not None:
        line["paper_shape"] = shape
    if nv_shape is not None:
        line["newsvendor_shape"] = nv_shape
    if nv_lp_shape is not None:
        line["newsvendor_lp_shape"] = nv_lp_shape
    if sqn_shape is not None:
        line["sqn_shape"] = sqn_shape
    if table2 is not None:
        line["table2"] = table2
    if uneven is not None:
        line["uneven"] = uneven
    if stress_r is not None:
        line["stress"] = stress_r
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, mu, sigma, args.cpu_seconds)
        line["oracle_single_core"] = oracle_single_core()
    print(json.dumps(line), flush=True)


def _pool(parts):
    """Pooled (n, mean, unbiased variance) of independent groups given as (n, mean, var)."""
    n = sum(k for k, _, _ in parts)
    m = sum(k * x for k, x, _ in parts) / n
    ss = sum((k - 1) * v + k * (x - m) ** 2 for k, x, v in parts)
    return n, m, ss / max(1, n - 1)


WAVE_MAX_PATHS = 1024     # plain stages up to here: a path per wavefront (64 lanes, an asset per lane)
SPLIT_LANES = 16          # lanes per path for larger small plain stages (assets x sample chunks)
SPLIT_MAX_PATHS = 8192    # above this the fused kernel (one lane per path) fills the chip


def cv_leg(ctx, sim, w, mu, sigma, args):
    """Wall time to a 95% CI half-width h for E f(w_T) on the paper-scale instance (T = 1e4, d = N =
    10): plain Monte Carlo, the MLP control variate, and a linear (least-squares) control variate
    on the same d+2 features. Each form runs stages of fresh paths (at least 1,024 per stage),
    pools them, and stops at the first stage after which its realized half-width is <= h; the next
    stage is sized from the pooled variance. The wall time covers every stage (for the MLP form:
    features, surrogate evaluation and draws from the features' known law; for the linear form:
    features and the residuals). One-off costs are reported apart: training the surrogate (pairs
    simulated, Adam, beta on a held-out run), fitting the linear coefficients (on the same
    held-out pilot), and the calibration of the aux draws per path.

    Features have mean 0 under their exact law, so the linear form needs no aux draws:
    Y_lin = mean(Y - b'x). Reported at h = 1e-3 and at the h for which plain Monte Carlo needs
    about 1e6 paths (below ~1e5 paths every form is bound by one path's latency).

    The plain form runs a stage of at most WAVE_MAX_PATHS paths with a path per wavefront, of at most
    SPLIT_MAX_PATHS paths on the batched tile kernel with SPLIT_LANES lanes per path (one path's
    latency is then shorter), larger stages on the fused kernel; `plain_one_lane` is the same
    estimator always on the fused kernel, for comparison. Stages hold at least 1,024 paths."""
    import numpy as np
    import torch

    T, N = w["T"], w["N"]
    d = len(mu)
    p = sim.Problem(mu=mu, sigma=sigma, N=N, M=w["M"], precision=sim.FP32, checkpoints=(T,))
    cvw = __import__("paper_2404_11631_amd.workloads", fromlist=["WORKLOADS"]).WORKLOADS["control_variate"]
    eval_seed = cvw["seed"]
    R_min = 1024

    def sync_time():
        torch.cuda.synchronize()
        return time.perf_counter()

    t0 = time.perf_counter()
    fit = ctx.cv_fit(p, T, 1, n_runs=args.cv_train_runs, epochs=args.cv_epochs, R_train=1_000_000,
                     R_pilot=1 << 16, batch=4096, lr=1e-3)
    train_wall = time.perf_counter() - t0
    print(f"[cv] trained on {fit.n_train} pairs: loss {fit.loss_first_epoch:.4f} -> {fit.loss_last_epoch:.4f}, "
          f"beta {fit.beta:.3f}, pilot rho2 {fit.rho2:.3f}, {train_wall:.1f} s", file=sys.stderr, flush=True)

    # calibration on a held-out pilot (untimed, like training): cost of an aux draw relative to a
    # path, and the linear coefficients b by least squares of Y on (1, x)
    pilot_R = 1 << 16
    t0 = sync_time()
    cs = ctx.run_cv(p, pilot_R, T, eval_seed + 2, 1 << 20)
    cal = ctx.cv_paths()
    X = np.vstack([np.ones(pilot_R), cal["x"].astype(np.float64)]).T
    coef, *_ = np.linalg.lstsq(X, cal["y"], rcond=None)
    lin_b = coef[1:]
    calib_s = sync_time() - t0
    beta = cs.beta
    beta2_vh = beta ** 2 * cs.var_h_aux
    c_aux = (cs.aux_ms / (1 << 20)) / (cs.paths_ms / pilot_R)
    ratio = min(100.0, max(1.0, math.sqrt(beta2_vh / (c_aux * max(cs.var_resid, 1e-300)))))
    s_plain = math.sqrt(cs.var_plain)
    pf = sim.Problem(mu=mu, sigma=sigma, N=N, M=w["M"], precision=sim.FP32, checkpoints=(T,), keep_paths=True,
                     cv_features=True, cv_ref=np.array(fit.ref[:d]))

    def plain_one_lane_stage(R, seed):
        ctx.run(p, R, T, seed)
        st = ctx.stats()
        return (R, st.mean, st.var), None

    def plain_stage(R, seed):
        # A stage this small leaves most SIMDs idle on the fused kernel (one lane per path), and each
        # path's T dependent iterations set the wall time: spread each path over a wavefront (up to
        # WAVE_MAX_PATHS paths, one wavefront per SIMD) or over 16 lanes of the batched tile kernel.
        # Larger stages fill the chip and take the fused kernel, which has the higher throughput.
        if R > SPLIT_MAX_PATHS:
            return plain_one_lane_stage(R, seed)
        ctx.run_batch([p], [R], [T], seed=seed, lanes_per_rep=[64 if R <= WAVE_MAX_PATHS else SPLIT_LANES])
        st = ctx.batch_stats(0)
        return (R, st.mean, st.var), None

    def mlp_stage(R, seed):
        o = ctx.run_cv(p, R, T, seed, min(max(2, math.ceil(ratio * R)), 1 << 31))
        return (o.R, o.mean_resid, o.var_resid), (o.R_aux, o.mean_h_aux, o.var_h_aux)

    def lin_stage(R, seed):
        ctx.run(pf, R, T, seed)
        g = ctx.paths()
        res = g["y"] - lin_b @ g["x"].astype(np.float64)
        return (R, math.fsum(res) / R, float(np.var(res, ddof=1))), None

    def sequential(stage, h, seed0):
        t = sync_time()
        parts, aux, k, R_next = [], [], 0, R_min
        while True:
            a, b = stage(R_next, seed0 + 1000 * k)
            parts.append(a)
            if b is not None:
                aux.append(b)
            k += 1
            n, m, v = _pool(parts)
            var_est = v / n
            if aux:
                na, ma, va = _pool(aux)
                m += beta * ma
                var_est += beta ** 2 * va / na
            ci = 1.96 * math.sqrt(var_est)
            if ci <= h or k >= 8:
                break
            # paths still needed at the pooled variance per path, with a 2% margin
            R_next = max(R_min, math.ceil(1.02 * n * (ci / h) ** 2) - n)
        wall = sync_time() - t
        return {"R": n, "stages": k, "mean": m, "ci95": ci, "met": ci <= h, "wall_s": wall,
                "R_aux": sum(x[0] for x in aux) if aux else 0}

    plain_stage(R_min, eval_seed + 9)   # first use of the batched kernels in this process, untimed

    # the linear form's rho^2 on fresh paths (its own held-out check)
    ctx.run(pf, pilot_R, T, eval_seed + 7)
    g = ctx.paths()
    res = g["y"] - lin_b @ g["x"].astype(np.float64)
    rho2_lin = 1.0 - float(np.var(res, ddof=1)) / float(np.var(g["y"], ddof=1))
    out = {"workload": "control_variate", "instance": "paper_scale (seed 0)", "T": T, "d": d, "N": N,
           "train": {"pairs": fit.n_train, "steps": fit.steps, "epochs": args.cv_epochs, "wall_s": train_wall,
                     "sim_ms": fit.sim_ms, "train_ms": fit.train_ms, "loss_first_epoch": fit.loss_first_epoch,
                     "loss_last_epoch": fit.loss_last_epoch, "beta": fit.beta, "pilot_rho2": fit.rho2},
           "calibration_s": calib_s, "sd_plain": s_plain, "rho2_mlp": cs.rho2, "rho2_linear": rho2_lin,
           "variance_ratio_mlp": cs.var_plain / max(cs.var_resid, 1e-300),
           "variance_ratio_linear": 1.0 / max(1.0 - rho2_lin, 1e-300), "aux_per_path": ratio,
           "aux_cost_per_path": c_aux, "min_paths_per_stage": R_min,
           "plain_split": {"wave_max_paths": WAVE_MAX_PATHS, "lanes_per_path": SPLIT_LANES,
                           "max_paths": SPLIT_MAX_PATHS}, "targets": []}
    for h in (1e-3, 1.96 * s_plain / 1000.0):
        row = {"h": h}
        for name, stage, seed0 in (("plain", plain_stage, eval_seed + 3), ("cv", mlp_stage, eval_seed + 4),
                                   ("cv_linear", lin_stage, eval_seed + 5),
                                   ("plain_one_lane", plain_one_lane_stage, eval_seed + 3)):
            row[name] = sequential(stage, h, seed0)
        row["speedup"] = row["plain"]["wall_s"] / row["cv"]["wall_s"]
        row["speedup_linear"] = row["plain"]["wall_s"] / row["cv_linear"]["wall_s"]
        out["targets"].append(row)
        print(f"[cv] h={h:.3e}: plain R={row['plain']['R']} {row['plain']['wall_s']:.3f} s "
              f"ci {row['plain']['ci95']:.3e}; mlp R={row['cv']['R']} {row['cv']['wall_s']:.3f} s "
              f"ci {row['cv']['ci95']:.3e}; linear R={row['cv_linear']['R']} {row['cv_linear']['wall_s']:.3f} s "
              f"ci {row['cv_linear']['ci95']:.3e}; plain one lane per path {row['plain_one_lane']['wall_s']:.3f} s",
              file=sys.stderr, flush=True)
    return out


def paper_shape_leg(ctx, sim, runs: int, warmup: int):
    """Algorithm 1 at the shape of Section 4.1 (Task 1): one replication of d assets, mu ~ U(-1,1),
    sigma ~ U(0, 0.025), K = 1500 iterations, N = 25 samples per gradient (50 at d = 1e5), on the
    wide path (sim_run_wide). Per size: device time of the whole run (HIP events around its ~3 K
    launches), the wall time of the call and its statistics read-back, and the ALU roofline of the
    method's algorithmic work (23 lane-ops per normal, N d normals and ~15 d further operations per
    iteration; the device draws each normal twice, which is not counted). The paper reports about
    6 h on a Threadripper 3970X and 1 h on an RTX 3090 for the d = 1e5 run (context, other hardware)."""
    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["paper_shape"]
    T, seed = w["T"], w["seed"]
    out = {"workload": "paper_shape", "T": T, "R": w["R"], "regime": w["regime"], "runs": runs, "sizes": [],
           "paper_reported_s_at_1e5": {"rtx_3090": 3600, "threadripper_3970x": 21600}}
    for d in w["sizes"]:
        N = w["N"][d]
        mu, sig = workloads.diag_instance(seed, 0, d, w["regime"])
        p = sim.Problem(mu=mu, sigma=sig, N=N, M=w["M"], checkpoints=w["checkpoints"])
        for k in range(warmup):
            ctx.run_wide(p, w["R"], T, seed + 1000 + k)
            ctx.wide_stats()
        kms, walls = [], []
        for k in range(runs):
            t0 = time.perf_counter()
            ctx.run_wide(p, w["R"], T, seed + k)
            st = ctx.wide_stats()
            walls.append(time.perf_counter() - t0)
            kms.append(st.kernel_ms)
        kavg = sum(kms) / len(kms)
        ops = (23.0 * N * d + 15.0 * d) * T * w["R"]
        out["sizes"].append({"d": d, "N": N, "device_ms": kavg, "wall_ms": 1e3 * sum(walls) / len(walls),
                             "iterations_per_s": T / (kavg * 1e-3), "normals_per_s": N * d * T / (kavg * 1e-3),
                             "alu_frac": ops / (kavg * 1e-3) / PEAK_OPS, "Y": st.mean})
        print(f"[paper_shape] d={d} N={N}: {kavg:.1f} ms per run", file=sys.stderr, flush=True)
    return out


def newsvendor_shape_leg(ctx, sim, runs: int, warmup: int):
    """Algorithm 2 (Task 2) at the shape of Section 4.1: one replication of n products, K = 1500, S = 25
    demand samples per product (50 at n = 1e6), mu ~ U(20, 50), sigma ~ U(10, 20), on
    sim_run_newsvendor. Per size: device time of the run (HIP events around its launches), the
    wall time of the call and its read-back, and the sample throughput (S n demand samples per
    iteration). The gradient is an integer count, so the ALU fraction counts 23 lane-ops per normal and
    2 per comparison."""
    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["newsvendor_shape"]
    T, seed = w["T"], w["seed"]
    out = {"workload": "newsvendor_shape", "T": T, "R": w["R"], "runs": runs, "sizes": []}
    for n in w["sizes"]:
        S = w["S"][n]
        inst = workloads.newsvendor_instance(seed, 0, n)
        kw = dict(S=S, M=w["M"], checkpoints=w["checkpoints"])
        for k in range(warmup):
            ctx.run_newsvendor(inst, w["R"], T, seed + 1000 + k, **kw)
            ctx.nv_stats()
        kms, walls = [], []
        for k in range(runs):
            t0 = time.perf_counter()
            ctx.run_newsvendor(inst, w["R"], T, seed + k, **kw)
            st = ctx.nv_stats()
            walls.append(time.perf_counter() - t0)
            kms.append(st.kernel_ms)
        kavg = sum(kms) / len(kms)
        ops = 25.0 * S * n * T * w["R"]
        out["sizes"].append({"n": n, "S": S, "device_ms": kavg, "wall_ms": 1e3 * sum(walls) / len(walls),
                             "iterations_per_s": T / (kavg * 1e-3), "samples_per_s": S * n * T / (kavg * 1e-3),
                             "alu_frac": ops / (kavg * 1e-3) / PEAK_OPS, "Y": st.mean})
        print(f"[newsvendor_shape] n={n} S={S}: {kavg:.1f} ms per run", file=sys.stderr, flush=True)
    return out


def newsvendor_lp_shape_leg(ctx, sim, runs: int, warmup: int):
    """Algorithm 2 over Eq. (7)'s general constraint set with M = 3 resource rows
    (sim_run_newsvendor_lp: the linear subproblem solved on the device by a revised simplex per
    replication): one replication of n products, K = 1500, S = 25. Per size: device time of the run,
    the wall time of the call, and the simplex pivots per iteration."""
    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["newsvendor_lp_shape"]
    T, seed, m = w["T"], w["seed"], w["resources"]
    out = {"workload": "newsvendor_lp_shape", "T": T, "R": w["R"], "resources": m, "S": w["S"], "runs": runs,
           "sizes": []}
    for n in w["sizes"]:
        inst = workloads.newsvendor_instance(seed, 0, n)
        A, C = workloads.newsvendor_constraints(seed, 0, n, m)
        kw = dict(S=w["S"], M=w["M"], checkpoints=w["checkpoints"])
        for k in range(warmup):
            ctx.run_newsvendor_lp(inst, A, C, w["R"], T, seed + 1000 + k, **kw)
            ctx.nv_lp_stats()
        kms, walls = [], []
        for k in range(runs):
            t0 = time.perf_counter()
            ctx.run_newsvendor_lp(inst, A, C, w["R"], T, seed + k, **kw)
            st = ctx.nv_lp_stats()
            walls.append(time.perf_counter() - t0)
            kms.append(st.kernel_ms)
        piv = ctx.nv_lp_paths()["pivots"]
        kavg = sum(kms) / len(kms)
        out["sizes"].append({"n": n, "device_ms": kavg, "wall_ms": 1e3 * sum(walls) / len(walls),
                             "iterations_per_s": T / (kavg * 1e-3), "pivots_per_iteration": float(piv.mean()),
                             "max_pivots": int(piv.max()), "Y": st.mean})
        print(f"[newsvendor_lp_shape] n={n} M={m}: {kavg:.1f} ms per run, {piv.mean():.2f} pivots per iteration",
              file=sys.stderr, flush=True)
    return out


def sqn_bytes(n: int, K: int, L: int, M: int, b: int, bH: int, pair_bytes: int = 8) -> float:
    """HBM bytes one replication of the SQN kernel must move over K iterations: per iteration the two
    passes over the stored pairs (S'g, Y'g, then S a + Y c: 2 x 2 m n doubles), the b sampled rows'
    bits twice (the dot products, then the gradient) and the window sum (read and written); per window
    the new pair (s and y written, the previous average read and written), the b_H Hessian rows' bits
    three times (x'wbar, x's, then y) and the pair's dot products with the m stored pairs
    (S_i, Y_i, and Y_i again: 3 m n values). The pairs take pair_bytes per value (8, or 4 in binary32)."""
    row = 4 * (((n + 31) // 32 + 3) // 4 * 4)
    total, m, t = 0.0, 0, -1
    for k in range(1, K + 1):
        total += 2 * b * row + 16 * n
        if k > 2 * L:
            total += 4 * pair_bytes * m * n
        if k % L == 0:
            t += 1
            if t > 0:
                m = min(m + 1, M)
                total += 2 * pair_bytes * n + 8 * 2 * n + 3 * bH * row + 3 * pair_bytes * m * n
    return total


def sqn_shape_leg(ctx, sim, runs: int, warmup: int, throughput_sizes=(5_000,), sizes=None):
    """Task 3 (Algorithms 3-4) at Section 4.1's settings on sim_run_sqn: per feature count n (N = 30 n
    rows, M = 25, L = 10, b = 50, beta = 2, K = 2000) and b_H in {300, 600}, the device time of one
    run (the paper's single replication) on one workgroup and, under `split`, with the replication
    spread over many workgroups (sim_run_sqn_split), and at the sizes in `throughput_sizes` the throughput of
    R = 1024 replications in one launch (replication-iterations per second) against HBM bandwidth,
    with sqn_bytes as the algorithmic traffic. The loss evaluations at the checkpoints are timed
    apart (loss_ms)."""
    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["sqn_shape"]
    K, seed = w["K"], w["seed"]
    kw0 = dict(L=w["L"], M=w["M"], b=w["b"], beta=w["beta"], checkpoints=w["checkpoints"])
    out = {"workload": "sqn_shape", "K": K, "L": w["L"], "M": w["M"], "b": w["b"], "beta": w["beta"],
           "runs": runs, "precision": "f64", "sizes": []}
    for n in (sizes or w["sizes"]):
        X, z = workloads.sqn_dataset(seed, n)
        ctx.sqn_load(X, z)
        del X, z
        for bH in w["bH"]:
            kw = dict(kw0, bH=bH)
            for k in range(warmup):
                ctx.run_sqn(1, K, seed + 1000 + k, **kw)
                ctx.sqn_stats()
            kms, walls = [], []
            for k in range(runs):
                t0 = time.perf_counter()
                ctx.run_sqn(1, K, seed + k, **kw)
                st = ctx.sqn_stats()
                walls.append(time.perf_counter() - t0)
                kms.append(st.kernel_ms)
            kavg = sum(kms) / len(kms)
            entry = {"n": n, "N": 30 * n, "bH": bH, "device_ms": kavg, "wall_ms": 1e3 * sum(walls) / len(walls),
                     "iterations_per_s": K / (kavg * 1e-3), "F": st.mean,
                     "F_ckpt": [st.f_mean[c] for c in range(len(w["checkpoints"]))]}
            # the same runs with the replication spread over many workgroups (sim_run_sqn_split)
            for k in range(warmup):
                ctx.run_sqn(1, K, seed + 1000 + k, split=True, **kw)
                ctx.sqn_stats()
            sk, sw = [], []
            for k in range(runs):
                t0 = time.perf_counter()
                ctx.run_sqn(1, K, seed + k, split=True, **kw)
                ss = ctx.sqn_stats()
                sw.append(time.perf_counter() - t0)
                sk.append(ss.kernel_ms)
            savg = sum(sk) / len(sk)
            entry["split"] = {"device_ms": savg, "wall_ms": 1e3 * sum(sw) / len(sw),
                              "iterations_per_s": K / (savg * 1e-3), "F": ss.mean,
                              "speedup_vs_one_workgroup": kavg / savg}
            if n in throughput_sizes and bH == w["bH"][0]:
                # Algorithm 4's matrix formed from the pairs of that run (sim_sqn_hessian): the n x n
                # product on the FP64 matrix cores, 2 n^2 Kp flops (Kp = 2m rounded up to 4) and the
                # 8 n^2 bytes of H written, over the call's four launches (the product kernel alone is
                # in the kernel trace)
                hs = [ctx.sqn_hessian(0, copy=False) for _ in range(runs + 1)][1:]
                hms = sum(h["device_ms"] for h in hs) / len(hs)
                m = hs[0]["m"]
                Kp = (2 * m + 3) // 4 * 4
                entry["hessian"] = {"m": m, "device_ms": hms,
                                    "scope": "four launches: Gram entries, middle matrix, U and V, product",
                                    "tflops": 2.0 * n * n * Kp / (hms * 1e-3) / 1e12,
                                    "frac_fp64_mfma": 2.0 * n * n * Kp / (hms * 1e-3) / PEAK_F64,
                                    "write_GBps": 8.0 * n * n / (hms * 1e-3) / 1e9}
                R = w["R_batch"]
                ctx.run_sqn(R, K, seed + 2000, **kw)
                ctx.sqn_stats()
                bms = []
                for k in range(runs):
                    ctx.run_sqn(R, K, seed + 3000 + k, **kw)
                    stb = ctx.sqn_stats()
                    bms.append(stb.kernel_ms)
                bavg = sum(bms) / len(bms)
                alg = sqn_bytes(n, K, w["L"], w["M"], w["b"], bH) * R
                entry["batch"] = {"R": R, "device_ms": bavg, "rep_iterations_per_s": R * K / (bavg * 1e-3),
                                  "F_mean": stb.mean, "F_ci95_halfwidth": stb.ci95_halfwidth,
                                  "roofline": {"bound": "hbm", "achieved": alg / (bavg * 1e-3) / 1e9,
                                               "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                               "frac": alg / (bavg * 1e-3) / PEAK_HBM,
                                               "bytes_per_rep": alg / R}}
                # the same launch with the pairs kept in binary32
                kw32 = dict(kw, pairs_fp32=True)
                ctx.run_sqn(R, K, seed + 2000, **kw32)
                ctx.sqn_stats()
                fms = []
                for k in range(runs):
                    ctx.run_sqn(R, K, seed + 3000 + k, **kw32)
                    stf = ctx.sqn_stats()
                    fms.append(stf.kernel_ms)
                favg = sum(fms) / len(fms)
                alg32 = sqn_bytes(n, K, w["L"], w["M"], w["b"], bH, pair_bytes=4) * R
                entry["batch_fp32_pairs"] = {
                    "R": R, "device_ms": favg, "rep_iterations_per_s": R * K / (favg * 1e-3), "F_mean": stf.mean,
                    "roofline": {"bound": "hbm", "achieved": alg32 / (favg * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                                 "unit": "GB/s", "frac": alg32 / (favg * 1e-3) / PEAK_HBM, "bytes_per_rep": alg32 / R}}
            out["sizes"].append(entry)
            print(f"[sqn_shape] n={n} bH={bH}: {kavg:.1f} ms per run (split: {savg:.1f} ms)"
                  + (f", R={entry['batch']['R']}: {entry['batch']['device_ms']:.1f} ms" if "batch" in entry else ""),
                  file=sys.stderr, flush=True)
    return out


# Table 2 of the paper (GPU column): mean RSE in percent at iterations 50, 100, 500, 1000 over seven
# runs, on the paper's own instances and hardware (context only: instances, seeds and start points
# differ here)
TABLE2_PAPER_GPU = {"asset_5k": [85.07, 62.41, 24.07, 13.39], "inventory_10k": [89.92, 76.25, 40.94, 20.58],
                    "classification_1k": [72.16, 51.06, 31.29, 15.59]}


def table2_leg(ctx, sim):
    """Table 2's statistic on this library: RSE_c = ((f_c - f_K) / f_c)^2 at c in {50, 100, 500, 1000},
    mean and standard deviation over R = 7 replications, in percent, for Task 1 at d = 5000 (wide
    path, paper regime, N = 25, K = 1500), Task 2 at n = 1e4 (S = 25, K = 1500) and Task 3 at
    n = 1000 (N = 30 n, K = 2000, b_H = 300), beside the paper's GPU column."""
    from paper_2404_11631_amd import workloads

    ck = (50, 100, 500, 1000)
    out = {"R": 7, "checkpoints": list(ck), "unit": "percent", "rows": {}}

    def row(name, st, device_ms):
        out["rows"][name] = {"rse_mean": [100.0 * st.rse_mean[c] for c in range(len(ck))],
                             "rse_sd": [100.0 * st.rse_sd[c] for c in range(len(ck))],
                             "paper_gpu_mean": TABLE2_PAPER_GPU[name], "device_ms": device_ms}

    mu, sig = workloads.diag_instance(0, 0, 5000, "paper")
    ctx.run_wide(sim.Problem(mu=mu, sigma=sig, N=25, checkpoints=ck), 7, 1500, 11)
    st = ctx.wide_stats()
    row("asset_5k", st, st.kernel_ms)
    inst = workloads.newsvendor_instance(0, 0, 10_000)
    ctx.run_newsvendor(inst, 7, 1500, 12, S=25, checkpoints=ck)
    st = ctx.nv_stats()
    row("inventory_10k", st, st.kernel_ms)
    X, z = workloads.sqn_dataset(0, 1000)
    ctx.sqn_load(X, z)
    ctx.run_sqn(7, 2000, 13, bH=300, checkpoints=ck)
    st = ctx.sqn_stats()
    row("classification_1k", st, st.kernel_ms)
    print("[table2] " + "; ".join(f"{k}: {[round(x, 2) for x in v['rse_mean']]}" for k, v in out["rows"].items()),
          file=sys.stderr, flush=True)
    return out


def uneven_batch_leg(ctx, sim, heavy_factor: float = 0.0, lanes=None, tune: bool = False):
    """The uneven workload (256 instances: d ~ U{2..32}, N ~ U{2..50}, T log-uniform in [100, 1e5],
    4096 replications each) in one sim_run_batch call: wavefront tiles of every instance, heavy
    instances split over several lanes per replication, longest tiles first, then the per-instance
    reduction. Wall time of the call to the last statistics read back; device time between the
    run's HIP events; ALU roofline of the method's algorithmic work over the device time."""
    import torch

    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["uneven"]
    batch = workloads.uneven_batch(w["seed"], w["n_instances"], w["R"], w["d_range"], w["n_range"], w["t_range"])
    probs = [sim.Problem(mu=b.mu, sigma=b.sigma, N=b.N, M=1, precision=sim.FP32, instance_id=b.instance)
             for b in batch]
    R = [b.R for b in batch]
    T = [b.T for b in batch]
    tuned = None
    if tune:
        # the measured plan knob, outside the timed region (cached across runs of the same box)
        import tempfile
        t0 = time.perf_counter()
        tuned = ctx.tune_batch(probs, R, T, seed=w["seed"] + 1, t_scale=16,
                               cache=os.path.join(tempfile.gettempdir(), "sim_batch_tune.json"))
        tuned["wall_s"] = time.perf_counter() - t0
        heavy_factor = tuned["heavy_factor"]
    # library set-up and buffers: one small batch of the same classes
    ctx.run_batch(probs[:4], [64] * 4, [100] * 4, seed=1)
    ctx.batch_stats(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_batch(probs, R, T, seed=w["seed"], heavy_factor=heavy_factor, lanes_per_rep=lanes)
    sts = [ctx.batch_stats(i) for i in range(len(batch))]
    wall = time.perf_counter() - t0
    kms = sts[0].kernel_ms
    plan_P = [ctx.batch_paths(i)["lanes_per_rep"] for i in range(len(batch))]
    steps = sum(b.R * b.T for b in batch)
    ops = sum(b.R * b.T * ops_per_path_step(b.d, b.N) for b in batch)
    heavy = max(range(len(batch)), key=lambda i: batch[i].T * batch[i].N * batch[i].d)
    return {"workload": "uneven", "instances": len(batch), "R": w["R"], "path_steps": steps,
            "normals": sum(b.R * b.T * b.N * b.d for b in batch), "wall_s": wall, "kernel_ms": kms,
            "path_steps_per_s": steps / wall,
            "roofline": {"bound": "alu", "achieved": ops / (kms * 1e-3) / 1e12, "peak": PEAK_OPS / 1e12,
                         "unit": "TOP/s", "frac": ops / (kms * 1e-3) / PEAK_OPS},
            "heavy_factor": heavy_factor or 0.5, "tuner": tuned,
            "lanes_per_rep_histogram": {str(p): plan_P.count(p) for p in sorted(set(plan_P))},
            "heaviest_instance": {"i": heavy, "d": batch[heavy].d, "N": batch[heavy].N, "T": batch[heavy].T,
                                  "lanes_per_rep": plan_P[heavy]},
            "mean_of_instance_0": sts[0].mean}


def uneven_plain(args):
    """The uneven workload (256 instances: d ~ U{2..32}, N ~ U{2..50}, T log-uniform in [100, 1e5],
    4096 replications each) on the plain fused path, instance by instance: four contexts on four
    streams of default priority, instances longest first, round robin, each context reading its
    statistics before it takes the next instance. The batched device path (one launch for all
    instances) is switched off; this measures the workload without it."""
    import torch

    from paper_2404_11631_amd import sim, workloads

    w = workloads.WORKLOADS["uneven"]
    batch = workloads.uneven_batch(w["seed"], w["n_instances"], w["R"], w["d_range"], w["n_range"], w["t_range"])
    torch.cuda.init()
    n_ctx = 4
    streams = [torch.cuda.Stream() for _ in range(n_ctx)]
    ctxs = [sim.Sim(0, s.cuda_stream) for s in streams]
    order = sorted(range(len(batch)), key=lambda i: -batch[i].T * batch[i].N * batch[i].d)
    problems = {i: sim.Problem(mu=batch[i].mu, sigma=batch[i].sigma, N=batch[i].N, M=1, precision=sim.FP32)
                for i in order}
    # one small run per context first (library set-up, buffers)
    for c in ctxs:
        c.run(problems[order[-1]], 64, 100, 1)
        c.stats()
    torch.cuda.synchronize()
    pending = [None] * n_ctx
    kms = {}
    t0 = time.perf_counter()
    for k, i in enumerate(order):
        c = k % n_ctx
        if pending[c] is not None:
            kms[pending[c]] = ctxs[c].stats().kernel_ms
        ctxs[c].run(problems[i], batch[i].R, batch[i].T, w["seed"] + 1 + i)
        pending[c] = i
        if k % 32 == 0:
            print(f"[uneven] {k} of {len(order)} instances launched", file=sys.stderr, flush=True)
    for c in range(n_ctx):
        if pending[c] is not None:
            kms[pending[c]] = ctxs[c].stats().kernel_ms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    steps = sum(b.R * b.T for b in batch)
    ops = sum(b.R * b.T * ops_per_path_step(b.d, b.N) for b in batch)
    line = {
        "metric": "path-steps/s, uneven workload on the plain path (instance by instance, 4 streams)",
        "value": steps / wall, "unit": "path-steps/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * wall, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven", "instances": len(batch), "R": w["R"], "d": list(w["d_range"]),
                   "N": list(w["n_range"]), "T": list(w["t_range"]), "streams": n_ctx},
        "roofline": {"bound": "alu", "achieved": ops / wall / 1e12, "peak": PEAK_OPS / 1e12, "unit": "TOP/s",
                     "frac": ops / wall / PEAK_OPS, "traffic": None},
        "path_steps": steps, "wall_s": wall, "sum_kernel_ms": sum(kms.values()),
        "longest_instance_ms": max(kms.values()),
    }
    print(json.dumps(line), flush=True)


def stress_cv(ctx, sim, p, T: int, seed: int, R_eval: int = 1 << 20):
    """The control variate on the stress shape (dense factor, t(3)): the MLP trained on the device
    from 2^20 simulated pairs, then one estimate over R_eval fresh paths with the aux draws sized as
    in the paper-scale leg; reports the variance ratio it reaches (the plain mean of the same paths
    is the judge of its bias)."""
    t0 = time.perf_counter()
    fit = ctx.cv_fit(p, T, seed + 1, n_runs=1, epochs=4, R_train=1 << 20, R_pilot=1 << 16, batch=4096, lr=2e-3)
    train_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = ctx.run_cv(p, R_eval, T, seed + 2, 4 * R_eval)
    wall = time.perf_counter() - t0
    joint = math.sqrt(st.ci95_plain ** 2 + st.ci95_cv ** 2)
    print(f"[stress] cv: rho2 {st.rho2:.4f}, variance gain {(st.var_plain / st.R) / st.var_est:.3f}, "
          f"train {train_s:.1f} s", file=sys.stderr, flush=True)
    return {"train_pairs": fit.n_train, "train_s": train_s, "train_sim_ms": fit.sim_ms, "train_ms": fit.train_ms,
            "pilot_rho2": fit.rho2, "beta": st.beta, "R": st.R, "R_aux": st.R_aux, "rho2": st.rho2,
            "variance_gain": (st.var_plain / st.R) / st.var_est, "mean_plain": st.mean_plain,
            "ci95_plain": st.ci95_plain, "mean_cv": st.mean_cv, "ci95_cv": st.ci95_cv,
            "cv_minus_plain_over_joint_ci95": (st.mean_cv - st.mean_plain) / joint, "wall_s": wall,
            "paths_ms": st.paths_ms, "aux_ms": st.aux_ms,
            "path_steps_per_s_with_features": st.R * T / (st.paths_ms * 1e-3)}


def stress_leg(ctx, sim, R: int, runs: int = 1, warmup: int = 0, cv: bool = True):
    """The stress workload (d = 64 dense L with Sigma = L L', standardized t(3) noise, N = 100,
    T = 1e3, R = 1e7 by default) on the dense-L kernel: per iteration the two d x d products
    v = L'w and g = L h run on the FP32 matrix cores, the normals on the vector ALUs. Reports the
    device time per run, path-steps/s, the ALU roofline of the method's algorithmic work and the
    matrix-core share (4 d^2 flops per path-step against the dense FP32 matrix peak)."""
    import torch

    from paper_2404_11631_amd import workloads

    w = workloads.WORKLOADS["stress"]
    T, d, N, nu, seed = w["T"], w["d"], w["N"], w["nu"], w["seed"]
    mu, L = workloads.dense_instance(seed, 0, d)
    p = sim.Problem(mu=mu, chol=L, N=N, M=w["M"], noise=sim.NOISE_T, nu=nu, checkpoints=w["checkpoints"])
    for k in range(warmup):
        ctx.run(p, min(R, 1 << 20), T, seed + 1000 + k)
        ctx.stats()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for k in range(runs):
        ctx.run(p, R, T, seed + k)
        st = ctx.stats()
        kernel_ms.append(st.kernel_ms)
        print(f"[stress] run {k}: R={R} {st.kernel_ms:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kavg = sum(kernel_ms) / len(kernel_ms)
    alg = ops_per_path_step_dense(d, N, nu) * R * T
    mfma = 4.0 * d * d * R * T
    cv_out = stress_cv(ctx, sim, p, T, seed) if cv else None
    return {"cv": cv_out, "workload": "stress", "R": R, "T": T, "d": d, "N": N, "noise": f"t({nu})", "L": "dense lower-triangular",
            "seed": seed, "runs": runs, "wall_s": wall, "kernel_ms": kavg, "path_steps_per_s": R * T * runs / wall,
            "roofline": {"bound": "alu", "achieved": alg / (kavg * 1e-3) / 1e12, "peak": PEAK_OPS / 1e12,
                         "unit": "TOP/s", "frac": alg / (kavg * 1e-3) / PEAK_OPS,
                         "ops_per_path_step": ops_per_path_step_dense(d, N, nu)},
            "mfma": {"achieved": mfma / (kavg * 1e-3) / 1e12, "peak": PEAK_F32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": mfma / (kavg * 1e-3) / PEAK_F32_MFMA, "flops_per_path_step": 4 * d * d},
            "stats": {"mean": st.mean, "ci95_halfwidth": st.ci95_halfwidth,
                      "decision_total_origin": int(st.decision_total[0])}}


def stress(args):
    """The stress workload alone (see stress_leg), one JSON line."""
    import torch

    from paper_2404_11631_amd import sim, workloads

    w = workloads.WORKLOADS["stress"]
    torch.cuda.init()
    ctx = sim.Sim(0, torch.cuda.current_stream().cuda_stream)
    leg = stress_leg(ctx, sim, args.reps or w["R"], max(1, args.steps), args.warmup)
    ctx.close()
    line = {"metric": "path-steps/s, dense-L t(3) stress workload", "value": leg["path_steps_per_s"],
            "unit": "path-steps/s", "n_gpus": 1, "steps": leg["runs"], "warmup": args.warmup,
            "ms_per_step": 1e3 * leg["wall_s"] / leg["runs"], "higher_is_better": True, "dtype": "f32",
            "data": "synthetic", "config": {k: leg[k] for k in ("workload", "R", "T", "d", "N", "noise", "L", "seed")},
            "roofline": leg["roofline"], "mfma": leg["mfma"], "stats": leg["stats"], "cv": leg["cv"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
