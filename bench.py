"""Throughput of the batched stochastic Frank-Wolfe simulation on one MI355X.

A step is one sim_run over the paper-scale workload (R = 1e6 replications of Algorithm 1,
T = 1e4 iterations, d = 10 assets, N = 10 samples per gradient, FP32 state, FP64 statistics),
fused with its cross-path reduction, followed by sim_stats; every step draws fresh noise (seed
+ step). Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--cpu-seconds 20] [--no-cpu-baseline]

Other measurements (not the headline line):
    --workload stress [--reps R]   the dense-L, t(3) stress workload (d = 64, N = 100, T = 1e3)
    --copy-probe BYTES             one plain device-to-device copy of BYTES, for calibrating the
                                   FETCH_SIZE / WRITE_SIZE counters against known traffic
"""
from __future__ import annotations

import argparse
import hashlib
import json
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


def cpu_baseline(w, mu, sigma, seconds: float):
    """The oracle as it stands, on the host cores, over a bounded sample of replications."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    threads = min(16, os.cpu_count() or 1)
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
            "sample": f"{n} replications x T={T} of the paper-scale workload "
                      f"({per_thread} per thread), serial FP64 oracle, {el:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="paper_scale", choices=("paper_scale", "stress"))
    ap.add_argument("--reps", type=int, default=0, help="replications (stress only; 0: the full 1e7)")
    ap.add_argument("--copy-probe", type=int, default=0)
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
        "stats": {"mean": st.mean, "ci95_halfwidth": st.ci95_halfwidth, "f_star": st.f_star},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, mu, sigma, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def stress(args):
    """The stress workload: d = 64 dense L (Sigma = L L'), standardized t(3) noise, N = 100, T = 1e3,
    R = 1e7 (or --reps); the two d x d products per iteration run on the matrix cores."""
    import torch

    from paper_2404_11631_amd import sim, workloads

    w = workloads.WORKLOADS["stress"]
    R = args.reps or w["R"]
    T, d, N, nu, seed = w["T"], w["d"], w["N"], w["nu"], w["seed"]
    mu, L = workloads.dense_instance(seed, 0, d)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = sim.Sim(0, stream.cuda_stream)
    p = sim.Problem(mu=mu, chol=L, N=N, M=w["M"], noise=sim.NOISE_T, nu=nu, checkpoints=w["checkpoints"])
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
        print(f"[stress] step {k}: {st.kernel_ms:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    kavg = sum(kernel_ms) / len(kernel_ms)
    alg = ops_per_path_step_dense(d, N, nu) * R * T
    line = {
        "metric": "path-steps/s, dense-L t(3) stress workload",
        "value": R * T * args.steps / wall, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stress", "R": R, "T": T, "d": d, "N": N, "noise": f"t({nu})",
                   "L": "dense lower-triangular", "seed": seed},
        "roofline": {"bound": "alu", "achieved": alg / (kavg * 1e-3) / 1e12, "peak": PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": alg / (kavg * 1e-3) / PEAK_OPS, "traffic": None,
                     "kernel_ms": kavg, "ops_per_path_step": ops_per_path_step_dense(d, N, nu)},
        "stats": {"mean": st.mean, "ci95_halfwidth": st.ci95_halfwidth},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
