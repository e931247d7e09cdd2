"""Throughput of the batched stochastic Frank-Wolfe simulation on one MI355X.

A step is one sim_run over the paper-scale workload (R = 1e6 replications of Algorithm 1,
T = 1e4 iterations, d = 10 assets, N = 10 samples per gradient, FP32 state, FP64 statistics),
fused with its cross-path reduction, followed by sim_stats; every step draws fresh noise (seed
+ step). Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--cpu-seconds 20] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "path-steps/sec and wall time to 95% CI half-width 1e-3, plain vs CV, 1 MI355X"

# Issue-slot roofline of the path: each normal costs 5 wide 32x32->64 integer
# products and 10 xors (Philox4x32-10, 10 rounds per 4 normals), 2 transcendentals (Box-Muller:
# log2, sqrt, sin, cos per pair), 3 uniform-map ops and 3 accumulation ops; each iteration adds
# ~15 d ops for gradient, linear subproblem and update. Costs in issue slots, measured on gfx950:
SLOT_MAD64 = 4.0     # v_mad_u64_u32
SLOT_TRANS = 4.0     # v_log_f32, v_sqrt_f32, v_sin_f32, v_cos_f32
SLOT_SIMPLE = 1.0
PEAK_SLOTS = 256 * 64 * 2.4e9   # 256 CUs x 64 lanes x 2.4 GHz: one 32-bit VALU op per lane per clock


def slots_per_path_step(d: int, N: int) -> float:
    per_normal = 5 * SLOT_MAD64 + 2 * SLOT_TRANS + (10 + 3 + 3) * SLOT_SIMPLE
    return N * d * per_normal + 15 * d * SLOT_SIMPLE


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the simulation shards replications across GPUs only by "
              f"design (see DESIGN.md); --gpus {args.gpus} is not run.", file=sys.stderr)
        sys.exit(2)

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
    alg = slots_per_path_step(d, N) * R * T
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
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS, "traffic": None,
                     "kernel_ms": kavg},
        "stats": {"mean": st.mean, "ci95_halfwidth": st.ci95_halfwidth, "f_star": st.f_star},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, mu, sigma, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
