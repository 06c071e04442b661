"""Benchmark of the K-means-seeded elitist GA for pilot assignment on one MI355X.

A step is one whole solve of the workload (K-means seeding, initial fitness,
G generations of elitism / selection / crossover / mutation / fitness, best
chromosome back on the host).  The default workload is a single instance with
L = 19 hexagonal cells, K = tau = 16 users, M = 256, T = 196, a population of
256, 500 generations and 8 elites.  `value` is chromosome fitness
evaluations per second: (N + (N - E) * G) per solve over the timed solves,
inputs resident in HBM.

Prints ONE JSON line on stdout (progress goes to stderr).
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

LDS_PEAK_GBS = 256 * 2.4e9 * 128 / 1e9  # 256 CUs x 2.4 GHz x 128 B/clk (ds_read_b32, 32 banks)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def evals_per_solve(N, E, G):
    return N + (N - E) * G


def cpu_baseline(drop, w, budget_s=12.0):
    """The FP64 oracle, single-threaded, on whole solves of the same workload."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    solves = 0
    while True:
        oracle.solve(drop.beta, drop.user_xy, drop.bs_xy, w["N"], w["gens"], w["E"], w["p_cross"],
                     w["p_mut"], w["kmeans_frac"], w["p_init"], w["seed"], 0, T=w["T"])
        solves += 1
        el = time.perf_counter() - t0
        if el >= budget_s or solves >= 3:
            break
    ev = solves * evals_per_solve(w["N"], w["E"], w["gens"])
    return {"value": ev / el, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{solves} full oracle solve(s) of the same workload ({el:.1f} s, FP64, 1 thread)"}


def run_batch(pa, scenario, torch, name):
    """Many independent instances in one graph-captured batch: evals/s and solves/s."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    L, K, N, G, E, n = w["L"], w["K"], w["N"], w["gens"], w["E"], w["instances"]
    ctx = pa.pa_context_create(0)
    insts, params = [], []
    for i in range(n):
        d = scenario.make_drop(L, K, seed=w["seed"], instance_id=i)
        insts.append(pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"],
                                           rho=scenario.snr_to_rho(w["snr_db"])))
        params.append(pa.GaParams(pop=N, gens=G, elite=E, p_cross=w["p_cross"], p_mut=w["p_mut"],
                                  kmeans_frac=w["kmeans_frac"], p_init=w["p_init"],
                                  seed=w["seed"], instance_id=i))
    pa.pa_solve_batch(ctx, insts, params)  # builds and captures the plan
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = []
    for _ in range(reps):
        res = pa.pa_solve_batch(ctx, insts, params)
        dev.append(res[0].device_ms)
    wall = (time.perf_counter() - t0) / reps
    ev = n * evals_per_solve(N, E, G)
    gathers = n * (N + (N - E) * G) * L * L * K
    out = {"workload": name, "instances": n, "L": L, "K": K, "pop": N, "gens": G,
           "ms_per_batch": wall * 1e3, "device_ms": float(np.median(dev)),
           "evals_per_s": ev / wall, "solves_per_s": n / wall,
           "lds_gbs": gathers * 4 / wall / 1e9,
           "lds_frac_of_peak": gathers * 4 / wall / 1e9 / LDS_PEAK_GBS,
           "best_fit_first": res[0].best_fit}
    log(f"batch {name}: {wall * 1e3:.1f} ms, {ev / wall:.3e} evals/s, {n / wall:.1f} solves/s, "
        f"LDS {out['lds_gbs']:.0f} GB/s ({100 * out['lds_frac_of_peak']:.1f}%)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single_L19_K16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--batch", default="batch64_L37_K32",
                    help="also time this batched workload ('' to skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (5 times) and exit: the "
                         "reference kernel that scales HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(each instance runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB x 5 (read {n >> 10} KiB, write {n >> 10} KiB per copy)")
        return

    import paper_2511_20511_amd as pa
    from paper_2511_20511_amd import scenario

    w = dict(scenario.WORKLOADS[args.workload])
    L, K, N, G, E = w["L"], w["K"], w["N"], w["gens"], w["E"]
    rho = scenario.snr_to_rho(w["snr_db"])
    drop = scenario.make_drop(L, K, seed=w["seed"], instance_id=0)
    ctx = pa.pa_context_create(0)
    inst = pa.pa_instance_create(ctx, drop.beta, drop.user_xy, drop.bs_xy, T=w["T"], M=w["M"],
                                 rho=rho)
    params = pa.GaParams(pop=N, gens=G, elite=E, p_cross=w["p_cross"], p_mut=w["p_mut"],
                         kmeans_frac=w["kmeans_frac"], p_init=w["p_init"], seed=w["seed"],
                         instance_id=0)
    stream = torch.cuda.current_stream()

    log(f"workload {args.workload}: L={L} K={K} N={N} G={G} E={E}")
    for _ in range(args.warmup):
        pa.pa_solve(inst, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    res = None
    for _ in range(args.steps):
        res = pa.pa_solve(inst, params)
        dev_ms.append(res.device_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    ev = evals_per_solve(N, E, G)
    value = ev * args.steps / wall
    log(f"solve: {ms_per_step:.3f} ms/solve wall, device {np.median(dev_ms):.3f} ms, "
        f"best {res.best_fit:.4f}")

    # plain comparator: one launch per step, no fusion, no graph
    pa.pa_solve_plain(inst, params)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain_steps = max(1, args.steps // 2)
    for _ in range(plain_steps):
        pa.pa_solve_plain(inst, params)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t1) * 1e3 / plain_steps
    log(f"plain solve (one launch per step): {plain_ms:.3f} ms/solve")

    # dominant kernel: the generation kernel, timed with events on the stream
    # it is launched on.  Persistent form: one launch runs all G generations
    # (pa_solve_next(G)); graph form: one launch per generation.
    shape = pa.pa_solve_shape(None, inst)
    log(f"solve plan: {shape}")
    TP = max(4, 1 << (K - 1).bit_length())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pa.pa_solve_begin(inst, params)
    if shape["persistent"]:
        gens_per_launch, launches = G, 1
        kname = f"k_gen_persist<{L},{TP},0,{shape['block']}>"
    else:
        pa.pa_solve_next(inst, 10)
        gens_per_launch, launches = 1, min(args.kernel_iters, G - 10)
        kname = f"k_gen_exact<{L},{TP},0,{shape['block']}>"
    e0.record(stream)
    pa.pa_solve_next(inst, gens_per_launch * launches)
    e1.record(stream)
    e1.synchronize()
    k_ms = e0.elapsed_time(e1) / launches
    # algorithmic LDS bytes of one launch: every child reads one 4-byte table
    # word per (BS, cell, pilot)
    lds_bytes = (N - E) * gens_per_launch * L * L * K * 4
    achieved = lds_bytes / (k_ms * 1e-3) / 1e9
    roofline = {"bound": "lds", "kernel": kname,
                "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / LDS_PEAK_GBS, "traffic": None,
                "avg_launch_us": k_ms * 1e3, "bytes_per_launch": lds_bytes,
                "generations_per_launch": gens_per_launch}
    log(f"generation kernel {kname}: {k_ms * 1e3:.2f} us/launch ({gens_per_launch} generation(s)), "
        f"{achieved:.0f} GB/s LDS ({100 * achieved / LDS_PEAK_GBS:.1f}% of {LDS_PEAK_GBS:.0f})")

    extra = {}
    if args.batch:
        extra["batch"] = run_batch(pa, scenario, torch, args.batch)
    line = {
        "metric": "chromosome fitness evals/s", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": L, "K": K, "tau": K, "M": w["M"], "T": w["T"],
                   "pop": N, "gens": G, "elite": E, "instances": 1},
        "solves_per_s": args.steps / wall,
        "solve_device_ms": float(np.median(dev_ms)),
        "plain_solve_ms": plain_ms,
        "solve_plan": shape,
        "roofline": roofline,
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(drop, w)
        log(f"oracle: {line['cpu_baseline']['value']:.0f} evals/s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
