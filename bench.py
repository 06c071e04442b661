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


def source_sha256():
    """Hash of the kernel sources and the C ABI header (the HBM counters in
    profiles/ are valid only for the sources they were taken from)."""
    import hashlib
    h = hashlib.sha256()
    for d in ("paper_2511_20511_amd/csrc", "include"):
        for f in sorted(os.listdir(os.path.join(ROOT, d))):
            h.update(f.encode())
            with open(os.path.join(ROOT, d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, gens_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter passes, or None
    when they were taken for another kernel, workload or source version."""
    path = os.path.join(ROOT, "profiles", f"k_gen_persist_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel") != kernel or rec.get("generations_per_launch") != gens_per_launch
            or rec.get("source_sha256") != source_sha256()):
        return None
    return float(rec["bytes_per_launch"])


def evals_per_solve(N, E, G):
    return N + (N - E) * G


def cpu_baseline(drop, w, best=None, best_fit=None, budget_s=12.0):
    """The FP64 oracle, single-threaded, on whole solves of the same workload;
    also the FP64 fitness of the GPU's best chromosome (its FP32 error)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    err = None
    if best is not None:
        f64 = float(oracle.fitness(drop.beta, best[None].astype(np.uint8), T=w["T"])[0])
        err = abs(best_fit - f64) / abs(f64)
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
            "sample": f"{solves} full oracle solve(s) of the same workload ({el:.1f} s, FP64, 1 thread)",
            "best_fp32_rel_err_vs_fp64": err}


def workload_sizes(scenario, w, n):
    """(L, K, N) of the n instances of a workload (uniform, or the uneven size mix)."""
    if w.get("mix"):
        return scenario.size_mix(n, w["seed"])
    return [(w["L"], w["K"], w["N"])] * n


def run_batch(pa, scenario, torch, name):
    """Many independent instances in one graph-captured batch: evals/s and solves/s."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    G, E, n = w["gens"], w["E"], w["instances"]
    sizes = workload_sizes(scenario, w, n)
    ctx = pa.pa_context_create(0)
    insts, params = [], []
    for i, (L, K, N) in enumerate(sizes):
        d = scenario.make_drop(L, K, seed=w["seed"], instance_id=i)
        insts.append(pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"],
                                           rho=scenario.snr_to_rho(w["snr_db"])))
        params.append(pa.GaParams(pop=N, gens=G, elite=E, p_cross=w["p_cross"], p_mut=w["p_mut"],
                                  kmeans_frac=w["kmeans_frac"], p_init=w["p_init"],
                                  seed=w["seed"], instance_id=i))
    t0 = time.perf_counter()
    pa.pa_solve_batch(ctx, insts, params)  # builds and captures the plan
    plan_s = time.perf_counter() - t0
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = []
    for _ in range(reps):
        res = pa.pa_solve_batch(ctx, insts, params)
        dev.append(res[0].device_ms)
    wall = (time.perf_counter() - t0) / reps
    ev = sum(evals_per_solve(N, E, G) for (_, _, N) in sizes)
    gathers = sum((N + (N - E) * G) * L * L * K for (L, K, N) in sizes)
    out = {"workload": name, "instances": n, "gens": G,
           "sizes": "size_mix: L {7,19,37}, K [4,32], N [128,1024]" if w.get("mix") else
           f"L={sizes[0][0]} K={sizes[0][1]} N={sizes[0][2]}",
           "ms_per_batch": wall * 1e3, "device_ms": float(np.median(dev)),
           "plan_build_s": plan_s,
           "evals_per_s": ev / wall, "solves_per_s": n / wall,
           "lds_gbs": gathers * 4 / wall / 1e9,
           "lds_frac_of_peak": gathers * 4 / wall / 1e9 / LDS_PEAK_GBS,
           "solve_plan": pa.pa_solve_shape(ctx, None)}
    log(f"batch {name}: {wall * 1e3:.1f} ms, {ev / wall:.3e} evals/s, {n / wall:.1f} solves/s, "
        f"LDS {out['lds_gbs']:.0f} GB/s ({100 * out['lds_frac_of_peak']:.1f}%)")
    for inst in insts:
        inst.close()
    return out


def run_serve(pa, scenario, torch, name, seconds, plain_sample):
    """Poisson arrivals of uneven solves through the continuous-batching server:
    solves/s and p50/p99 latency (scheduled arrival -> result on the host),
    beside a FIFO one-instance-at-a-time plain path on the same arrival trace."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    G, E, P = w["gens"], w["E"], w["pool"]
    sizes = scenario.size_mix(P, w["seed"])
    drops = [scenario.make_drop(L, K, seed=w["seed"], instance_id=i)
             for i, (L, K, N) in enumerate(sizes)]
    rho = scenario.snr_to_rho(w["snr_db"])
    arrivals = scenario.poisson_arrivals(w["rate"], seconds, w["seed"])
    n = len(arrivals)

    def params(i):
        return pa.GaParams(pop=sizes[i % P][2], gens=G, elite=E, p_cross=w["p_cross"],
                           p_mut=w["p_mut"], kmeans_frac=w["kmeans_frac"], p_init=w["p_init"],
                           seed=w["seed"] + i, instance_id=i)

    ctx = pa.pa_context_create(0)
    srv = pa.pa_server_create(ctx, max_L=37, max_K=32, max_pop=1024, max_gens=G)
    # warm-up: one request of each size class
    for i in range(min(P, 16)):
        d = drops[i]
        t = pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params(i), T=w["T"], M=w["M"],
                                rho=rho)
        pa.pa_server_poll(srv, t)
    tickets = []
    t_submit = np.zeros(n)
    t0 = time.perf_counter()
    for i in range(n):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        d = drops[i % P]
        t_submit[i] = time.perf_counter() - t0
        tickets.append(pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params(i), T=w["T"],
                                           M=w["M"], rho=rho))
    lat = np.zeros(n)
    for i, t in enumerate(tickets):
        r = pa.pa_server_poll(srv, t)
        lat[i] = (t_submit[i] - arrivals[i]) + r.device_ms * 1e-3
    t_end = time.perf_counter() - t0
    stats = pa.pa_server_stats(srv)
    srv.close()
    done = arrivals + lat
    solves_per_s = n / (done.max() - arrivals[0])
    # plain comparator: measured pa_solve_plain service time of each pool entry,
    # FIFO over the same arrival trace
    svc = np.zeros(P)
    m = min(P, plain_sample)
    for i in range(m):
        d = drops[i]
        inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"], rho=rho)
        pa.pa_solve_plain(inst, params(i))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pa.pa_solve_plain(inst, params(i))
        svc[i] = time.perf_counter() - t1
        inst.close()
    if m < P:
        svc[m:] = np.resize(svc[:m], P - m)
    fin = 0.0
    plat = np.zeros(n)
    for i in range(n):
        fin = max(arrivals[i], fin) + svc[i % P]
        plat[i] = fin - arrivals[i]
    out = {"workload": name, "rate_per_s": w["rate"], "seconds": seconds, "requests": n,
           "gens": G, "sizes": "size_mix: L {7,19,37}, K [4,32], N [128,1024]",
           "solves_per_s": solves_per_s,
           "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "slots": stats["slots"], "ticks": stats["ticks"],
           "plain": {"kind": "FIFO pa_solve_plain, one instance at a time, same arrival trace "
                             "(measured service time per pool entry)",
                     "mean_service_ms": float(svc.mean() * 1e3),
                     "solves_per_s": n / (fin - arrivals[0]) if n else 0.0,
                     "p50_ms": float(np.percentile(plat, 50) * 1e3),
                     "p99_ms": float(np.percentile(plat, 99) * 1e3)}}
    log(f"serve {name}: {n} requests in {t_end:.1f} s, {solves_per_s:.0f} solves/s, "
        f"p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms; plain FIFO: "
        f"{out['plain']['solves_per_s']:.0f} solves/s, p99 {out['plain']['p99_ms']:.0f} ms")
    return out


def run_convergence(pa, scenario, torch, drops, gens):
    """K-means-seeded (kmeans_frac = 0.5) vs randomly initialised (0) GA on the
    same drops (L=19, K=16, N=256, E=8): best sum SE at the end, generations
    until the trace reaches 99% of its final value, and the distribution of
    the final best next to a random pilot assignment (one random chromosome)
    and the K-means seed alone."""
    import numpy as np
    L, K, N, E = 19, 16, 256, 8
    ctx = pa.pa_context_create(0)
    rho = scenario.snr_to_rho(10.0)
    insts, params, rpa, seed_fit = [], [], [], []
    pop = torch.empty((N, L, K), dtype=torch.uint8, device="cuda")
    fit = torch.empty(N, dtype=torch.float32, device="cuda")
    for i in range(drops):
        d = scenario.make_drop(L, K, seed=7, instance_id=i)
        inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=196, M=256, rho=rho)
        for km in (0.5, 0.0):
            insts.append(inst)
            params.append(pa.GaParams(pop=N, gens=gens, elite=E, p_cross=0.8, p_mut=0.05,
                                      kmeans_frac=km, p_init=0.1, seed=100 + i, instance_id=i))
        # slot 0 of a random population: one random assignment; of a K-means
        # population: the seed itself
        for km, dst in ((0.0, rpa), (0.5, seed_fit)):
            pa.pa_kmeans_init(inst, pa.GaParams(pop=N, kmeans_frac=km, seed=100 + i,
                                                instance_id=i), pop)
            pa.pa_fitness(inst, pop, 1, fit)
            torch.cuda.synchronize()
            dst.append(float(fit[0].item()))
    # a batch may hold an instance once: run the two initialisations apart
    res_km = pa.pa_solve_batch(ctx, insts[0::2], params[0::2])
    res_rd = pa.pa_solve_batch(ctx, insts[1::2], params[1::2])

    def to99(tr):
        target = 0.99 * tr[-1]
        return int(np.argmax(tr >= target))

    out = {"workload": f"{drops} drops, L={L} K={K} N={N} G={gens} E={E}, M=256, T=196, SNR 10 dB"}
    for name, res in (("kmeans_init", res_km), ("random_init", res_rd)):
        best = np.array([r.best_fit for r in res])
        g99 = np.array([to99(r.trace) for r in res])
        out[name] = {"best_mean": float(best.mean()),
                     "best_p10_p50_p90": [float(x) for x in np.percentile(best, [10, 50, 90])],
                     "gens_to_99pct_mean": float(g99.mean()),
                     "gens_to_99pct_median": float(np.median(g99)),
                     "initial_best_mean": float(np.mean([r.trace[0] for r in res]))}
    for name, vals in (("random_assignment", rpa), ("kmeans_seed_only", seed_fit)):
        v = np.array(vals)
        out[name] = {"mean": float(v.mean()),
                     "p10_p50_p90": [float(x) for x in np.percentile(v, [10, 50, 90])]}
    g_km = np.array([to99(r.trace) for r in res_km])
    g_rd = np.array([to99(r.trace) for r in res_rd])
    out["kmeans_reaches_99pct_first_frac"] = float(np.mean(g_km < g_rd))
    out["reduction_of_mean_gens_to_99pct"] = float(1.0 - g_km.mean() / max(g_rd.mean(), 1e-9))
    out["kmeans_final_better_frac"] = float(np.mean(
        np.array([r.best_fit for r in res_km]) > np.array([r.best_fit for r in res_rd])))
    return out


def run_fitness(pa, scenario, torch, stream):
    """pa_fitness alone on a resident population: evals/s and LDS roofline."""
    out = []
    for (L, K, n) in ((37, 32, 16384), (19, 16, 65536)):
        d = scenario.make_drop(L, K, seed=1, instance_id=0)
        ctx = pa.pa_context_create(0)
        inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=196)
        pop = torch.empty((n, L, K), dtype=torch.uint8, device="cuda")
        pa.pa_kmeans_init(inst, pa.GaParams(pop=n, kmeans_frac=0.0, seed=3), pop)
        fit = torch.empty(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            pa.pa_fitness(inst, pop, n, fit)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        iters = 20
        e0.record(stream)
        for _ in range(iters):
            pa.pa_fitness(inst, pop, n, fit)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / iters
        gbs = n * L * L * K * 4 / (ms * 1e-3) / 1e9
        TP = max(4, 1 << (K - 1).bit_length())
        out.append({"kernel": f"k_fitness_exact<{L},{TP},0,*>", "L": L, "K": K, "n": n,
                    "avg_launch_us": ms * 1e3, "evals_per_s": n / (ms * 1e-3),
                    "achieved_gbs": gbs, "frac": gbs / LDS_PEAK_GBS})
        log(f"pa_fitness L={L} K={K} n={n}: {ms * 1e3:.1f} us, {n / (ms * 1e-3):.3e} evals/s, "
            f"{gbs:.0f} GB/s LDS ({100 * gbs / LDS_PEAK_GBS:.1f}%)")
        inst.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single_L19_K16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--batch", default="batch64_L37_K32,batch512_mix",
                    help="also time these batched workloads (comma-separated, '' to skip)")
    ap.add_argument("--serve", default="serve_mix_2000rps",
                    help="also run this served workload ('' to skip)")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--plain-sample", type=int, default=64,
                    help="pool entries whose plain service time is measured for the comparator")
    ap.add_argument("--no-fitness", action="store_true", help="skip the pa_fitness roofline lines")
    ap.add_argument("--experiment", default="", choices=["", "convergence"],
                    help="only run this experiment and print its JSON line")
    ap.add_argument("--drops", type=int, default=256)
    ap.add_argument("--exp-gens", type=int, default=200)
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

    if args.experiment == "convergence":
        print(json.dumps({"experiment": "convergence",
                          **run_convergence(pa, scenario, torch, args.drops, args.exp_gens)}),
              flush=True)
        return

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
                "frac": achieved / LDS_PEAK_GBS,
                "traffic": measured_traffic(kname, args.workload, gens_per_launch),
                "avg_launch_us": k_ms * 1e3, "bytes_per_launch": lds_bytes,
                "generations_per_launch": gens_per_launch}
    log(f"generation kernel {kname}: {k_ms * 1e3:.2f} us/launch ({gens_per_launch} generation(s)), "
        f"{achieved:.0f} GB/s LDS ({100 * achieved / LDS_PEAK_GBS:.1f}% of {LDS_PEAK_GBS:.0f})")

    extra = {}
    if not args.no_fitness:
        extra["fitness"] = run_fitness(pa, scenario, torch, stream)
    if args.batch:
        extra["batch"] = [run_batch(pa, scenario, torch, b) for b in args.batch.split(",") if b]
    if args.serve:
        extra["serve"] = run_serve(pa, scenario, torch, args.serve, args.serve_seconds,
                                   args.plain_sample)
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
        line["cpu_baseline"] = cpu_baseline(drop, w, res.best, res.best_fit)
        log(f"oracle: {line['cpu_baseline']['value']:.0f} evals/s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
