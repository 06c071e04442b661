"""Benchmark of the K-means-seeded elitist GA for pilot assignment on one MI355X.

Headline workload: 64 independent instances of L = 37 hexagonal cells,
K = tau = 32 users, M = 256, T = 196, each with its own user drop, a
population of 1024, 200 generations and 8 elites, solved together by
pa_solve_batch (one generation launch per generation, captured in a
hipGraph).  A step is one whole batch (K-means seeding, initial fitness,
200 generations of elitism / selection / crossover / mutation / fitness, the
best chromosome of every instance back on the host); `value` is chromosome
fitness evaluations per second, sum over instances of N + (N - E) * G per
batch, over the timed batches, inputs resident in HBM.

Also measured (extra keys): the peak LDS and VALU rates of the device
(probe kernels), pa_fitness alone, the single L=19 / K=16 and L=7 / K=4
solves, the 512-instance uneven batch with each instance's FP32-vs-FP64
error, the Poisson-arrival server run and the plain one-launch-per-step path
on the same arrivals, and the oracle on the host cores.

Prints ONE JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LDS_NOMINAL_B_PER_CLK = 128  # 32 banks x 4 bytes per clock and CU (ds_read_b32)


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


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter passes, or None
    when they were taken for another kernel, workload or source version."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    for rec in recs:
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("source_sha256") == source_sha256()):
            return float(rec["bytes_per_launch"])
    return None


def evals_per_solve(N, E, G):
    return N + (N - E) * G


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


# ---- the oracle on the host (never touches the GPU) --------------------------

def oracle_sample(L, K, N, G, E, seed, inst, T):
    """Child-process mode: one oracle solve of instance `inst` of a workload with
    G generations; prints {"evals": .., "seconds": ..}."""
    import oracle
    from paper_2511_20511_amd import scenario
    oracle.build(force=False)
    d = scenario.make_drop(L, K, seed=seed, instance_id=inst)
    t0 = time.perf_counter()
    oracle.solve(d.beta, d.user_xy, d.bs_xy, N, G, E, 0.8, 0.05, 0.5, 0.1, seed, inst, T=T)
    el = time.perf_counter() - t0
    print(json.dumps({"evals": evals_per_solve(N, E, G), "seconds": el}), flush=True)


def cpu_baseline(w, sample_gens, procs):
    """The FP64 oracle (single-threaded C, as written) on a bounded sample of
    the headline workload: instance 0 with `sample_gens` generations on one
    core, then `procs` independent processes, one instance each, at once.
    Run before the GPU is touched; children are fresh interpreters."""
    import oracle
    oracle.build(force=False)
    args = lambda i: [sys.executable, os.path.abspath(__file__), "--oracle-sample",
                      ",".join(str(x) for x in (w["L"], w["K"], w["N"], sample_gens, w["E"],
                                                w["seed"], i, w["T"]))]
    one = json.loads(subprocess.run(args(0), capture_output=True, text=True, check=True).stdout)
    single = one["evals"] / one["seconds"]
    t0 = time.perf_counter()
    ps = [subprocess.Popen(args(i), stdout=subprocess.PIPE, text=True) for i in range(procs)]
    outs = [json.loads(p.communicate()[0]) for p in ps]
    wall = time.perf_counter() - t0
    multi = sum(o["evals"] for o in outs) / wall
    return {"value": single, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": (f"instance 0 of {w['instances']} x (L={w['L']} K={w['K']} N={w['N']} "
                       f"E={w['E']}), K-means init + {sample_gens} generations, FP64, one "
                       f"thread: {one['evals']} evaluations in {one['seconds']:.1f} s (the "
                       f"workload's rate per evaluation; its full batch is "
                       f"{w['instances'] * evals_per_solve(w['N'], w['E'], w['gens'])} "
                       f"evaluations)"),
            "cpu_model": cpu_model(), "nproc": usable_cores(),
            "multicore": {"value": multi, "unit": "evals/s", "cores": procs,
                          "sample": f"{procs} oracle processes at once, instances 0..{procs - 1}, "
                                    f"same sample each, {wall:.1f} s wall"}}


def oracle_full_and_service(scenario, procs, n_requests=16):
    """The oracle on the two small single instances in full (one core each), and
    its service time on the first n_requests of the serving mix (G = 50), one
    single-threaded process per request, `procs` at a time: the distribution,
    and the cores that the serving rate would need at that mean."""
    def run(L, K, N, G, E, seed, inst, T):
        return [sys.executable, os.path.abspath(__file__), "--oracle-sample",
                ",".join(str(x) for x in (L, K, N, G, E, seed, inst, T))]
    full = {}
    for name in ("single_L7_K4", "single_L19_K16"):
        w = scenario.WORKLOADS[name]
        o = json.loads(subprocess.run(run(w["L"], w["K"], w["N"], w["gens"], w["E"], w["seed"], 0,
                                          w["T"]), capture_output=True, text=True,
                                      check=True).stdout)
        full[name] = {"solve_s": o["seconds"], "evals": o["evals"],
                      "evals_per_s": o["evals"] / o["seconds"], "cores": 1}
    w = scenario.WORKLOADS["serve_mix_2000rps"]
    sizes = scenario.size_mix(w["pool"], w["seed"])[:n_requests]
    secs = []
    for i0 in range(0, len(sizes), procs):
        ps = [subprocess.Popen(run(L, K, N, w["gens"], w["E"], w["seed"], i0 + j, w["T"]),
                               stdout=subprocess.PIPE, text=True)
              for j, (L, K, N) in enumerate(sizes[i0:i0 + procs])]
        secs += [json.loads(p.communicate()[0])["seconds"] for p in ps]
    a = sorted(secs)
    mean = sum(a) / len(a)
    q = lambda f: a[min(len(a) - 1, int(f * len(a)))]
    service = {"requests": len(a), "gens": w["gens"], "mean_s": mean, "p50_s": q(0.5),
               "p90_s": q(0.9), "max_s": a[-1], "rate_per_s": w["rate"],
               "cores_for_rate": w["rate"] * mean,
               "sample": (f"the first {len(a)} drops of the serving pool (size mix), one "
                          f"single-threaded oracle process per request, {procs} at a time")}
    return full, service


# ---- GPU measurements ---------------------------------------------------------

def make_batch(pa, scenario, ctx, w, sizes):
    insts, params, drops = [], [], []
    for i, (L, K, N) in enumerate(sizes):
        d = scenario.make_drop(L, K, seed=w["seed"], instance_id=i)
        insts.append(pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"],
                                           rho=scenario.snr_to_rho(w["snr_db"])))
        params.append(pa.GaParams(pop=N, gens=w["gens"], elite=w["E"], p_cross=w["p_cross"],
                                  p_mut=w["p_mut"], kmeans_frac=w["kmeans_frac"],
                                  p_init=w["p_init"], seed=w["seed"], instance_id=i))
        drops.append(d)
    return insts, params, drops


def workload_sizes(scenario, w):
    if w.get("mix"):
        return scenario.size_mix(w["instances"], w["seed"])
    return [(w["L"], w["K"], w["N"])] * w["instances"]


def lds_peak(peaks, kind):
    """Measured peak LDS bytes/s of the device for ds_read_b32 or ds_read_b128."""
    return peaks[kind] * peaks["cus"] * peaks["clock_mhz"] * 1e6


def kernel_roofline(pa, torch, ctx, insts, params, w, peaks, launches, workload):
    """The batch's generation kernel alone: stepwise batch, HIP events around
    `launches` generation launches on the stream they run on."""
    stream = torch.cuda.current_stream()
    pa.pa_solve_batch_begin(ctx, insts, params)
    pa.pa_solve_batch_next(ctx, 5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pa.pa_solve_batch_next(ctx, launches)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / launches
    shape = pa.pa_solve_shape(ctx, None)
    L, K = w["L"], w["K"]
    TP = max(4, 1 << (K - 1).bit_length())
    kname = f"k_gen_exact<{L},{TP},0,{shape['block']}>"
    per_child = 4 * L * L * K  # algorithmic LDS bytes: one table word per (BS, cell, pilot)
    children = w["instances"] * (w["N"] - w["E"])
    bytes_launch = per_child * children
    achieved = bytes_launch / (us * 1e-6) / 1e9
    peak = lds_peak(peaks, "lds_b32") / 1e9
    nominal = LDS_NOMINAL_B_PER_CLK * peaks["cus"] * peaks["clock_mhz"] * 1e6 / 1e9
    return {"bound": "lds", "kernel": kname, "instruction": "ds_read_b32",
            "achieved": achieved, "peak": peak, "unit": "GB/s", "frac": achieved / peak,
            "traffic": measured_traffic(kname, workload),
            "peak_source": "measured conflict-free ds_read_b32 rate (pa_device_peaks)",
            "peak_nominal": nominal, "frac_of_nominal": achieved / nominal,
            "avg_launch_us": us, "launches_timed": launches,
            "algorithmic_bytes_per_launch": bytes_launch,
            "per_unit": f"{per_child} B of LDS reads per child (4 L^2 K), "
                        f"{children} children per launch"}


def run_batch_extra(pa, scenario, torch, oracle_mod, name, reps=3):
    """A batched workload timed end to end; with oracle_mod, the FP64 error of
    every instance's best FP32 fitness."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    sizes = workload_sizes(scenario, w)
    ctx = pa.pa_context_create(0)
    insts, params, drops = make_batch(pa, scenario, ctx, w, sizes)
    t0 = time.perf_counter()
    res = pa.pa_solve_batch(ctx, insts, params)
    plan_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = pa.pa_solve_batch(ctx, insts, params)
    wall = (time.perf_counter() - t0) / reps
    G, E = w["gens"], w["E"]
    ev = sum(evals_per_solve(N, E, G) for (_, _, N) in sizes)
    out = {"workload": name, "instances": len(sizes), "gens": G,
           "sizes": "size_mix: L {7,19,37}, K [4,32], N [128,1024]" if w.get("mix") else
           f"L={sizes[0][0]} K={sizes[0][1]} N={sizes[0][2]}",
           "ms_per_batch": wall * 1e3, "device_ms": res[0].device_ms, "plan_build_s": plan_s,
           "evals_per_s": ev / wall, "solves_per_s": len(sizes) / wall,
           "solve_plan": pa.pa_solve_shape(ctx, None)}
    if oracle_mod is not None:
        errs = []
        for i, r in enumerate(res):
            want = float(oracle_mod.fitness(drops[i].beta, r.best[None], T=w["T"])[0])
            errs.append(abs(r.best_fit - want) / abs(want))
        errs = np.array(errs)
        out["best_fp32_vs_fp64_rel_err"] = {"max": float(errs.max()),
                                            "p99": float(np.percentile(errs, 99)),
                                            "median": float(np.median(errs)),
                                            "instances": len(errs), "tolerance": 1e-5}
    log(f"batch {name}: {wall * 1e3:.1f} ms, {ev / wall:.3e} evals/s, "
        f"{len(sizes) / wall:.1f} solves/s")
    for inst in insts:
        inst.close()
    ctx.close()
    return out


def run_single(pa, scenario, torch, name, steps, peaks):
    """A single-instance solve (pa_solve): latency, and for the persistent form
    its one launch timed with events (all generations)."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    L, K, N, G, E = w["L"], w["K"], w["N"], w["gens"], w["E"]
    ctx = pa.pa_context_create(0)
    d = scenario.make_drop(L, K, seed=w["seed"], instance_id=0)
    inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"],
                                 rho=scenario.snr_to_rho(w["snr_db"]))
    p = pa.GaParams(pop=N, gens=G, elite=E, p_cross=w["p_cross"], p_mut=w["p_mut"],
                    kmeans_frac=w["kmeans_frac"], p_init=w["p_init"], seed=w["seed"],
                    instance_id=0)
    for _ in range(2):
        pa.pa_solve(inst, p)
    torch.cuda.synchronize()
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        r = pa.pa_solve(inst, p)
        lat.append(time.perf_counter() - t0)
    dev = r.device_ms
    pa.pa_solve_plain(inst, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, steps // 2)):
        pa.pa_solve_plain(inst, p)
    plain_ms = (time.perf_counter() - t0) * 1e3 / max(1, steps // 2)
    shape = pa.pa_solve_shape(None, inst)
    out = {"workload": name, "L": L, "K": K, "pop": N, "gens": G, "elite": E,
           "solve_ms_median": float(np.median(lat) * 1e3), "solve_ms_min": float(min(lat) * 1e3),
           "solve_device_ms": dev, "evals_per_s": evals_per_solve(N, E, G) / np.median(lat),
           "plain_solve_ms": plain_ms, "solve_plan": shape}
    if shape["persistent"]:
        stream = torch.cuda.current_stream()
        TP = max(4, 1 << (K - 1).bit_length())
        form = "k_gen_wg" if shape["persistent"] == 2 else "k_gen_persist"
        kname = f"{form}<{L},{TP},0,{shape['block']}>"
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pa.pa_solve_begin(inst, p)
        e0.record(stream)
        pa.pa_solve_next(inst, G)
        e1.record(stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3
        b = (N - E) * G * 4 * L * L * K
        out["generation_kernel"] = {"kernel": kname, "avg_launch_us": us,
                                    "generations_per_launch": G,
                                    "lds_gbs": b / (us * 1e-6) / 1e9,
                                    "frac_of_measured_b32": b / (us * 1e-6) / lds_peak(peaks, "lds_b32")}
    log(f"single {name}: {out['solve_ms_median']:.3f} ms per solve (device {dev:.3f} ms), "
        f"plain {plain_ms:.3f} ms, plan {shape}")
    inst.close()
    ctx.close()
    return out


def run_fitness(pa, scenario, torch, peaks):
    """pa_fitness alone on a resident population of 65,536 chromosomes (the
    64 x 1024 a generation of the L=37 batch evaluates): evals/s and LDS
    roofline against the measured peak of the instruction each layout issues."""
    out = []
    stream = torch.cuda.current_stream()
    for (L, K, n, instr) in ((37, 32, 65536, "lds_b32"), (19, 16, 65536, "lds_b128")):
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
        peak = lds_peak(peaks, instr) / 1e9
        TP = max(4, 1 << (K - 1).bit_length())
        out.append({"kernel": f"k_fitness_exact<{L},{TP},0,*>", "L": L, "K": K, "n": n,
                    "instruction": "ds_read_b32" if instr == "lds_b32" else "ds_read_b128",
                    "avg_launch_us": ms * 1e3, "evals_per_s": n / (ms * 1e-3),
                    "achieved_gbs": gbs, "peak_gbs": peak, "frac": gbs / peak})
        log(f"pa_fitness L={L} K={K} n={n}: {ms * 1e3:.1f} us, {n / (ms * 1e-3):.3e} evals/s, "
            f"{gbs:.0f} GB/s LDS ({100 * gbs / peak:.1f}% of the measured {instr} peak)")
        inst.close()
        ctx.close()
    return out


def run_objectives(pa, scenario, torch, oracle_mod):
    """pa_fitness of one resident population (L=19, K=16, n=65536) under each
    objective: sum SE (Eq. 7), max-min SIR, Eq. 8; FP32 against FP64 on a sample."""
    import numpy as np
    out = []
    stream = torch.cuda.current_stream()
    L, K, n = 19, 16, 65536
    d = scenario.make_drop(L, K, seed=1, instance_id=0)
    ctx = pa.pa_context_create(0)
    for obj, name in ((pa.OBJ_SUM_SE, "sum_se"), (pa.OBJ_MIN_SINR, "min_sinr"),
                      (pa.OBJ_INTERCLUSTER, "eq8_intercluster")):
        inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=196, objective=obj)
        pop = torch.empty((n, L, K), dtype=torch.uint8, device="cuda")
        pa.pa_kmeans_init(inst, pa.GaParams(pop=n, kmeans_frac=0.0, seed=3), pop)
        fit = torch.empty(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            pa.pa_fitness(inst, pop, n, fit)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            pa.pa_fitness(inst, pop, n, fit)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 20
        got = fit[:256].cpu().numpy().astype(np.float64)
        want = oracle_mod.fitness(d.beta, pop[:256].cpu().numpy(), T=196, objective=obj)
        out.append({"objective": name, "L": L, "K": K, "n": n, "avg_launch_us": ms * 1e3,
                    "evals_per_s": n / (ms * 1e-3),
                    "fp32_vs_fp64_rel_err_max": float(np.max(np.abs(got - want) / np.abs(want)))})
        log(f"objective {name}: {ms * 1e3:.1f} us per launch of {n}")
        inst.close()
    ctx.close()
    return out


def run_island(pa, scenario, torch, oracle_mod, name="single_L19_K16", clusters=5, every=3,
               reps=5):
    """The PK-means GA (Alg. 2; C = 5 islands re-clustered every 3 generations,
    Sec. 6.1) on one instance beside the panmictic solve of the same parameters."""
    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    L, K, N, G, E = w["L"], w["K"], w["N"], w["gens"], w["E"]
    ctx = pa.pa_context_create(0)
    d = scenario.make_drop(L, K, seed=w["seed"], instance_id=0)
    inst = pa.pa_instance_create(ctx, d.beta, d.user_xy, d.bs_xy, T=w["T"], M=w["M"],
                                 rho=scenario.snr_to_rho(w["snr_db"]))
    p = pa.GaParams(pop=N, gens=G, elite=E, p_cross=w["p_cross"], p_mut=w["p_mut"],
                    kmeans_frac=w["kmeans_frac"], p_init=w["p_init"], seed=w["seed"],
                    instance_id=0)
    res, _ = pa.pa_island_solve(inst, p, clusters, every)
    torch.cuda.synchronize()
    lat, dev = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        res, labels = pa.pa_island_solve(inst, p, clusters, every)
        lat.append(time.perf_counter() - t0)
        dev.append(res.device_ms)
    pan = pa.pa_solve(inst, p)
    want = float(oracle_mod.fitness(d.beta, res.best[None], T=w["T"])[0])
    counts = np.bincount(labels, minlength=clusters)
    out = {"workload": name, "clusters": clusters, "recluster_every": every,
           "solve_ms_median": float(np.median(lat) * 1e3), "solve_device_ms": float(np.median(dev)),
           "best_fit": float(res.best_fit), "panmictic_best_fit": float(pan.best_fit),
           "best_fp32_vs_fp64_rel_err": abs(res.best_fit - want) / abs(want),
           "last_island_sizes": [int(x) for x in counts]}
    log(f"island GA {name} C={clusters} R={every}: {out['solve_ms_median']:.2f} ms per solve, "
        f"best {res.best_fit:.2f} (panmictic {pan.best_fit:.2f})")
    inst.close()
    ctx.close()
    return out


def run_serve(pa, scenario, torch, name, warm_s, seconds, plain_s):
    """Poisson arrivals of uneven solves through the continuous-batching server
    (warm-up, then the measured window): solves/s and p50/p99 latency
    (scheduled arrival -> result on the host); then the plain path
    (pa_solve_plain, one request at a time, FIFO) run on the first `plain_s`
    seconds of the same arrival trace."""
    import threading

    import numpy as np
    w = dict(scenario.WORKLOADS[name])
    G, E, P = w["gens"], w["E"], w["pool"]
    sizes = scenario.size_mix(P, w["seed"])
    drops = [scenario.make_drop(L, K, seed=w["seed"], instance_id=i)
             for i, (L, K, N) in enumerate(sizes)]
    rho = scenario.snr_to_rho(w["snr_db"])
    arrivals = scenario.poisson_arrivals(w["rate"], warm_s + seconds, w["seed"])
    n = len(arrivals)

    def params(i):
        return pa.GaParams(pop=sizes[i % P][2], gens=G, elite=E, p_cross=w["p_cross"],
                           p_mut=w["p_mut"], kmeans_frac=w["kmeans_frac"], p_init=w["p_init"],
                           seed=w["seed"] + i, instance_id=i)

    ctx = pa.pa_context_create(0)
    srv = pa.pa_server_create(ctx, max_L=37, max_K=32, max_pop=1024, max_gens=G)
    tickets = [None] * n
    t_submit = np.zeros(n)
    lat = np.zeros(n)
    done_at = np.zeros(n)
    t0 = time.perf_counter()

    def poller():
        for i in range(n):
            while tickets[i] is None:
                time.sleep(0.0002)
            r = pa.pa_server_poll(srv, tickets[i])
            lat[i] = (t_submit[i] - arrivals[i]) + r.device_ms * 1e-3
            done_at[i] = arrivals[i] + lat[i]

    th = threading.Thread(target=poller)
    th.start()
    for i in range(n):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        d = drops[i % P]
        t_submit[i] = time.perf_counter() - t0
        tickets[i] = pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params(i), T=w["T"],
                                         M=w["M"], rho=rho)
    th.join()
    stats = pa.pa_server_stats(srv)
    srv.close()
    m = arrivals >= warm_s
    lm = lat[m]
    span = done_at[m].max() - arrivals[m][0]
    out = {"workload": name, "rate_per_s": w["rate"], "warmup_s": warm_s, "seconds": seconds,
           "requests_measured": int(m.sum()), "gens": G,
           "sizes": "size_mix: L {7,19,37}, K [4,32], N [128,1024]",
           "solves_per_s": float(m.sum() / span),
           "p50_ms": float(np.percentile(lm, 50) * 1e3),
           "p99_ms": float(np.percentile(lm, 99) * 1e3),
           "slots": stats["slots"], "ticks": stats["ticks"]}
    log(f"serve {name}: {int(m.sum())} requests measured, {out['solves_per_s']:.0f} solves/s, "
        f"p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms")
    # plain path on the same trace (prefix), measured: one request at a time;
    # each pool entry's instance is created (uploaded) once, before the run
    insts = {i: pa.pa_instance_create(ctx, drops[i].beta, drops[i].user_xy, drops[i].bs_xy,
                                      T=w["T"], M=w["M"], rho=rho) for i in range(P)}
    np_ = int(np.searchsorted(arrivals, plain_s))
    plat = np.zeros(np_)
    pdone = np.zeros(np_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(np_):
        now = time.perf_counter() - t0
        if now < arrivals[i]:
            while time.perf_counter() - t0 < arrivals[i]:
                pass
        pa.pa_solve_plain(insts[i % P], params(i))
        pdone[i] = time.perf_counter() - t0
        plat[i] = pdone[i] - arrivals[i]
    for inst in insts.values():
        inst.close()
    ctx.close()
    out["plain"] = {"kind": "pa_solve_plain one request at a time (FIFO, one stream, no graph, "
                            "no batching), run on the first "
                            f"{plain_s:.0f} s of the same arrival trace",
                    "requests": np_,
                    "solves_per_s": float(np_ / (pdone[-1] - arrivals[0])) if np_ else 0.0,
                    "p50_ms": float(np.percentile(plat, 50) * 1e3) if np_ else 0.0,
                    "p99_ms": float(np.percentile(plat, 99) * 1e3) if np_ else 0.0}
    log(f"plain on the first {plain_s:.0f} s: {np_} requests, "
        f"{out['plain']['solves_per_s']:.0f} solves/s, p99 {out['plain']['p99_ms']:.0f} ms")
    return out


def run_convergence(pa, scenario, torch, drops, gens, keep=None):
    """K-means-seeded (kmeans_frac = 0.5) vs randomly initialised (0) GA on the
    same drops (L=19, K=16, N=256, E=8): best sum SE at the end, generations
    and wall time until the trace reaches 99% of its final value, the whole
    distribution of the final best, and a random pilot assignment (one random
    chromosome) and the K-means seed alone."""
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
        for km, dst in ((0.0, rpa), (0.5, seed_fit)):
            pa.pa_kmeans_init(inst, pa.GaParams(pop=N, kmeans_frac=km, seed=100 + i,
                                                instance_id=i), pop)
            pa.pa_fitness(inst, pop, 1, fit)
            torch.cuda.synchronize()
            dst.append(float(fit[0].item()))
    # wall time per generation of one solve (the single-instance persistent
    # form, stepwise): time to 99% = init + generations x per-generation time
    one = insts[0]
    pa.pa_solve(one, params[0])
    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    pa.pa_solve_begin(one, params[0])
    e1.record(stream)
    pa.pa_solve_next(one, gens)
    e2.record(stream)
    e2.synchronize()
    init_ms = e0.elapsed_time(e1)
    gen_ms = e1.elapsed_time(e2) / gens
    res_km = pa.pa_solve_batch(ctx, insts[0::2], params[0::2])
    res_rd = pa.pa_solve_batch(ctx, insts[1::2], params[1::2])

    def to99(tr):
        return int(np.argmax(tr >= 0.99 * tr[-1]))

    out = {"workload": f"{drops} drops, L={L} K={K} N={N} G={gens} E={E}, M=256, T=196, SNR 10 dB",
           "solve_init_ms": init_ms, "solve_ms_per_generation": gen_ms}
    for name, res in (("kmeans_init", res_km), ("random_init", res_rd)):
        best = np.array([r.best_fit for r in res])
        g99 = np.array([to99(r.trace) for r in res])
        out[name] = {"best_mean": float(best.mean()),
                     "best_quantiles_0_5_10_25_50_75_90_95_100": [
                         float(x) for x in np.percentile(best, [0, 5, 10, 25, 50, 75, 90, 95, 100])],
                     "gens_to_99pct_mean": float(g99.mean()),
                     "gens_to_99pct_median": float(np.median(g99)),
                     "ms_to_99pct_mean": float(init_ms + g99.mean() * gen_ms),
                     "initial_best_mean": float(np.mean([r.trace[0] for r in res])),
                     "best": [float(x) for x in best]}
    for name, vals in (("random_assignment", rpa), ("kmeans_seed_only", seed_fit)):
        v = np.array(vals)
        out[name] = {"mean": float(v.mean()),
                     "quantiles_0_5_10_25_50_75_90_95_100": [
                         float(x) for x in np.percentile(v, [0, 5, 10, 25, 50, 75, 90, 95, 100])],
                     "values": [float(x) for x in v]}
    g_km = np.array([to99(r.trace) for r in res_km])
    g_rd = np.array([to99(r.trace) for r in res_rd])
    out["kmeans_reaches_99pct_first_frac"] = float(np.mean(g_km < g_rd))
    out["reduction_of_mean_gens_to_99pct"] = float(1.0 - g_km.mean() / max(g_rd.mean(), 1e-9))
    out["kmeans_final_better_frac"] = float(np.mean(
        np.array([r.best_fit for r in res_km]) > np.array([r.best_fit for r in res_rd])))
    if keep is not None:  # the solves themselves, for checks against the oracle
        keep.update(kmeans_init=res_km, random_init=res_rd, params=params)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch64_L37_K32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-gens", type=int, default=100)
    ap.add_argument("--kernel-launches", type=int, default=100)
    ap.add_argument("--batch", default="batch512_mix",
                    help="also time these batched workloads (comma-separated, '' to skip)")
    ap.add_argument("--single", default="single_L19_K16,single_L7_K4",
                    help="also time these single-instance solves ('' to skip)")
    ap.add_argument("--serve", default="serve_mix_2000rps",
                    help="also run this served workload ('' to skip)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--plain-seconds", type=float, default=3.0,
                    help="the plain path runs on this prefix of the arrival trace")
    ap.add_argument("--no-fitness", action="store_true", help="skip the pa_fitness roofline lines")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the objectives and island GA lines")
    ap.add_argument("--experiment", default="", choices=["", "convergence"],
                    help="only run this experiment and print its JSON line")
    ap.add_argument("--drops", type=int, default=256)
    ap.add_argument("--exp-gens", type=int, default=200)
    ap.add_argument("--oracle-sample", default="", help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (5 times) and exit: the "
                         "reference kernel that scales HBM byte counters")
    args = ap.parse_args()
    if args.oracle_sample:
        v = [int(x) for x in args.oracle_sample.split(",")]
        oracle_sample(*v)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(each instance runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2511_20511_amd import scenario
    w = dict(scenario.WORKLOADS[args.workload])
    cpu = None
    if not args.no_cpu_baseline and not args.experiment and not args.calibrate_copy:
        procs = min(usable_cores(), 16)
        log(f"cpu baseline: oracle sample on 1 core, then {procs} processes ...")
        cpu = cpu_baseline(w, args.cpu_sample_gens, procs)
        log(f"oracle: {cpu['value']:.0f} evals/s on one core, "
            f"{cpu['multicore']['value']:.0f} evals/s on {procs}")
        cpu["full_solves"], cpu["serve_service_time"] = oracle_full_and_service(scenario, procs)
        sv = cpu["serve_service_time"]
        log(f"oracle full solves: " + ", ".join(f"{k} {v['solve_s']:.2f} s"
                                              for k, v in cpu["full_solves"].items())
            + f"; serving mix service time mean {sv['mean_s']:.2f} s, p90 {sv['p90_s']:.2f} s "
            f"({sv['cores_for_rate']:.0f} cores for {sv['rate_per_s']:.0f} req/s)")

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

    if args.experiment == "convergence":
        print(json.dumps({"experiment": "convergence",
                          **run_convergence(pa, scenario, torch, args.drops, args.exp_gens)}),
              flush=True)
        return

    ctx = pa.pa_context_create(0)
    peaks = pa.pa_device_peaks(ctx)
    log(f"device peaks: {peaks}")
    sizes = workload_sizes(scenario, w)
    insts, params, drops = make_batch(pa, scenario, ctx, w, sizes)
    log(f"workload {args.workload}: {len(sizes)} instances, sizes {sizes[0]}, G={w['gens']}")
    t0 = time.perf_counter()
    pa.pa_solve_batch(ctx, insts, params)  # builds and captures the plan
    plan_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        pa.pa_solve_batch(ctx, insts, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    res = None
    for _ in range(args.steps):
        res = pa.pa_solve_batch(ctx, insts, params)
        dev_ms.append(res[0].device_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    ev = sum(evals_per_solve(N, w["E"], w["gens"]) for (_, _, N) in sizes)
    value = ev * args.steps / wall
    shape = pa.pa_solve_shape(ctx, None)
    log(f"batch: {ms_per_step:.2f} ms per batch, device {np.median(dev_ms):.2f} ms, "
        f"{value:.3e} evals/s, plan {shape}")
    roofline = kernel_roofline(pa, torch, ctx, insts, params, w, peaks, args.kernel_launches,
                               args.workload)
    log(f"generation kernel {roofline['kernel']}: {roofline['avg_launch_us']:.1f} us/launch, "
        f"{roofline['achieved']:.0f} GB/s LDS = {100 * roofline['frac']:.1f}% of the measured "
        f"ds_read_b32 peak ({100 * roofline['frac_of_nominal']:.1f}% of nominal)")
    # the FP32 best of every instance against the FP64 definition
    import oracle
    oracle.build(force=False)
    want = [float(oracle.fitness(d.beta, r.best[None], T=w["T"])[0]) for r, d in zip(res, drops)]
    errs = [abs(r.best_fit - f) / abs(f) for r, f in zip(res, want)]
    for inst in insts:
        inst.close()

    line = {
        "metric": "chromosome fitness evals/s", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "instances": len(sizes), "L": w.get("L"),
                   "K": w.get("K"), "tau": w.get("K"), "M": w["M"], "T": w["T"],
                   "pop": w.get("N"), "gens": w["gens"], "elite": w["E"],
                   "evals_per_step": ev},
        "solves_per_s": len(sizes) * args.steps / wall,
        "batch_device_ms": float(np.median(dev_ms)),
        "plan_build_s": plan_s,
        "solve_plan": shape,
        "best_fp32_vs_fp64_rel_err_max": float(max(errs)),
        "roofline": roofline,
        "device_peaks": peaks,
    }
    if args.single:
        line["single"] = [run_single(pa, scenario, torch, s, args.steps, peaks)
                          for s in args.single.split(",") if s]
    if not args.no_fitness:
        line["fitness"] = run_fitness(pa, scenario, torch, peaks)
    if not args.no_next:
        line["objectives"] = run_objectives(pa, scenario, torch, oracle)
        line["island"] = run_island(pa, scenario, torch, oracle)
    if args.batch:
        line["batch"] = [run_batch_extra(pa, scenario, torch, oracle, b)
                         for b in args.batch.split(",") if b]
    if args.serve:
        line["serve"] = run_serve(pa, scenario, torch, args.serve, args.serve_warmup,
                                  args.serve_seconds, args.plain_seconds)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
