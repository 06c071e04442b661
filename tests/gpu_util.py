"""Helpers shared by the GPU tests: device setup and seeded inputs."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


_CTX = {}


def ctx():
    import paper_2511_20511_amd as pa
    if "ctx" not in _CTX:
        _CTX["ctx"] = pa.pa_context_create(0)
    return _CTX["ctx"]


def rand_pop(rng, n, L, K):
    """n chromosomes with uniformly random permutation rows."""
    keys = rng.random((n, L, K))
    return np.argsort(keys, axis=2).astype(np.uint8)


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return np.abs(got - want) / np.maximum(np.abs(want), 1e-300)


def flush(msg):
    print(msg, flush=True)


def lockstep(pa, oracle_mod, torch, drop, inst, params, T=196):
    """Alg. 1 generation by generation with the oracle's operators fed the
    GPU's FP32 fitness of each population (pa_fitness): returns the last
    population, its FP32 fitness, the trace of best FP32 fitness per
    generation and the worst relative error of the FP32 fitness against the
    oracle's FP64 value."""
    L, K, N = drop.L, drop.K, params.pop
    seed = (oracle_mod.kmeans_seed(drop.user_xy, drop.bs_xy)[0]
            if params.kmeans_frac > 0 else None)
    pop = oracle_mod.init_pop(L, K, N, params.kmeans_frac, params.p_init, params.seed,
                              params.instance_id, seed)
    d_pop = torch.empty((N, L, K), dtype=torch.uint8, device="cuda")
    d_fit = torch.empty(N, dtype=torch.float32, device="cuda")
    worst = 0.0
    trace = []
    for g in range(params.gens + 1):
        d_pop.copy_(torch.from_numpy(pop))
        pa.pa_fitness(inst, d_pop, N, d_fit)
        torch.cuda.synchronize()
        fit = d_fit.cpu().numpy()
        want = oracle_mod.fitness(drop.beta, pop, T=T)
        worst = max(worst, float(rel_err(fit, want).max()))
        trace.append(fit[oracle_mod.rank(fit.astype(np.float64))[0]])
        if g == params.gens:
            break
        pop = oracle_mod.ga_step(pop, fit.astype(np.float64), params.elite, params.p_cross,
                                 params.p_mut, params.seed, params.instance_id, g)
    return pop, fit, np.array(trace, dtype=np.float32), worst
