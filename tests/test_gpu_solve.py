"""GPU solve against the oracle, generation by generation (lockstep).

At every generation the GPU's FP32 fitness must lie within 1e-5 of the
oracle's FP64 fitness of the same population, and the oracle's ga_step, fed
the GPU's FP32 fitness, must reproduce the GPU's next population exactly.
pa_solve and pa_solve_plain must return the best chromosome, fitness and
trace of that same trajectory, bit for bit."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu, rel_err
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu


def _trajectory(pa, oracle_mod, torch, drop, inst, params, T, se_mode=0, M=1, rho=1.0):
    N, L, K = params.pop, drop.L, drop.K
    d_pop = torch.zeros((N, L, K), dtype=torch.uint8, device="cuda")
    d_next = torch.zeros_like(d_pop)
    d_fit = torch.zeros(N, dtype=torch.float32, device="cuda")
    pa.pa_kmeans_init(inst, params, d_pop)
    trace = []
    worst = 0.0
    for g in range(params.gens + 1):
        pa.pa_fitness(inst, d_pop, N, d_fit)
        torch.cuda.synchronize()
        pop = d_pop.cpu().numpy()
        fit = d_fit.cpu().numpy()
        want = oracle_mod.fitness(drop.beta, pop, T=T, se_mode=se_mode, M=M, rho=rho)
        worst = max(worst, rel_err(fit, want).max())
        trace.append(fit[oracle_mod.rank(fit.astype(np.float64))[0]])
        if g == params.gens:
            break
        pa.pa_ga_step(inst, params, g, d_pop, d_fit, d_next)
        torch.cuda.synchronize()
        nxt = oracle_mod.ga_step(pop, fit.astype(np.float64), params.elite, params.p_cross,
                                 params.p_mut, params.seed, params.instance_id, g)
        assert np.array_equal(d_next.cpu().numpy(), nxt), f"generation {g} differs"
        d_pop, d_next = d_next, d_pop
    best = oracle_mod.rank(fit.astype(np.float64))[0]
    return pop[best], fit[best], best, np.array(trace, dtype=np.float32), worst


@pytest.mark.parametrize("L,K,N,G,E,se_mode", [(7, 4, 50, 100, 2, 0), (19, 16, 256, 12, 8, 0),
                                               (7, 5, 31, 10, 3, 1), (37, 32, 64, 3, 8, 0),
                                               (3, 3, 20, 15, 0, 0)])
def test_solve_lockstep(oracle_mod, L, K, N, G, E, se_mode):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"solve lockstep L={L} K={K} N={N} G={G} mode={se_mode}")
    drop = scenario.make_drop(L, K, seed=1, instance_id=0)
    rho = scenario.snr_to_rho(10.0)
    M = 128
    inst = pa.pa_instance_create(ctx(), drop.beta, drop.user_xy, drop.bs_xy, T=196, M=M,
                                 rho=rho, se_mode=se_mode)
    params = pa.GaParams(pop=N, gens=G, elite=E, p_cross=0.8, p_mut=0.05, kmeans_frac=0.5,
                         p_init=0.1, seed=1, instance_id=0)
    best, bf, bi, trace, worst = _trajectory(pa, oracle_mod, torch, drop, inst, params, 196,
                                             se_mode, M, rho)
    flush(f"  worst fitness rel err {worst:.3e}, best {bf:.6f}")
    assert worst <= 1e-5
    for fn in (pa.pa_solve, pa.pa_solve_plain):
        r = fn(inst, params)
        assert np.array_equal(r.best, best)
        assert np.float32(r.best_fit).view(np.uint32) == np.float32(bf).view(np.uint32)
        assert r.best_index == bi
        assert np.array_equal(r.trace.view(np.uint32), trace.view(np.uint32))
        assert r.device_ms > 0
    # the best fitness of the GPU solve, recomputed by the oracle in FP64
    want = oracle_mod.fitness(drop.beta, best[None], T=196, se_mode=se_mode, M=M, rho=rho)[0]
    assert abs(bf - want) / want <= 1e-5


def test_solve_random_init_and_zero_generations(oracle_mod):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    drop = scenario.make_drop(7, 4, seed=2, instance_id=1)
    inst = pa.pa_instance_create(ctx(), drop.beta, None, None, T=0)
    p = pa.GaParams(pop=20, gens=0, elite=2, kmeans_frac=0.0, seed=5)
    r = pa.pa_solve(inst, p)
    pop = oracle_mod.init_pop(7, 4, 20, 0.0, 0.1, 5, 0, None)
    f = oracle_mod.fitness(drop.beta, pop)
    b = oracle_mod.rank(f)[0]
    assert np.array_equal(r.best, pop[b])
    assert abs(r.best_fit - f[b]) / f[b] <= 1e-5
    with pytest.raises(pa.PaError):
        pa.pa_solve(inst, pa.GaParams(pop=20, kmeans_frac=0.5))  # no positions


def test_stepwise_matches_solve():
    """Stepping generation by generation (caller-controlled termination) gives the
    same bits as a whole solve; stopping after k generations equals a solve
    with gens = k (random words are keyed by generation, not by the total)."""
    need_gpu()
    import paper_2511_20511_amd as pa
    drop = scenario.make_drop(19, 16, seed=4, instance_id=2)
    inst = pa.pa_instance_create(ctx(), drop.beta, drop.user_xy, drop.bs_xy, T=196)
    p = pa.GaParams(pop=96, gens=30, elite=4, seed=9, instance_id=2)
    pa.pa_solve_begin(inst, p)
    pa.pa_solve_next(inst, 10)
    r10, done = pa.pa_solve_state(inst)
    assert done == 10
    ref10 = pa.pa_solve(inst, pa.GaParams(pop=96, gens=10, elite=4, seed=9, instance_id=2))
    pa.pa_solve_begin(inst, p)
    pa.pa_solve_next(inst, 10)
    r10b, _ = pa.pa_solve_state(inst)
    pa.pa_solve_next(inst, 20)
    r30, done = pa.pa_solve_state(inst)
    assert done == 30
    ref30 = pa.pa_solve(inst, p)
    for a, b in ((r10, ref10), (r10b, ref10), (r30, ref30)):
        assert np.array_equal(a.best, b.best)
        assert np.float32(a.best_fit).view(np.uint32) == np.float32(b.best_fit).view(np.uint32)
        assert np.array_equal(a.trace.view(np.uint32), b.trace.view(np.uint32))
    with pytest.raises(pa.PaError):
        pa.pa_solve_next(inst, 1)


def test_persistent_block_override_keeps_bits():
    """PA_PERSIST_BLOCK restricts the persistent autotuner to one workgroup
    size; the shape follows it and the results do not change."""
    need_gpu()
    import os
    import paper_2511_20511_amd as pa
    flush("persistent block override")
    d = scenario.make_drop(19, 16, seed=4, instance_id=2)
    prob = dict(beta=d.beta, user_xy=d.user_xy, bs_xy=d.bs_xy, T=196, M=256,
                rho=scenario.snr_to_rho(10.0))
    params = pa.GaParams(pop=256, gens=30, elite=8, seed=4, instance_id=2)
    results, shapes = [], []
    saved = os.environ.get("PA_PERSIST_BLOCK")
    try:
        for only in ("256", "512", None):
            if only is None:
                os.environ.pop("PA_PERSIST_BLOCK", None)
            else:
                os.environ["PA_PERSIST_BLOCK"] = only
            inst = pa.pa_instance_create(ctx(), **prob)  # a new plan per setting
            results.append(pa.pa_solve(inst, params))
            shapes.append(pa.pa_solve_shape(ctx(), inst))
            inst.close()
    finally:
        if saved is None:
            os.environ.pop("PA_PERSIST_BLOCK", None)
        else:
            os.environ["PA_PERSIST_BLOCK"] = saved
    assert all(s["persistent"] == 1 for s in shapes)
    assert shapes[0]["block"] == 256 and shapes[1]["block"] == 512
    for r in results[1:]:
        assert np.array_equal(r.best, results[0].best)
        assert np.array_equal(r.trace.view(np.uint32), results[0].trace.view(np.uint32))
        assert np.float32(r.best_fit).view(np.uint32) == np.float32(results[0].best_fit).view(np.uint32)
