"""Max-min objective (smallest per-user SE): FP32 fitness within 1e-5 of the
FP64 oracle on every kernel path, and solves in lockstep with the oracle's GA
(which ranks by whatever fitness it is fed)."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu, rel_err
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,K,n,se_mode", [(7, 4, 300, 0), (19, 16, 257, 0), (37, 32, 70, 0),
                                           (37, 16, 40, 1), (5, 6, 90, 0), (12, 9, 33, 1)])
def test_maxmin_fitness(oracle_mod, L, K, n, se_mode):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"max-min fitness L={L} K={K} n={n} mode={se_mode}")
    d = scenario.make_drop(L, K, seed=9, instance_id=1)
    rho = scenario.snr_to_rho(10.0)
    inst = pa.pa_instance_create(ctx(), d.beta, T=196, M=128, rho=rho, se_mode=se_mode,
                                 objective=pa.OBJ_MIN_SINR)
    rng = np.random.default_rng(L * 100 + K)
    pop = np.stack([np.stack([rng.permutation(K) for _ in range(L)]) for _ in range(n)]).astype(np.uint8)
    d_pop = torch.from_numpy(pop).cuda()
    d_fit = torch.zeros(n, dtype=torch.float32, device="cuda")
    pa.pa_fitness(inst, d_pop, n, d_fit)
    got = d_fit.cpu().numpy()
    want = oracle_mod.fitness(d.beta, pop, T=196, se_mode=se_mode, M=128, rho=rho, objective=1)
    assert rel_err(got, want).max() <= 1e-5
    # the sum objective on the same instance data is unchanged
    inst_sum = pa.pa_instance_create(ctx(), d.beta, T=196, M=128, rho=rho, se_mode=se_mode)
    pa.pa_fitness(inst_sum, d_pop, n, d_fit)
    want_sum = oracle_mod.fitness(d.beta, pop, T=196, se_mode=se_mode, M=128, rho=rho)
    assert rel_err(d_fit.cpu().numpy(), want_sum).max() <= 1e-5
    inst.close()
    inst_sum.close()


@pytest.mark.parametrize("L,K,N,G,E", [(19, 16, 96, 8, 4), (7, 4, 50, 20, 2), (5, 6, 33, 6, 3)])
def test_maxmin_solve_lockstep(oracle_mod, L, K, N, G, E):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"max-min solve L={L} K={K} N={N} G={G}")
    d = scenario.make_drop(L, K, seed=2, instance_id=3)
    inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196,
                                 objective=pa.OBJ_MIN_SINR)
    p = pa.GaParams(pop=N, gens=G, elite=E, seed=4, instance_id=3)
    d_pop = torch.zeros((N, L, K), dtype=torch.uint8, device="cuda")
    d_next = torch.zeros_like(d_pop)
    d_fit = torch.zeros(N, dtype=torch.float32, device="cuda")
    pa.pa_kmeans_init(inst, p, d_pop)
    trace = []
    for g in range(G + 1):
        pa.pa_fitness(inst, d_pop, N, d_fit)
        torch.cuda.synchronize()
        pop, fit = d_pop.cpu().numpy(), d_fit.cpu().numpy()
        want = oracle_mod.fitness(d.beta, pop, T=196, objective=1)
        assert rel_err(fit, want).max() <= 1e-5
        trace.append(fit[oracle_mod.rank(fit.astype(np.float64))[0]])
        if g == G:
            break
        pa.pa_ga_step(inst, p, g, d_pop, d_fit, d_next)
        torch.cuda.synchronize()
        nxt = oracle_mod.ga_step(pop, fit.astype(np.float64), E, p.p_cross, p.p_mut, p.seed,
                                 p.instance_id, g)
        assert np.array_equal(d_next.cpu().numpy(), nxt)
        d_pop, d_next = d_next, d_pop
    trace = np.array(trace, dtype=np.float32)
    for fn in (pa.pa_solve, pa.pa_solve_plain):
        r = fn(inst, p)
        assert np.array_equal(r.trace.view(np.uint32), trace.view(np.uint32))
    shape = pa.pa_solve_shape(None, inst)
    flush(f"  solve plan {shape}")
    inst.close()


# ---- Eq. 8 (Sec. 4.2): minus the inter-cluster interference ---------------

@pytest.mark.parametrize("L,K,n", [(7, 4, 300), (19, 16, 257), (37, 32, 70), (37, 16, 40),
                                   (5, 6, 90), (12, 9, 33), (61, 8, 20), (3, 64, 11)])
def test_eq8_fitness(oracle_mod, L, K, n):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"Eq. 8 fitness L={L} K={K} n={n}")
    d = scenario.make_drop(L, K, seed=5, instance_id=2)
    inst = pa.pa_instance_create(ctx(), d.beta, T=196, objective=pa.OBJ_INTERCLUSTER)
    rng = np.random.default_rng(L * 1000 + K)
    pop = np.argsort(rng.random((n, L, K)), axis=2).astype(np.uint8)
    d_fit = torch.zeros(n, dtype=torch.float32, device="cuda")
    pa.pa_fitness(inst, torch.from_numpy(pop).cuda(), n, d_fit)
    want = oracle_mod.fitness(d.beta, pop, T=196, objective=2)
    assert np.all(want < 0)
    assert rel_err(d_fit.cpu().numpy(), want).max() <= 1e-5
    inst.close()


def test_eq8_hand_worked_exact():
    """The hand-worked instances (power-of-two gains and ratios) come out exact
    in FP32: the per-BS scaling is a power of two and so is every ratio."""
    import json
    import os
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    with open(os.path.join(os.path.dirname(__file__), "golden", "eq8_hand.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        flush(f"Eq. 8 hand-worked {case['name']}")
        beta = np.array(case["beta"], dtype=np.float64)
        chrom = np.array(case["chrom"], dtype=np.uint8)[None]
        inst = pa.pa_instance_create(ctx(), beta, objective=pa.OBJ_INTERCLUSTER)
        d_fit = torch.zeros(1, dtype=torch.float32, device="cuda")
        pa.pa_fitness(inst, torch.from_numpy(chrom).cuda(), 1, d_fit)
        assert float(d_fit.cpu()[0]) == -case["interference"]
        inst.close()


@pytest.mark.parametrize("L,K,N,G,E", [(19, 16, 96, 8, 4), (7, 4, 50, 20, 2)])
def test_eq8_solve_lockstep(oracle_mod, L, K, N, G, E):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"Eq. 8 solve L={L} K={K} N={N} G={G}")
    d = scenario.make_drop(L, K, seed=6, instance_id=1)
    inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196,
                                 objective=pa.OBJ_INTERCLUSTER)
    p = pa.GaParams(pop=N, gens=G, elite=E, seed=8, instance_id=1)
    d_pop = torch.zeros((N, L, K), dtype=torch.uint8, device="cuda")
    d_next = torch.zeros_like(d_pop)
    d_fit = torch.zeros(N, dtype=torch.float32, device="cuda")
    pa.pa_kmeans_init(inst, p, d_pop)
    trace = []
    for g in range(G + 1):
        pa.pa_fitness(inst, d_pop, N, d_fit)
        torch.cuda.synchronize()
        pop, fit = d_pop.cpu().numpy(), d_fit.cpu().numpy()
        assert rel_err(fit, oracle_mod.fitness(d.beta, pop, objective=2)).max() <= 1e-5
        trace.append(fit[oracle_mod.rank(fit.astype(np.float64))[0]])
        if g == G:
            break
        pa.pa_ga_step(inst, p, g, d_pop, d_fit, d_next)
        torch.cuda.synchronize()
        nxt = oracle_mod.ga_step(pop, fit.astype(np.float64), E, p.p_cross, p.p_mut, p.seed,
                                 p.instance_id, g)
        assert np.array_equal(d_next.cpu().numpy(), nxt)
        d_pop, d_next = d_next, d_pop
    trace = np.array(trace, dtype=np.float32)
    assert np.all(np.diff(trace) >= 0)
    for fn in (pa.pa_solve, pa.pa_solve_plain):
        r = fn(inst, p)
        assert np.array_equal(r.trace.view(np.uint32), trace.view(np.uint32))
    inst.close()


def test_eq8_tiled_batch_matches_alone(oracle_mod):
    """L = 37, K = 32 (tiled tables in the batch generation kernel) with the Eq.
    8 objective: a batch beside a sum-SE instance gives each instance the bits
    of its own solve, and the best chromosome's fitness matches the oracle."""
    need_gpu()
    import paper_2511_20511_amd as pa
    flush("Eq. 8 batch L=37 K=32")
    insts, params, drops = [], [], []
    for i, obj in enumerate((pa.OBJ_INTERCLUSTER, pa.OBJ_SUM_SE, pa.OBJ_INTERCLUSTER)):
        d = scenario.make_drop(37, 32, seed=3, instance_id=i)
        drops.append(d)
        insts.append(pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196,
                                           objective=obj))
        params.append(pa.GaParams(pop=160, gens=3, elite=4, seed=2, instance_id=i))
    res = pa.pa_solve_batch(ctx(), insts, params)
    for i, (inst, p, d) in enumerate(zip(insts, params, drops)):
        alone = pa.pa_solve(inst, p)
        assert np.array_equal(res[i].best, alone.best)
        assert np.array_equal(res[i].trace.view(np.uint32), alone.trace.view(np.uint32))
        obj = 2 if i != 1 else 0
        want = oracle_mod.fitness(d.beta, res[i].best[None], T=196, objective=obj)[0]
        assert abs(res[i].best_fit - want) <= 1e-5 * abs(want)
    for inst in insts:
        inst.close()
