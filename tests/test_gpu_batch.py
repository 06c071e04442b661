"""pa_solve_batch: many uneven instances in one graph-captured solve.

Each instance's result inside a mixed batch (different L, K, population,
generations, SE mode, K-means share; unrolled, tiled and runtime-L kernels)
must be bit-identical to the same instance solved alone with pa_solve, whose
trajectory the lockstep tests tie to the oracle; the best fitness is checked
against the oracle's FP64 value."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu

MIX = [
    # L, K, N, G, E, se_mode, kmeans_frac
    (7, 4, 50, 20, 2, 0, 0.5), (19, 16, 256, 10, 8, 0, 0.5), (37, 32, 64, 3, 8, 0, 0.5),
    (7, 5, 40, 15, 2, 1, 0.5), (5, 6, 30, 12, 3, 0, 0.0), (19, 17, 100, 8, 8, 0, 0.3),
    (37, 16, 40, 4, 4, 1, 0.5), (7, 4, 33, 0, 2, 0, 0.5), (19, 16, 129, 6, 1, 0, 1.0),
]


def _make(pa, i, L, K, se_mode):
    drop = scenario.make_drop(L, K, seed=11, instance_id=i)
    rho = scenario.snr_to_rho(10.0)
    inst = pa.pa_instance_create(ctx(), drop.beta, drop.user_xy, drop.bs_xy, T=196, M=128,
                                 rho=rho, se_mode=se_mode)
    return drop, inst, rho


def test_batch_equals_alone(oracle_mod):
    need_gpu()
    import paper_2511_20511_amd as pa
    insts, params, drops, rhos, modes = [], [], [], [], []
    for i, (L, K, N, G, E, mode, frac) in enumerate(MIX):
        drop, inst, rho = _make(pa, i, L, K, mode)
        insts.append(inst)
        drops.append(drop)
        rhos.append(rho)
        modes.append(mode)
        params.append(pa.GaParams(pop=N, gens=G, elite=E, p_cross=0.8, p_mut=0.05,
                                  kmeans_frac=frac, p_init=0.1, seed=1234 + i, instance_id=i))
    flush(f"batch of {len(insts)} mixed instances")
    batch = pa.pa_solve_batch(ctx(), insts, params)
    again = pa.pa_solve_batch(ctx(), insts, params)  # replay of the captured graph
    for i, inst in enumerate(insts):
        alone = pa.pa_solve(inst, params[i])
        for r in (batch[i], again[i]):
            assert np.array_equal(r.best, alone.best), i
            assert np.float32(r.best_fit).view(np.uint32) == np.float32(alone.best_fit).view(np.uint32)
            assert r.best_index == alone.best_index
            assert np.array_equal(r.trace.view(np.uint32), alone.trace.view(np.uint32))
        want = oracle_mod.fitness(drops[i].beta, alone.best[None], T=196, se_mode=modes[i], M=128,
                                  rho=rhos[i])[0]
        assert abs(alone.best_fit - want) / want <= 1e-5
        assert np.all(np.diff(alone.trace) >= 0)


def test_uneven_mix_small(oracle_mod):
    """An uneven mix drawn like the large batched workload (L in {7, 19, 37},
    K in [4, 32], N in [128, 1024]) with few generations; every instance is
    identical alone and in the batch."""
    need_gpu()
    import paper_2511_20511_amd as pa
    sizes = scenario.size_mix(12, seed=3)
    insts, params = [], []
    for i, (L, K, N) in enumerate(sizes):
        _, inst, _ = _make(pa, 100 + i, L, K, 0)
        insts.append(inst)
        params.append(pa.GaParams(pop=N, gens=3, elite=8, seed=5, instance_id=i))
    flush(f"uneven batch {sizes}")
    batch = pa.pa_solve_batch(ctx(), insts, params)
    for i, inst in enumerate(insts):
        alone = pa.pa_solve(inst, params[i])
        assert np.array_equal(batch[i].best, alone.best)
        assert np.array_equal(batch[i].trace.view(np.uint32), alone.trace.view(np.uint32))


def test_batch_rejects_bad_input():
    need_gpu()
    import paper_2511_20511_amd as pa
    _, inst, _ = _make(pa, 0, 7, 4, 0)
    p = pa.GaParams(pop=20, gens=2)
    with pytest.raises(pa.PaError):
        pa.pa_solve_batch(ctx(), [inst, inst], [p, p])
    with pytest.raises(pa.PaError):
        pa.pa_solve_batch(ctx(), [], [])
    with pytest.raises(pa.PaError):
        pa.pa_solve_batch(ctx(), [inst], [pa.GaParams(pop=1)])
