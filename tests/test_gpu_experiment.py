"""The convergence experiment (K-means-seeded vs random initialisation,
Sec. 6.2, Fig. 3) runs end to end, reports consistent figures, and its solves
are the GA of the oracle: for a few drops, both initialisations, the
oracle's operators fed the GPU's FP32 fitness generation by generation
(Alg. 1 loop body) reproduce the experiment's best chromosome, fitness and
trace bit for bit, and the FP32 fitness stays within 1e-5 of the FP64
definition (Eq. 5-7)."""
import numpy as np
import pytest

from gpu_util import ctx, flush, lockstep, need_gpu

pytestmark = pytest.mark.gpu


def test_convergence_experiment_small(oracle_mod):
    torch = need_gpu()
    import bench
    import paper_2511_20511_amd as pa
    from paper_2511_20511_amd import scenario
    drops, gens = 6, 15
    flush(f"convergence experiment: {drops} drops, {gens} generations")
    keep = {}
    out = bench.run_convergence(pa, scenario, torch, drops=drops, gens=gens, keep=keep)
    for name in ("kmeans_init", "random_init"):
        r = out[name]
        assert 0 <= r["gens_to_99pct_mean"] <= gens
        assert r["best_mean"] >= r["initial_best_mean"] > 0
        q = r["best_quantiles_0_5_10_25_50_75_90_95_100"]
        assert all(a <= b for a, b in zip(q, q[1:]))
        assert len(r["best"]) == drops
        assert r["ms_to_99pct_mean"] > 0
    # the GA never ends below one random assignment or the seed it starts from
    assert out["random_init"]["best_mean"] >= out["random_assignment"]["mean"]
    assert out["kmeans_init"]["best_mean"] >= out["kmeans_seed_only"]["mean"]
    assert 0.0 <= out["kmeans_reaches_99pct_first_frac"] <= 1.0
    assert out["solve_ms_per_generation"] > 0
    # a few drops against the oracle
    params = keep["params"]
    for i in range(2):
        d = scenario.make_drop(19, 16, seed=7, instance_id=i)
        inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196, M=256,
                                     rho=scenario.snr_to_rho(10.0))
        for k, name in ((0, "kmeans_init"), (1, "random_init")):
            r = keep[name][i]
            pop, fit, trace, worst = lockstep(pa, oracle_mod, torch, d, inst, params[2 * i + k])
            b = oracle_mod.rank(fit.astype(np.float64))[0]
            flush(f"  drop {i} {name}: best {r.best_fit:.5f}, worst fitness rel err {worst:.1e}")
            assert worst <= 1e-5
            assert np.array_equal(r.best, pop[b]) and r.best_index == b
            assert np.float32(r.best_fit).view(np.uint32) == fit[b].view(np.uint32)
            assert np.array_equal(r.trace.view(np.uint32), trace.view(np.uint32))
        inst.close()
