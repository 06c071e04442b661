"""The convergence experiment (K-means-seeded vs random initialisation) runs
end to end and reports consistent figures."""
import pytest

from gpu_util import flush, need_gpu

pytestmark = pytest.mark.gpu


def test_convergence_experiment_small():
    torch = need_gpu()
    import bench
    import paper_2511_20511_amd as pa
    from paper_2511_20511_amd import scenario
    flush("convergence experiment: 6 drops, 15 generations")
    out = bench.run_convergence(pa, scenario, torch, drops=6, gens=15)
    for name in ("kmeans_init", "random_init"):
        r = out[name]
        assert 0 <= r["gens_to_99pct_mean"] <= 15
        assert r["best_mean"] >= r["initial_best_mean"] > 0
        lo, mid, hi = r["best_p10_p50_p90"]
        assert lo <= mid <= hi
    # the GA never ends below one random assignment or the seed it starts from
    assert out["random_init"]["best_mean"] >= out["random_assignment"]["mean"]
    assert out["kmeans_init"]["best_mean"] >= out["kmeans_seed_only"]["mean"]
    assert 0.0 <= out["kmeans_reaches_99pct_first_frac"] <= 1.0
