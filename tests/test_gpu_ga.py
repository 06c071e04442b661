"""GPU parity of the genetic operators and the K-means seeding (bit-exact).

pa_ga_step is fed the same FP32 fitness as the oracle (widened exactly to
FP64), so selection, crossover, mutation and elitism must reproduce the
oracle's population byte for byte.  pa_kmeans_init is integer-only and must
match the oracle's seed chromosome, centroids, labels, iteration count and
initial population exactly."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu, rand_pop, to_dev
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu


def _inst(pa, L, K, seed=1, inst_id=0):
    drop = scenario.make_drop(L, K, seed=seed, instance_id=inst_id)
    return drop, pa.pa_instance_create(ctx(), drop.beta, drop.user_xy, drop.bs_xy, T=196)


GA_CASES = [
    # L, K, N, E, p_cross, p_mut
    (7, 4, 50, 2, 0.8, 0.05), (19, 16, 256, 8, 0.8, 0.05), (37, 32, 1024, 8, 0.8, 0.05),
    (7, 5, 33, 0, 0.9, 0.02), (5, 3, 12, 12, 0.8, 0.5), (4, 7, 10, 3, 1.0, 1.0),
    (2, 1, 9, 2, 1.0, 1.0), (19, 17, 65, 64, 0.5, 0.1), (3, 3, 70, 66, 0.8, 0.3),
    (12, 9, 101, 1, 0.0, 0.0), (61, 4, 40, 4, 0.8, 0.05), (6, 64, 20, 2, 0.8, 0.05),
]


@pytest.mark.parametrize("L,K,N,E,pc,pm", GA_CASES)
def test_ga_step_bit_exact(oracle_mod, L, K, N, E, pc, pm):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"ga_step L={L} K={K} N={N} E={E}")
    _, inst = _inst(pa, L, K)
    rng = np.random.default_rng(L * 1000 + N)
    pop = rand_pop(rng, N, L, K)
    fit = rng.normal(100.0, 3.0, N).astype(np.float32)
    fit[rng.choice(N, min(5, N), replace=False)] = fit[0]        # ties
    if N > 8:
        fit[3] = np.nan
        fit[5] = -np.inf
    params = pa.GaParams(pop=N, gens=1, elite=E, p_cross=pc, p_mut=pm, seed=0x1234ABCD5678,
                         instance_id=7)
    d_in, d_fit = to_dev(pop, torch), to_dev(fit, torch)
    d_out = torch.zeros_like(d_in)
    for gen in (0, 13):
        pa.pa_ga_step(inst, params, gen, d_in, d_fit, d_out)
        torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        want = oracle_mod.ga_step(pop, fit.astype(np.float64), E, pc, pm, params.seed, 7, gen)
        assert np.array_equal(got, want), f"gen {gen}: first diff at {np.argwhere(got != want)[:3]}"


@pytest.mark.parametrize("L,K,N,frac", [(7, 4, 50, 0.5), (19, 16, 256, 0.5), (37, 32, 1024, 0.5),
                                        (7, 5, 40, 0.0), (19, 17, 64, 1.0), (2, 1, 4, 0.5),
                                        (61, 4, 30, 0.3), (6, 64, 10, 0.5)])
def test_kmeans_init_bit_exact(oracle_mod, L, K, N, frac):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"kmeans_init L={L} K={K} N={N} frac={frac}")
    drop, inst = _inst(pa, L, K, seed=9, inst_id=L + K)
    params = pa.GaParams(pop=N, gens=0, elite=2, kmeans_frac=frac, p_init=0.1, seed=77,
                         instance_id=3)
    d_pop = torch.zeros((N, L, K), dtype=torch.uint8, device="cuda")
    pa.pa_kmeans_init(inst, params, d_pop)
    torch.cuda.synchronize()
    got = d_pop.cpu().numpy()
    seed_o = None
    if frac > 0:
        seed_o, cent_o, lab_o, it_o = oracle_mod.kmeans_seed(drop.user_xy, drop.bs_xy)
        seed_g, cent_g, lab_g, it_g = pa.pa_instance_kmeans_state(inst)
        assert np.array_equal(seed_g, seed_o)
        assert np.array_equal(cent_g, cent_o)
        assert np.array_equal(lab_g, lab_o)
        assert it_g == it_o
    want = oracle_mod.init_pop(L, K, N, frac, 0.1, 77, 3, seed_o)
    assert np.array_equal(got, want)


def test_kmeans_hand_worked_on_gpu():
    """The hand-worked two-cell instance of the oracle tests, on the GPU."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    bs = np.array([[0.0, 0.0], [1000.0, 0.0]])
    users = np.array([[[0.0, 0.0], [0.1, 0.002]], [[1000.0, 0.002], [1000.1, 0.0]]])
    beta = np.full((2, 2, 2), 1e-9)
    inst = pa.pa_instance_create(ctx(), beta, users, bs)
    d_pop = torch.zeros((2, 2, 2), dtype=torch.uint8, device="cuda")
    pa.pa_kmeans_init(inst, pa.GaParams(pop=2, gens=0, kmeans_frac=1.0), d_pop)
    seed, cent, labels, iters = pa.pa_instance_kmeans_state(inst)
    assert cent.tolist() == [[100, 1], [0, 1]]
    assert labels.tolist() == [1, 0, 1, 0]
    assert iters == 1
    assert seed.tolist() == [[1, 0], [1, 0]]


def test_ga_step_rejects_overlap_and_bad_params():
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    _, inst = _inst(pa, 7, 4)
    d = torch.zeros((10, 7, 4), dtype=torch.uint8, device="cuda")
    f = torch.zeros(10, dtype=torch.float32, device="cuda")
    p = pa.GaParams(pop=10, elite=2)
    with pytest.raises(pa.PaError):
        pa.pa_ga_step(inst, p, 0, d, f, d)
    with pytest.raises(pa.PaError):
        pa.pa_ga_step(inst, pa.GaParams(pop=10, elite=11), 0, d, f, torch.zeros_like(d))
    with pytest.raises(pa.PaError):
        pa.pa_ga_step(inst, pa.GaParams(pop=10, p_mut=1.5), 0, d, f, torch.zeros_like(d))
