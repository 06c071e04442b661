"""GPU parity of pa_fitness (uplink sum SE, Eq. 5-7) against the FP64 oracle.

Tolerance: 1e-5 relative on the sum SE, the bound the FP32 kernel is held to.
Shapes cover the 1-, 2- and 3-ring layouts (L = 7, 19, 37, the unrolled
kernels), other L (the runtime-L kernel), non-power-of-two K (padded pilot
stride, chromosomes straddling waves), ragged tails of a round, a tiled table
(L = 37, K = 32 does not fit LDS), and both SE modes.  Every launch shape must
give identical bits."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu, rand_pop, rel_err, to_dev
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = [
    # (L, K, n): several rounds + a ragged tail for every variant
    (7, 4, 1000), (19, 16, 301), (37, 32, 97), (7, 5, 259), (19, 17, 131), (37, 23, 45),
    (37, 4, 200), (19, 32, 70), (3, 3, 216), (2, 1, 7), (5, 6, 123), (12, 9, 77), (61, 4, 30),
    (40, 64, 9), (7, 32, 65), (2, 64, 3), (37, 16, 50),
]


def _instance(pa, L, K, se_mode, seed=3):
    drop = scenario.make_drop(L, K, seed=seed, instance_id=L * 100 + K)
    rho = scenario.snr_to_rho(10.0)
    inst = pa.pa_instance_create(ctx(), drop.beta, drop.user_xy, drop.bs_xy, T=196, M=128,
                                 rho=rho, se_mode=se_mode)
    return drop, inst, rho


@pytest.mark.parametrize("se_mode", [0, 1])
@pytest.mark.parametrize("L,K,n", CASES)
def test_fitness_matches_oracle(oracle_mod, L, K, n, se_mode):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"fitness parity L={L} K={K} n={n} mode={se_mode}")
    drop, inst, rho = _instance(pa, L, K, se_mode)
    pop = rand_pop(np.random.default_rng(L * K + n), n, L, K)
    d_pop = to_dev(pop, torch)
    d_fit = torch.empty(n, dtype=torch.float32, device="cuda")
    pa.pa_fitness(inst, d_pop, n, d_fit)
    torch.cuda.synchronize()
    got = d_fit.cpu().numpy()
    want = oracle_mod.fitness(drop.beta, pop, T=196, se_mode=se_mode, M=128, rho=rho)
    err = rel_err(got, want)
    flush(f"  max rel err {err.max():.3e}  p99 {np.quantile(err, 0.99):.3e}")
    assert err.max() <= TOL


# the unrolled kernels stage a whole table in the quad layout (L = 7, 19 and
# L = 37 up to K = 16, asymptotic SE) or the row layout (finite-M, tiled L = 37,
# K = 32); the runtime-L kernel always uses the row layout
@pytest.mark.parametrize("L,K", [(7, 4), (19, 16), (37, 32), (7, 5), (19, 17), (5, 6), (37, 16),
                                 (37, 4)])
def test_every_launch_shape_gives_same_bits(L, K):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"fitness shapes L={L} K={K}")
    for se_mode in (0, 1):
        _, inst, _ = _instance(pa, L, K, se_mode)
        n = 203
        pop = rand_pop(np.random.default_rng(7), n, L, K)
        d_pop = to_dev(pop, torch)
        ref = torch.empty(n, dtype=torch.float32, device="cuda")
        pa.pa_fitness(inst, d_pop, n, ref)
        outs = []
        for block, grid, generic in [(0, 1, 0), (0, 3, 0), (64 if K <= 64 else 128, 0, 1),
                                     (256, 0, 1), (1024, 0, 1), (128, 2, 1)]:
            if block and block < K:
                continue
            out = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
            pa.pa_fitness_shaped(inst, d_pop, n, out, block=block, grid_cap=grid, generic=generic)
            outs.append(out)
        # alone vs in a batch: each chromosome evaluated by itself
        single = torch.empty(1, dtype=torch.float32, device="cuda")
        alone = []
        for c in (0, 1, n - 1):
            pa.pa_fitness(inst, d_pop[c:c + 1].contiguous(), 1, single)
            alone.append((c, single.clone()))
        torch.cuda.synchronize()
        r = ref.cpu().numpy().view(np.uint32)
        for o in outs:
            assert np.array_equal(o.cpu().numpy().view(np.uint32), r)
        for c, v in alone:
            assert v.cpu().numpy().view(np.uint32)[0] == r[c]


def test_full_size_sampled(oracle_mod):
    """L = 37, K = 32, a population of 1024 (one instance of the batched
    workload): every chromosome of a sample against the oracle."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush("fitness full size L=37 K=32 n=1024")
    drop, inst, rho = _instance(pa, 37, 32, 0, seed=1)
    n = 1024
    pop = rand_pop(np.random.default_rng(99), n, 37, 32)
    d_pop = to_dev(pop, torch)
    d_fit = torch.empty(n, dtype=torch.float32, device="cuda")
    pa.pa_fitness(inst, d_pop, n, d_fit)
    torch.cuda.synchronize()
    got = d_fit.cpu().numpy()
    idx = np.random.default_rng(5).choice(n, 48, replace=False)
    want = oracle_mod.fitness(drop.beta, pop[idx], T=196)
    assert rel_err(got[idx], want).max() <= TOL


def test_zero_and_invalid_sizes():
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    _, inst, _ = _instance(pa, 7, 4, 0)
    d_pop = torch.zeros((1, 7, 4), dtype=torch.uint8, device="cuda")
    d_fit = torch.zeros(1, dtype=torch.float32, device="cuda")
    pa.pa_fitness(inst, d_pop, 0, d_fit)  # no-op
    with pytest.raises(pa.PaError):
        pa.pa_fitness(inst, d_pop, -1, d_fit)
    with pytest.raises(pa.PaError):
        pa.pa_fitness_shaped(inst, d_pop, 1, d_fit, block=96)


# the population's bytes may start anywhere: every staging path (tiled with
# per-wave staging, tiled and untiled with workgroup staging, permutes or byte
# scatters for the inverse rows, the runtime-L kernel) must give the same
# bits from a population 1, 2 or 3 bytes past a 4-byte boundary
@pytest.mark.parametrize("se_mode", [0, 1])
@pytest.mark.parametrize("L,K,n", [(37, 32, 97), (37, 23, 45), (19, 16, 301), (7, 5, 259),
                                   (19, 17, 131), (37, 16, 50), (37, 4, 200), (12, 9, 77)])
def test_fitness_of_unaligned_population(L, K, n, se_mode):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"fitness unaligned population L={L} K={K} n={n} mode={se_mode}")
    _, inst, _ = _instance(pa, L, K, se_mode)
    pop = rand_pop(np.random.default_rng(7 * L + K), n, L, K)
    nb = n * L * K
    fits = []
    for off in range(4):
        buf = torch.zeros(nb + 8, dtype=torch.uint8, device="cuda")
        d_pop = buf[off:off + nb].view(n, L, K)
        d_pop.copy_(torch.from_numpy(pop))
        assert d_pop.data_ptr() % 4 == off % 4
        d_fit = torch.empty(n, dtype=torch.float32, device="cuda")
        pa.pa_fitness(inst, d_pop, n, d_fit)
        torch.cuda.synchronize()
        fits.append(d_fit.cpu().numpy().view(np.uint32))
    for f in fits[1:]:
        assert np.array_equal(f, fits[0])
