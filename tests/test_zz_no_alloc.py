"""pa_solve_noalloc: the solve without device allocation (scratch array of
the library) gives the same bits as pa_solve, call after call on one device,
including a second call with a smaller problem than the first (the scratch
keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu


def _noalloc(pa, torch, inst, params):
    """One pa_solve_noalloc call through the C ABI into fresh device tensors."""
    d_best = torch.full((inst.L, inst.K), 255, dtype=torch.uint8, device="cuda")
    d_fit = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    d_trace = torch.full((params.gens + 1,), -1.0, dtype=torch.float32, device="cuda")
    p = params.to_c()
    st = pa.lib().pa_solve_noalloc(inst.h, ctypes.byref(p), ctypes.c_void_p(d_best.data_ptr()),
                                   ctypes.c_void_p(d_fit.data_ptr()),
                                   ctypes.c_void_p(d_trace.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, pa.pa_last_error()
    torch.cuda.synchronize()
    return d_best.cpu().numpy(), float(d_fit.cpu().numpy()[0]), d_trace.cpu().numpy()


def _check(pa, torch, L, K, N, G, E, seed, se_mode=0):
    d = scenario.make_drop(L, K, seed=seed, instance_id=0)
    inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196, M=128,
                                 rho=scenario.snr_to_rho(10.0), se_mode=se_mode)
    params = pa.GaParams(pop=N, gens=G, elite=E, p_cross=0.8, p_mut=0.05, kmeans_frac=0.5,
                         p_init=0.1, seed=seed, instance_id=0)
    flush(f"no-alloc solve L={L} K={K} N={N} G={G} mode={se_mode}")
    best, fit, trace = _noalloc(pa, torch, inst, params)
    ref = pa.pa_solve(inst, params)
    assert np.array_equal(best, ref.best)
    assert np.float32(fit).view(np.uint32) == np.float32(ref.best_fit).view(np.uint32)
    assert np.array_equal(trace.view(np.uint32), ref.trace.view(np.uint32))
    inst.close()


def test_noalloc_matches_solve_twice_second_smaller():
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    _check(pa, torch, 19, 16, 256, 30, 8, seed=3)
    _check(pa, torch, 7, 4, 50, 20, 2, seed=4)


def test_noalloc_other_shapes():
    """Tiled table (L=37, K=32) at full population, the runtime-L kernel and
    the finite-M mode."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    _check(pa, torch, 37, 32, 1024, 3, 8, seed=5)
    _check(pa, torch, 12, 7, 45, 6, 5, seed=6, se_mode=1)


def test_noalloc_rejects_what_does_not_fit():
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    d = scenario.make_drop(37, 32, seed=1, instance_id=0)
    inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196)
    # 2 x 4096 x 37 x 32 bytes of populations alone exceed the 8 MiB scratch
    params = pa.GaParams(pop=4096, gens=2, elite=8)
    d_best = torch.empty((37, 32), dtype=torch.uint8, device="cuda")
    d_fit = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(pa.PaError) as ei:
        pa.pa_solve_noalloc(inst, params, d_best, d_fit)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    inst.close()
