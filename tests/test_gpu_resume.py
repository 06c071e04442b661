"""Checkpoint and resume of a solve (Alg. 1 loop state): G generations in one
go against gen generations, the state saved to disk, a new context and
instance, the state restored with pa_solve_resume and the G - gen remaining
generations.  The populations, best chromosome, fitness and trace must be the
same bits, in each execution form of the solve (one-workgroup, persistent,
one launch per generation in a graph)."""
import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu

# (L, K, N, G, E, gen, form: PA_SMALL_FORM or None, expected shape["persistent"])
CASES = [
    (7, 4, 50, 40, 2, 13, "workgroup", 2),
    (19, 16, 256, 30, 8, 11, "persistent", 1),
    (37, 32, 8192, 6, 8, 2, None, 0),  # 512 tasks: more than fit at once, graph form
]


def _bits(x):
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def _instance(pa, c, L, K, inst_id):
    d = scenario.make_drop(L, K, seed=31, instance_id=inst_id)
    return pa.pa_instance_create(c, d.beta, d.user_xy, d.bs_xy, T=196)


@pytest.mark.parametrize("L,K,N,G,E,gen,form,persistent", CASES)
def test_resume_from_saved_state(monkeypatch, tmp_path, L, K, N, G, E, gen, form, persistent):
    need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"resume L={L} K={K} N={N} G={G} gen={gen} form={form}")
    if form is None:
        monkeypatch.delenv("PA_SMALL_FORM", raising=False)
    else:
        monkeypatch.setenv("PA_SMALL_FORM", form)
    p = pa.GaParams(pop=N, gens=G, elite=E, seed=17, instance_id=5)
    inst = _instance(pa, ctx(), L, K, 5)
    ref = pa.pa_solve(inst, p)
    assert pa.pa_solve_shape(None, inst)["persistent"] == persistent
    pop_ref, fit_ref, g_ref = pa.pa_solve_population(None, inst, 0, L, K, N)
    assert g_ref == G
    # stop after gen generations and save the state
    pa.pa_solve_begin(inst, p)
    pa.pa_solve_next(inst, gen)
    r_gen, done = pa.pa_solve_state(inst)
    assert done == gen
    pop_g, fit_g, g_g = pa.pa_solve_population(None, inst, 0, L, K, N)
    assert g_g == gen
    path = tmp_path / "state.npz"
    np.savez(path, pop=pop_g, fit=fit_g, trace=r_gen.trace, gen=gen)
    inst.close()

    # a new context and instance restore it and finish the solve
    c2 = pa.pa_context_create(0)
    try:
        inst2 = _instance(pa, c2, L, K, 5)
        z = np.load(path)
        g0 = int(z["gen"])
        pa.pa_solve_resume(inst2, p, g0, z["pop"], z["fit"], z["trace"][:g0])
        pa.pa_solve_next(inst2, G - g0)
        r, done = pa.pa_solve_state(inst2)
        assert done == G
        assert np.array_equal(r.best, ref.best) and r.best_index == ref.best_index
        assert _bits(r.best_fit) == _bits(ref.best_fit)
        assert np.array_equal(_bits(r.trace), _bits(ref.trace))
        pop2, fit2, g2 = pa.pa_solve_population(None, inst2, 0, L, K, N)
        assert g2 == G
        assert np.array_equal(pop2, pop_ref)
        assert np.array_equal(_bits(fit2), _bits(fit_ref))

        # without the fitness (recomputed on the device) and without the
        # trace (its first gen entries NaN), in two steps
        pa.pa_solve_resume(inst2, p, g0, z["pop"])
        first = (G - g0) // 2
        pa.pa_solve_next(inst2, first)
        pa.pa_solve_next(inst2, G - g0 - first)
        r3, done = pa.pa_solve_state(inst2)
        assert done == G
        assert np.array_equal(r3.best, ref.best)
        assert _bits(r3.best_fit) == _bits(ref.best_fit)
        assert np.all(np.isnan(r3.trace[:g0]))
        assert np.array_equal(_bits(r3.trace[g0:]), _bits(ref.trace[g0:]))
        inst2.close()
    finally:
        c2.close()


def test_resume_rejects_invalid_states():
    need_gpu()
    import paper_2511_20511_amd as pa
    flush("resume: invalid states")
    L, K, N = 7, 4, 50
    p = pa.GaParams(pop=N, gens=10, elite=2, seed=3, instance_id=0)
    inst = _instance(pa, ctx(), L, K, 0)
    pop = np.tile(np.arange(K, dtype=np.uint8), (N, L, 1))
    pa.pa_solve_resume(inst, p, 0, pop)  # a valid state
    pa.pa_solve_next(inst, 10)
    _, done = pa.pa_solve_state(inst)
    assert done == 10
    bad = pop.copy()
    bad[3, 2, 1] = bad[3, 2, 0]  # a repeated pilot in one cell
    with pytest.raises(pa.PaError, match="permutation"):
        pa.pa_solve_resume(inst, p, 0, bad)
    bad = pop.copy()
    bad[0, 0, 0] = K  # a pilot outside 0..K-1
    with pytest.raises(pa.PaError, match="permutation"):
        pa.pa_solve_resume(inst, p, 0, bad)
    with pytest.raises(pa.PaError, match="gen"):
        pa.pa_solve_resume(inst, p, 11, pop)
    with pytest.raises(pa.PaError, match="gen"):
        pa.pa_solve_resume(inst, p, -1, pop)
    with pytest.raises(ValueError):
        pa.pa_solve_resume(inst, p, 0, pop[:-1])
    # a resumed state at the last generation: no generation left to run
    pa.pa_solve_resume(inst, p, 10, pop)
    with pytest.raises(pa.PaError):
        pa.pa_solve_next(inst, 1)
    r, done = pa.pa_solve_state(inst)
    assert done == 10 and r.best.shape == (L, K)
    inst.close()
