"""The one-workgroup solve (population, fitness and table resident in one
workgroup's LDS) against the persistent form and the oracle: the same bits
for every shape, SE mode and objective it takes, in whole, stepwise and
batched solves (Alg. 1); and in lockstep with the oracle's GA fed the GPU's
FP32 fitness."""
import numpy as np
import pytest

from gpu_util import ctx, flush, lockstep, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu

# (L, K, N, G, E, se_mode, objective)
SHAPES = [(7, 4, 50, 100, 2, 0, 0), (7, 8, 37, 15, 3, 0, 0), (19, 4, 64, 12, 4, 0, 0),
          (19, 16, 32, 10, 2, 0, 0), (37, 8, 20, 5, 2, 0, 0), (7, 4, 40, 10, 0, 0, 0),
          (7, 5, 30, 12, 2, 1, 0), (7, 4, 30, 12, 2, 0, 1), (7, 4, 30, 12, 2, 0, 2),
          (19, 32, 12, 6, 1, 0, 0)]


def _inst(pa, L, K, mode, obj, inst_id=0):
    d = scenario.make_drop(L, K, seed=21, instance_id=inst_id)
    inst = pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196, M=64,
                                 rho=scenario.snr_to_rho(10.0), se_mode=mode, objective=obj)
    return d, inst


def _solve_form(pa, monkeypatch, form, L, K, mode, obj, params, inst_id=0):
    monkeypatch.setenv("PA_SMALL_FORM", form)
    d, inst = _inst(pa, L, K, mode, obj, inst_id)
    r = pa.pa_solve(inst, params)
    shape = pa.pa_solve_shape(None, inst)
    return d, inst, r, shape


def _same(a, b):
    assert np.array_equal(a.best, b.best) and a.best_index == b.best_index
    assert np.float32(a.best_fit).view(np.uint32) == np.float32(b.best_fit).view(np.uint32)
    assert np.array_equal(a.trace.view(np.uint32), b.trace.view(np.uint32))


@pytest.mark.parametrize("L,K,N,G,E,mode,obj", SHAPES)
def test_workgroup_form_equals_persistent(monkeypatch, L, K, N, G, E, mode, obj):
    need_gpu()
    import paper_2511_20511_amd as pa
    p = pa.GaParams(pop=N, gens=G, elite=E, seed=9, instance_id=0)
    flush(f"one-workgroup vs persistent L={L} K={K} N={N} G={G} E={E} mode={mode} obj={obj}")
    _, i1, r1, s1 = _solve_form(pa, monkeypatch, "workgroup", L, K, mode, obj, p)
    _, i2, r2, s2 = _solve_form(pa, monkeypatch, "persistent", L, K, mode, obj, p)
    assert s1["persistent"] == 2 and s1["workgroups"] == 1, s1
    assert s2["persistent"] == 1, s2
    _same(r1, r2)
    if E > 0:  # without elites the best may be lost
        assert np.all(np.diff(r1.trace) >= 0)
    # a replay of the plan gives the same bits
    _same(pa.pa_solve(i1, p), r1)
    i1.close()
    i2.close()


def test_workgroup_form_lockstep_with_oracle(monkeypatch, oracle_mod):
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    p = pa.GaParams(pop=50, gens=100, elite=2, seed=3, instance_id=0)
    flush("one-workgroup solve L=7 K=4 N=50 G=100 against the oracle")
    d, inst, r, s = _solve_form(pa, monkeypatch, "workgroup", 7, 4, 0, 0, p)
    assert s["persistent"] == 2
    pop, fit, trace, worst = lockstep(pa, oracle_mod, torch, d, inst, p)
    b = oracle_mod.rank(fit.astype(np.float64))[0]
    assert worst <= 1e-5
    assert np.array_equal(r.best, pop[b]) and r.best_index == b
    assert np.array_equal(r.trace.view(np.uint32), trace.view(np.uint32))
    inst.close()


def test_workgroup_form_stepwise(monkeypatch):
    need_gpu()
    import paper_2511_20511_amd as pa
    p = pa.GaParams(pop=46, gens=20, elite=3, seed=5, instance_id=0)
    flush("one-workgroup stepwise solve L=19 K=4")
    monkeypatch.setenv("PA_SMALL_FORM", "workgroup")
    _, inst = _inst(pa, 19, 4, 0, 0)
    whole = pa.pa_solve(inst, p)
    assert pa.pa_solve_shape(None, inst)["persistent"] == 2
    pa.pa_solve_begin(inst, p)
    for n in (0, 3, 1, 9):
        pa.pa_solve_next(inst, n)
    mid, done = pa.pa_solve_state(inst)
    assert done == 13
    assert np.array_equal(mid.trace[:14].view(np.uint32), whole.trace[:14].view(np.uint32))
    pa.pa_solve_next(inst, 7)
    end, done = pa.pa_solve_state(inst)
    assert done == 20
    _same(end, whole)
    inst.close()


def test_workgroup_form_batch(monkeypatch):
    need_gpu()
    import paper_2511_20511_amd as pa
    flush("one-workgroup batch of 6 L=7 K=4 instances")
    monkeypatch.setenv("PA_SMALL_FORM", "workgroup")
    insts, params = [], []
    for i in range(6):
        _, inst = _inst(pa, 7, 4, 0, 0, inst_id=i)
        insts.append(inst)
        params.append(pa.GaParams(pop=40 + 2 * i, gens=10 + i, elite=2, seed=11, instance_id=i))
    res = pa.pa_solve_batch(ctx(), insts, params)
    shape = pa.pa_solve_shape(ctx(), None)
    assert shape["persistent"] == 2 and shape["workgroups"] == 6, shape
    monkeypatch.setenv("PA_SMALL_FORM", "persistent")
    for i, (inst, p) in enumerate(zip(insts, params)):
        _, other = _inst(pa, 7, 4, 0, 0, inst_id=i)
        _same(res[i], pa.pa_solve(other, p))
        other.close()
    for inst in insts:
        inst.close()
