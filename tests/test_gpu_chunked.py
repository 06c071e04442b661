"""Batches and server ticks with more generation tasks than workgroups.

A workgroup of the batched generation kernel then runs several tasks in one
launch: it keeps the table (or, tiled, the tile it last loaded) of its
instance in LDS across consecutive tasks, switches instance in the middle of
its run (across instances of different K inside one padded-pilot class, so
the row pass changes between the K % 4 == 0 and the other branch), and with
tiled tables alternates the order of its tile visits.  Every instance must
still come out bit-identical to a pa_solve of it alone, and one instance per
batch is followed generation by generation against the oracle (Alg. 1 loop
body: the oracle's GA step fed the GPU's FP32 fitness reproduces the batch's
population; the fitness is within 1e-5 of the FP64 definition, Eq. 5-7).
"""
import numpy as np
import pytest

from gpu_util import ctx, flush, lockstep, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu


def _instances(pa, sizes, seed0):
    drops, insts, params = [], [], []
    for i, (L, K, N, G) in enumerate(sizes):
        d = scenario.make_drop(L, K, seed=seed0, instance_id=i)
        insts.append(pa.pa_instance_create(ctx(), d.beta, d.user_xy, d.bs_xy, T=196, M=256,
                                           rho=scenario.snr_to_rho(10.0)))
        params.append(pa.GaParams(pop=N, gens=G, elite=8, p_cross=0.8, p_mut=0.05,
                                  kmeans_frac=0.5, p_init=0.1, seed=seed0 + i, instance_id=i))
        drops.append(d)
    return drops, insts, params


def _tasks(block, sizes):
    """Generation tasks of one launch of the first instance's class (same L and
    padded pilot count): an elite task and ceil((N-E)/(block//K)) child tasks
    per instance."""
    def pad(k):
        return max(4, 1 << (k - 1).bit_length())
    L0, TP0 = sizes[0][0], pad(sizes[0][1])
    return sum(1 + -(-(N - 8) // max(1, block // K)) for (L, K, N, _) in sizes
               if L == L0 and pad(K) == TP0)


def _same(a, b):
    assert np.array_equal(a.best, b.best)
    assert np.float32(a.best_fit).view(np.uint32) == np.float32(b.best_fit).view(np.uint32)
    assert a.best_index == b.best_index
    assert np.array_equal(a.trace.view(np.uint32), b.trace.view(np.uint32))


def _check_batch(pa, oracle_mod, torch, sizes, seed0, follow):
    drops, insts, params = _instances(pa, sizes, seed0)
    flush(f"batch of {len(sizes)}: {sizes[:4]} ...")
    batch = pa.pa_solve_batch(ctx(), insts, params)
    shape = pa.pa_solve_shape(ctx(), None)
    ntasks = _tasks(shape["block"], sizes)
    flush(f"  plan {shape}, {ntasks} tasks per generation launch")
    assert shape["persistent"] == 0
    assert ntasks > shape["workgroups"], "the case must give workgroups several tasks"
    # the batch's final population of the followed instance, lockstep with the oracle
    L, K, N, G = sizes[follow]
    got_pop, got_fit, gen = pa.pa_solve_population(ctx(), None, follow, L, K, N)
    assert gen == G
    want_pop, want_fit, _, worst = lockstep(pa, oracle_mod, torch, drops[follow], insts[follow],
                                            params[follow])
    flush(f"  instance {follow}: worst fitness rel err {worst:.2e}")
    assert worst <= 1e-5
    assert np.array_equal(got_pop, want_pop)
    assert np.array_equal(got_fit.view(np.uint32), want_fit.view(np.uint32))
    # every instance: the same bits as alone
    for i, inst in enumerate(insts):
        alone = pa.pa_solve(inst, params[i])
        _same(batch[i], alone)
    for inst in insts:
        inst.close()


def test_tiled_class_more_tasks_than_workgroups(oracle_mod):
    """Five instances of the 64-instance L=37 workload's shape with 2
    generations: 325 tasks on at most 256 workgroups (tiled table)."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    _check_batch(pa, oracle_mod, torch, [(37, 32, 1024, 2)] * 5, 41, follow=3)


def test_tiled_class_mixed_k(oracle_mod):
    """L=37 instances of K = 17, 20, 25, 32 in the padded-pilot class 32:
    workgroups switch instance, K and row-pass branch inside their runs."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    ks = [17, 32, 20, 25, 32, 17, 25, 20, 32, 17, 24]
    sizes = [(37, k, 1024 - 37 * i, 2) for i, k in enumerate(ks)]
    _check_batch(pa, oracle_mod, torch, sizes, 53, follow=5)


def test_whole_table_class_mixed_k(oracle_mod):
    """L=19 instances of K = 17..32 (whole table in LDS) with about three tasks
    per workgroup, plus an L=7 class beside them."""
    torch = need_gpu()
    import paper_2511_20511_amd as pa
    ks = [17, 32, 20, 25] * 6
    sizes = [(19, k, 1024 - 11 * i, 2) for i, k in enumerate(ks)] + [(7, 4, 200, 3)] * 3
    _check_batch(pa, oracle_mod, torch, sizes, 67, follow=10)


def test_server_ticks_with_more_tasks_than_workgroups():
    """Ten L=37 requests resident at once: each tick's launch gives
    workgroups several tasks; every result equals pa_solve alone."""
    need_gpu()
    import paper_2511_20511_amd as pa
    ks = [32, 17, 25, 32, 20, 32, 17, 32, 24, 32]
    sizes = [(37, k, 1024, 6) for k in ks]
    drops, insts, params = _instances(pa, sizes, 71)
    flush(f"server with {len(sizes)} L=37 requests")
    srv = pa.pa_server_create(ctx(), max_slots=len(sizes), max_L=37, max_K=32, max_pop=1024,
                              max_gens=8)
    tickets = [pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params=p, T=196, M=256,
                                   rho=scenario.snr_to_rho(10.0))
               for d, p in zip(drops, params)]
    results = [pa.pa_server_poll(srv, t) for t in tickets]
    st = pa.pa_server_stats(srv)
    srv.close()
    flush(f"  {st}")
    assert st["max_tasks_per_workgroup"] > 1
    for i, inst in enumerate(insts):
        _same(results[i], pa.pa_solve(inst, params[i]))
        inst.close()


def test_graph_shapes_keep_bits():
    """Every shape the graph-form autotuner can pick (threads per workgroup,
    children per task) gives the same bits: a mixed batch under forced shapes
    against the tuned one."""
    need_gpu()
    import os
    import paper_2511_20511_amd as pa
    sizes = [(37, 32, 300, 3), (37, 20, 200, 3), (19, 16, 256, 4), (19, 25, 180, 4),
             (7, 4, 128, 5), (7, 9, 150, 5), (12, 7, 64, 3)]
    drops, insts, params = _instances(pa, sizes, 83)
    saved = os.environ.get("PA_GRAPH_SHAPE")
    results = {}
    try:
        for force in (None, "256,1", "512,1", "512,2", "256,4", "512,8"):
            if force is None:
                os.environ.pop("PA_GRAPH_SHAPE", None)
            else:
                os.environ["PA_GRAPH_SHAPE"] = force
            # a new plan per setting: another instance set is planned in between
            pa.pa_solve_batch(ctx(), insts[:1], params[:1])
            results[force] = pa.pa_solve_batch(ctx(), insts, params)
            flush(f"  shape {force}: {pa.pa_solve_shape(ctx(), None)}")
    finally:
        if saved is None:
            os.environ.pop("PA_GRAPH_SHAPE", None)
        else:
            os.environ["PA_GRAPH_SHAPE"] = saved
    ref = results[None]
    for force, res in results.items():
        for a, b in zip(res, ref):
            _same(a, b)
    for inst in insts:
        inst.close()
