"""Continuous-batching server: every request's result is bit-identical to a
pa_solve of the same problem and parameters, whatever else is resident, when
it was admitted and which generation the others are at."""
import ctypes
import threading

import numpy as np
import pytest

from gpu_util import ctx, flush, need_gpu
from paper_2511_20511_amd import scenario

pytestmark = pytest.mark.gpu

# (L, K, N, G, E, se_mode, kmeans_frac): unrolled and runtime-L classes, both
# SE modes, random and K-means initialisation, odd N - E, G = 0
MIX = [(7, 4, 50, 12, 2, 0, 0.5), (19, 16, 96, 7, 4, 0, 0.5), (37, 32, 40, 3, 8, 0, 0.5),
       (5, 6, 33, 9, 3, 0, 0.0), (7, 5, 31, 5, 3, 1, 0.5), (19, 9, 64, 0, 2, 0, 0.5),
       (7, 4, 20, 20, 0, 0, 0.0), (12, 7, 45, 6, 5, 1, 0.3)]


def _requests(pa, seed0=11):
    reqs = []
    for i, (L, K, N, G, E, mode, km) in enumerate(MIX):
        d = scenario.make_drop(L, K, seed=seed0, instance_id=i)
        prob = dict(beta=d.beta, user_xy=d.user_xy, bs_xy=d.bs_xy, T=196, M=128,
                    rho=scenario.snr_to_rho(10.0), se_mode=mode)
        params = pa.GaParams(pop=N, gens=G, elite=E, p_cross=0.8, p_mut=0.05, kmeans_frac=km,
                             p_init=0.1, seed=seed0 + i, instance_id=i)
        reqs.append((prob, params))
    return reqs


def _alone(pa, prob, params):
    inst = pa.pa_instance_create(ctx(), **prob)
    r = pa.pa_solve(inst, params)
    inst.close()
    return r


def _same(a, b):
    assert np.array_equal(a.best, b.best)
    assert np.float32(a.best_fit).view(np.uint32) == np.float32(b.best_fit).view(np.uint32)
    assert a.best_index == b.best_index
    assert np.array_equal(a.trace.view(np.uint32), b.trace.view(np.uint32))


@pytest.mark.parametrize("slots", [2, 64])
def test_server_matches_solve(slots):
    need_gpu()
    import paper_2511_20511_amd as pa
    flush(f"server slots={slots}")
    reqs = _requests(pa)
    srv = pa.pa_server_create(ctx(), max_slots=slots, max_L=40, max_K=32, max_pop=128,
                              max_gens=32)
    tickets = [pa.pa_server_submit(srv, params=p, **prob) for prob, p in reqs]
    results = [pa.pa_server_poll(srv, t) for t in tickets]
    st = pa.pa_server_stats(srv)
    assert st["completed"] == len(reqs) and st["resident"] == 0 and st["queued"] == 0
    assert st["slots"] == slots
    srv.close()
    for (prob, p), r in zip(reqs, results):
        assert r.device_ms > 0
        _same(r, _alone(pa, prob, p))


def test_server_requests_join_mid_batch_and_from_threads():
    """Requests submitted while others run (and from two threads) join between
    generations; results are unchanged."""
    need_gpu()
    import paper_2511_20511_amd as pa
    reqs = _requests(pa, seed0=23)
    srv = pa.pa_server_create(ctx(), max_slots=4, max_L=40, max_K=32, max_pop=128, max_gens=32)
    first = [pa.pa_server_submit(srv, params=p, **prob) for prob, p in reqs[:3]]
    out = {}

    def submit(part):
        for k in part:
            prob, p = reqs[k]
            out[k] = pa.pa_server_submit(srv, params=p, **prob)

    th = [threading.Thread(target=submit, args=(list(range(3, 8, 2)),)),
          threading.Thread(target=submit, args=(list(range(4, 8, 2)),))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    tickets = first + [out[k] for k in range(3, 8)]
    results = [pa.pa_server_poll(srv, t) for t in tickets]
    srv.close()
    for (prob, p), r in zip(reqs, results):
        _same(r, _alone(pa, prob, p))


def test_server_rejects_and_reports():
    need_gpu()
    import paper_2511_20511_amd as pa
    srv = pa.pa_server_create(ctx(), max_slots=2, max_L=8, max_K=8, max_pop=64, max_gens=16)
    d = scenario.make_drop(19, 16, seed=1, instance_id=0)
    with pytest.raises(pa.PaError):  # larger than the slots
        pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params=pa.GaParams(pop=32, gens=4))
    d = scenario.make_drop(7, 4, seed=1, instance_id=0)
    with pytest.raises(pa.PaError):  # K-means without positions
        pa.pa_server_submit(srv, d.beta, params=pa.GaParams(pop=32, gens=4, kmeans_frac=0.5))
    t = pa.pa_server_submit(srv, d.beta, d.user_xy, d.bs_xy, params=pa.GaParams(pop=32, gens=4))
    r = pa.pa_server_poll(srv, t)
    assert r.trace.shape == (5,)
    empty = pa._Result(None, 0.0, 0, None, 0.0)
    assert pa.lib().pa_server_poll(srv.h, t, ctypes.byref(empty), 1) == -1  # ticket consumed
    srv.close()


def _small(pa, i, G=6, N=64, L=7, K=4, seed0=300):
    d = scenario.make_drop(L, K, seed=seed0, instance_id=i)
    prob = dict(beta=d.beta, user_xy=d.user_xy, bs_xy=d.bs_xy, T=196)
    return prob, pa.GaParams(pop=N, gens=G, elite=2, seed=seed0 + i, instance_id=i)


def test_server_admits_by_request_bytes():
    """With a budget of two of the largest accepted requests, many small ones
    are resident together (each takes its own bytes, not a largest-size
    slot); every result still equals pa_solve alone."""
    need_gpu()
    import paper_2511_20511_amd as pa
    probe = pa.pa_server_create(ctx(), max_slots=2, max_L=37, max_K=32, max_pop=1024, max_gens=8)
    big = pa.pa_server_stats(probe)["slot_bytes"]
    probe.close()
    srv = pa.pa_server_create(ctx(), max_slots=64, max_L=37, max_K=32, max_pop=1024, max_gens=8,
                              hbm_budget=2 * big)
    reqs = [_small(pa, i) for i in range(24)]
    d = scenario.make_drop(37, 32, seed=5, instance_id=99)
    reqs.append((dict(beta=d.beta, user_xy=d.user_xy, bs_xy=d.bs_xy, T=196),
                 pa.GaParams(pop=1024, gens=3, elite=8, seed=5, instance_id=99)))
    tickets = [pa.pa_server_submit(srv, params=p, **prob) for prob, p in reqs]
    results = [pa.pa_server_poll(srv, t) for t in tickets]
    st = pa.pa_server_stats(srv)
    srv.close()
    flush(f"  {st}")
    assert st["arena_bytes"] <= 2 * big
    assert st["max_resident"] > 2, "small requests must share the arena"
    assert st["arena_peak_bytes"] <= st["arena_bytes"]
    for (prob, p), r in zip(reqs, results):
        _same(r, _alone(pa, prob, p))
    # a request larger than the whole arena is refused at once
    srv = pa.pa_server_create(ctx(), max_slots=4, max_L=37, max_K=32, max_pop=1024, max_gens=8,
                              hbm_budget=big // 2)
    with pytest.raises(pa.PaError) as ei:
        pa.pa_server_submit(srv, params=reqs[-1][1], **reqs[-1][0])
    assert ei.value.status == -2
    srv.close()


def test_server_cancel():
    """A queued and a resident request are cancelled (PA_ECANCELED on poll);
    the others finish with the same bits as alone."""
    need_gpu()
    import paper_2511_20511_amd as pa
    srv = pa.pa_server_create(ctx(), max_slots=2, max_L=8, max_K=8, max_pop=256, max_gens=400)
    reqs = [_small(pa, i, G=300, N=200) for i in range(5)]
    tickets = [pa.pa_server_submit(srv, params=p, **prob) for prob, p in reqs]
    pa.pa_server_cancel(srv, tickets[4])  # still queued behind two slots
    pa.pa_server_cancel(srv, tickets[0])  # resident (or about to be)
    out = {}
    for k, t in enumerate(tickets):
        try:
            out[k] = pa.pa_server_poll(srv, t)
        except pa.PaError as e:
            out[k] = e.status
    st = pa.pa_server_stats(srv)
    with pytest.raises(pa.PaError):  # finished tickets cannot be cancelled
        pa.pa_server_cancel(srv, tickets[1])
    srv.close()
    assert out[4] == -5 and out[0] == -5
    assert st["cancelled"] == 2
    for k in (1, 2, 3):
        _same(out[k], _alone(pa, *reqs[k]))


def test_server_recovers_from_a_failed_tick():
    """A tick that reports a device error (forced from the host: the work
    itself runs normally) fails the requests resident at that moment with
    PA_EDEVICE; the worker keeps serving and later requests match pa_solve."""
    need_gpu()
    import os
    import paper_2511_20511_amd as pa
    os.environ["PA_SERVER_FAULT_TICK"] = "3"
    try:
        srv = pa.pa_server_create(ctx(), max_slots=2, max_L=8, max_K=8, max_pop=256,
                                  max_gens=16)
    finally:
        os.environ.pop("PA_SERVER_FAULT_TICK", None)
    reqs = [_small(pa, i, G=8) for i in range(6)]
    tickets = [pa.pa_server_submit(srv, params=p, **prob) for prob, p in reqs]
    status = []
    for (prob, p), t in zip(reqs, tickets):
        try:
            r = pa.pa_server_poll(srv, t)
            _same(r, _alone(pa, prob, p))
            status.append(0)
        except pa.PaError as e:
            status.append(e.status)
    # later submissions are still served
    prob, p = _small(pa, 50, G=5)
    _same(pa.pa_server_poll(srv, pa.pa_server_submit(srv, params=p, **prob)), _alone(pa, prob, p))
    st = pa.pa_server_stats(srv)
    srv.close()
    flush(f"  statuses {status}, {st}")
    assert -3 in status and 0 in status
    assert st["failed"] == status.count(-3)
