"""Helpers shared by the GPU tests: device setup and seeded inputs."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


_CTX = {}


def ctx():
    import paper_2511_20511_amd as pa
    if "ctx" not in _CTX:
        _CTX["ctx"] = pa.pa_context_create(0)
    return _CTX["ctx"]


def rand_pop(rng, n, L, K):
    """n chromosomes with uniformly random permutation rows."""
    keys = rng.random((n, L, K))
    return np.argsort(keys, axis=2).astype(np.uint8)


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return np.abs(got - want) / np.maximum(np.abs(want), 1e-300)


def flush(msg):
    print(msg, flush=True)
