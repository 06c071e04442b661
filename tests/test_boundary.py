"""The C-ABI boundary on the CPU: the library loads, exports every function
include/pa.h declares, and rejects invalid problems and parameters through
its host-only checks (no device needed, no compute call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_2511_20511_amd import scenario

HEADER = os.path.join(ROOT, "include", "pa.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2511_20511_amd as pa
    lib = pa.lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert "gfx950" in pa.pa_version()


def test_status_strings():
    import paper_2511_20511_amd as pa
    assert pa.pa_status_string(0) == "ok"
    assert pa.pa_status_string(-1) == "invalid argument"
    assert pa.pa_status_string(-99) == "unknown status"


def _ok_problem():
    d = scenario.make_drop(7, 4, seed=1)
    return d


@pytest.mark.parametrize("mutate,needle", [
    (lambda b: b.__setitem__((0, 1, 2), -1.0), "<= 0"),
    (lambda b: b.__setitem__((3, 3, 0), np.nan), "non-finite"),
    (lambda b: b.__setitem__((2, 0, 1), np.inf), "non-finite"),
    (lambda b: b.__setitem__((1, 4, 3), 0.0), "<= 0"),
    (lambda b: b.__setitem__((5, 5, 2), 1e30), "2^60"),
])
def test_problem_rejects_bad_beta(mutate, needle):
    import paper_2511_20511_amd as pa
    d = _ok_problem()
    beta = d.beta.copy()
    mutate(beta)
    assert pa.pa_problem_check(beta, d.user_xy, d.bs_xy, T=196) == -1
    assert needle in pa.pa_last_error()


def test_problem_ranges():
    import paper_2511_20511_amd as pa
    d = _ok_problem()
    assert pa.pa_problem_check(d.beta, d.user_xy, d.bs_xy, T=196) == 0
    assert pa.pa_problem_check(d.beta, T=0) == 0
    assert pa.pa_problem_check(d.beta, T=4) == -1          # T must exceed tau
    assert pa.pa_problem_check(d.beta, T=-5) == -1
    assert pa.pa_problem_check(d.beta, se_mode=2) == -1
    assert pa.pa_problem_check(d.beta, se_mode=1, M=0, rho=1.0) == -1
    assert pa.pa_problem_check(d.beta, se_mode=1, M=8, rho=0.0) == -1
    assert pa.pa_problem_check(d.beta, se_mode=1, M=8, rho=2.0) == 0
    one = scenario.make_drop(1, 4, seed=1)
    assert pa.pa_problem_check(one.beta) == -1             # asymptotic needs L >= 2
    assert pa.pa_problem_check(one.beta, se_mode=1, M=8, rho=1.0) == 0
    big = np.ones((65, 65, 2))
    assert pa.pa_problem_check(big) == -1                  # L > 64
    wide = np.ones((2, 2, 65))
    assert pa.pa_problem_check(wide) == -1                 # K > 64
    far = d.user_xy.copy()
    far[3, 1, 0] += 9000.0
    assert pa.pa_problem_check(d.beta, far, d.bs_xy) == -1
    assert pa.pa_problem_check(d.beta, d.user_xy, None) == -1
    fm = d.beta.copy()
    fm[0, 3, :] = 0.0                                      # zeros allowed in finite-M mode
    assert pa.pa_problem_check(fm, se_mode=1, M=8, rho=1.0) == 0


@pytest.mark.parametrize("kw,ok", [
    (dict(pop=1), False), (dict(pop=2, elite=2), True), (dict(pop=65537), False),
    (dict(gens=-1), False), (dict(elite=-1), False), (dict(pop=10, elite=11), False),
    (dict(p_cross=1.5), False), (dict(p_mut=-0.1), False), (dict(p_init=float("nan")), False),
    (dict(kmeans_frac=2.0), False), (dict(p_cross=1.0, p_mut=1.0, p_init=0.0), True),
])
def test_params_ranges(kw, ok):
    import paper_2511_20511_amd as pa
    d = _ok_problem()
    p = pa.GaParams(**kw)
    st = pa.pa_params_check(d.beta, p, d.user_xy, d.bs_xy, T=196)
    assert (st == 0) == ok, pa.pa_last_error()


def test_kmeans_needs_positions():
    import paper_2511_20511_amd as pa
    d = _ok_problem()
    assert pa.pa_params_check(d.beta, pa.GaParams(kmeans_frac=0.5)) == -1
    assert pa.pa_params_check(d.beta, pa.GaParams(kmeans_frac=0.0)) == 0


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import paper_2511_20511_amd as pa
    with pytest.raises(pa.PaError):
        pa.pa_context_create(0)


def test_product_path_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2511_20511_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pa_oracle" not in text and "pao_" not in text, f


def test_objective_is_validated():
    import paper_2511_20511_amd as pa
    from paper_2511_20511_amd import scenario
    d = scenario.make_drop(7, 4, seed=1, instance_id=0)
    for obj, want in ((0, 0), (1, 0), (2, 0), (3, -1), (-1, -1)):
        h = pa._Host(d.beta, d.user_xy, d.bs_xy, 196, 1, 1.0, 0, obj)
        assert pa.lib().pa_problem_check(ctypes.byref(h.c)) == want
    # the Eq. 8 objective has no finite-M form
    for mode, want in ((0, 0), (1, -1)):
        h = pa._Host(d.beta, d.user_xy, d.bs_xy, 196, 64, 10.0, mode, 2)
        assert pa.lib().pa_problem_check(ctypes.byref(h.c)) == want
