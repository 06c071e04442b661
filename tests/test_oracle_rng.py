"""Pins of the oracle's random streams (CPU only).

Philox4x32-10 is pinned to the published known-answer vectors; the bounded
draw and the probability threshold to their exact edge cases; the stream
layout to its definition (counter = (c0, c1, c2, tag << 24 | block))."""
import os

import numpy as np
import pytest
from scipy import stats

from conftest import GOLDEN

pytestmark = pytest.mark.filterwarnings("ignore")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle_mod.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_stream_word_layout(oracle_mod):
    seed = 0x0123456789ABCDEF
    for c0, c1, c2, tag, idx in [(0, 0, 0, 1, 0), (5, 7, 3, 2, 13), (1023, 0xFFFFFFFF, 63, 0x12, 4095)]:
        blk = oracle_mod.philox4x32_10([c0, c1, c2, (tag << 24) | (idx >> 2)],
                                       [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle_mod.word(seed, c0, c1, c2, tag, idx) == int(blk[idx & 3])


def test_bounded_edges(oracle_mod):
    b = oracle_mod.bounded
    for w in (0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF):
        assert b(w, 1) == 0
        assert b(w, 1 << 31) == w >> 1
    for n in (1, 2, 3, 7, 1000, 1 << 31, 0xFFFFFFFF):
        assert b(0, n) == 0
        assert b(0xFFFFFFFF, n) == n - 1
    assert b(0x80000000, 2) == 1 and b(0x7FFFFFFF, 2) == 0


def test_threshold_edges(oracle_mod):
    t = oracle_mod.threshold
    assert t(0.0) == 0
    assert t(1.0) == 1 << 32
    assert t(0.5) == 1 << 31
    assert t(0.25) == 1 << 30
    # 0.05 * 2^32 = 214748364.8 -> floor
    assert t(0.05) == 214748364
    assert t(2.0 ** -32) == 1
    assert t(2.0 ** -33) == 0


def test_bounded_uniformity(oracle_mod):
    n = 7
    counts = np.zeros(n, dtype=np.int64)
    for i in range(14000):
        counts[oracle_mod.bounded(oracle_mod.word(99, i, 0, 0, 1, i & 3), n)] += 1
    _, p = stats.chisquare(counts)
    assert p > 1e-4


def test_streams_differ_by_every_counter_field(oracle_mod):
    base = oracle_mod.word(1, 2, 3, 4, 1, 5)
    assert oracle_mod.word(2, 2, 3, 4, 1, 5) != base
    assert oracle_mod.word(1, 3, 3, 4, 1, 5) != base
    assert oracle_mod.word(1, 2, 4, 4, 1, 5) != base
    assert oracle_mod.word(1, 2, 3, 5, 1, 5) != base
    assert oracle_mod.word(1, 2, 3, 4, 2, 5) != base
    assert oracle_mod.word(1, 2, 3, 4, 1, 9) != base
