"""Seeded synthetic drops for the multi-cell massive-MIMO uplink (inputs only).

This module produces the inputs both the GPU library and the test oracle
consume; it holds none of the pilot-assignment method's arithmetic.

System model (Sec. 3.1): L cells, one BS per cell, K single-antenna users per
cell; the large-scale fading of user k of cell j at BS l is
beta[l][j][k] = z / d^alpha (Eq. 2) with log-normal shadowing z.  The paper
gives neither alpha, the shadowing spread nor the layout, so the drops use a
hexagonal grid of pointy-top cells of circumradius R = 500 m numbered ring by
ring (1, 7, 19, 37, 61 cells fill 0..4 rings), the BS at each centre, users
uniform over their hexagon at least 35 m from the BS, alpha = 3.8, 8 dB
shadowing drawn i.i.d. per (BS, user) link, and no wrap-around.

Random numbers come from numpy's SeedSequence keyed by (seed, instance, tag),
so a drop is a pure function of (L, K, seed, instance_id).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

RADIUS_M = 500.0
MIN_DIST_M = 35.0
ALPHA = 3.8
SHADOW_DB = 8.0

_TAG_POS, _TAG_SHADOW, _TAG_SIZE, _TAG_ARRIVAL = 0x20, 0x21, 0x22, 0x23


def _rng(seed: int, instance_id: int, tag: int) -> np.random.Generator:
    seed = int(seed) & ((1 << 64) - 1)
    return np.random.default_rng(
        np.random.SeedSequence([seed & 0xFFFFFFFF, seed >> 32, int(instance_id) & 0xFFFFFFFF, tag]))


def hex_centres(L: int, radius: float = RADIUS_M) -> np.ndarray:
    """Centres [L][2] of the first L pointy-top hexagons, spiralling out ring by ring."""
    dirs = [(1, 0), (1, -1), (0, -1), (-1, 0), (-1, 1), (0, 1)]
    axial = [(0, 0)]
    ring = 1
    while len(axial) < L:
        q, r = -ring, ring  # start of ring `ring`: `ring` steps along direction 4
        for d in range(6):
            for _ in range(ring):
                axial.append((q, r))
                q, r = q + dirs[d][0], r + dirs[d][1]
        ring += 1
    out = np.zeros((L, 2), dtype=np.float64)
    for i in range(L):
        q, r = axial[i]
        out[i, 0] = radius * math.sqrt(3.0) * (q + r / 2.0)
        out[i, 1] = radius * 1.5 * r
    return out


def _in_hex(x: np.ndarray, y: np.ndarray, radius: float) -> np.ndarray:
    ax, ay = np.abs(x), np.abs(y)
    return (ax <= radius * math.sqrt(3.0) / 2.0) & (ay <= radius - ax / math.sqrt(3.0))


@dataclass
class Drop:
    beta: np.ndarray      # [L][L][K] float64, beta[l][j][k]
    user_xy: np.ndarray   # [L][K][2] float64 metres
    bs_xy: np.ndarray     # [L][2] float64 metres
    L: int
    K: int

    @property
    def tau(self) -> int:
        return self.K


def make_drop(L: int, K: int, seed: int = 1, instance_id: int = 0, radius: float = RADIUS_M,
              min_dist: float = MIN_DIST_M, alpha: float = ALPHA,
              shadow_db: float = SHADOW_DB) -> Drop:
    """One user drop and its large-scale fading table (Eq. 2)."""
    bs = hex_centres(L, radius)
    rng = _rng(seed, instance_id, _TAG_POS)
    users = np.zeros((L, K, 2), dtype=np.float64)
    half_w = radius * math.sqrt(3.0) / 2.0
    for j in range(L):
        got = 0
        while got < K:
            m = 4 * (K - got) + 8
            x = rng.uniform(-half_w, half_w, m)
            y = rng.uniform(-radius, radius, m)
            ok = _in_hex(x, y, radius) & (np.hypot(x, y) >= min_dist)
            x, y = x[ok], y[ok]
            take = min(K - got, x.shape[0])
            users[j, got:got + take, 0] = bs[j, 0] + x[:take]
            users[j, got:got + take, 1] = bs[j, 1] + y[:take]
            got += take
    d = np.linalg.norm(users[None, :, :, :] - bs[:, None, None, :], axis=-1)  # [l][j][k]
    shadow = _rng(seed, instance_id, _TAG_SHADOW).standard_normal((L, L, K))
    beta = np.power(10.0, shadow_db * shadow / 10.0) * np.power(d, -alpha)
    return Drop(beta=np.ascontiguousarray(beta), user_xy=users, bs_xy=bs, L=L, K=K)


def snr_to_rho(snr_db: float, radius: float = RADIUS_M, alpha: float = ALPHA) -> float:
    """Transmit SNR such that an unshadowed user at the cell edge is received at `snr_db`."""
    return 10.0 ** (snr_db / 10.0) * radius ** alpha


def size_mix(n: int, seed: int = 1) -> list[tuple[int, int, int]]:
    """(L, K, N) of n uneven instances: L from {7, 19, 37}, K in [4, 32], N in [128, 1024]."""
    out = []
    for i in range(n):
        r = _rng(seed, i, _TAG_SIZE)
        L = (7, 19, 37)[int(r.integers(0, 3))]
        K = int(r.integers(4, 33))
        N = int(r.integers(128, 1025))
        out.append((L, K, N))
    return out


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int = 1) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate over [0, duration)."""
    r = _rng(seed, 0, _TAG_ARRIVAL)
    n_guess = int(rate_per_s * duration_s * 1.2) + 16
    t = np.cumsum(r.exponential(1.0 / rate_per_s, n_guess))
    while t[-1] < duration_s:
        t = np.concatenate([t, t[-1] + np.cumsum(r.exponential(1.0 / rate_per_s, n_guess))])
    return t[t < duration_s]


# Workloads with the sizes used throughout the tests and the benchmark.
WORKLOADS = {
    "single_L7_K4": dict(L=7, K=4, M=128, T=196, snr_db=10.0, N=50, gens=100, E=2,
                         p_cross=0.8, p_mut=0.05, kmeans_frac=0.5, p_init=0.1, seed=1, instances=1),
    "single_L19_K16": dict(L=19, K=16, M=256, T=196, snr_db=10.0, N=256, gens=500, E=8,
                           p_cross=0.8, p_mut=0.05, kmeans_frac=0.5, p_init=0.1, seed=1,
                           instances=1),
    "batch64_L37_K32": dict(L=37, K=32, M=256, T=196, snr_db=10.0, N=1024, gens=200, E=8,
                            p_cross=0.8, p_mut=0.05, kmeans_frac=0.5, p_init=0.1, seed=1,
                            instances=64),
    # uneven sizes from size_mix (L in {7, 19, 37}, K in [4, 32], N in [128, 1024])
    "batch512_mix": dict(mix=True, M=256, T=196, snr_db=10.0, gens=200, E=8, p_cross=0.8,
                         p_mut=0.05, kmeans_frac=0.5, p_init=0.1, seed=1, instances=512),
    # Poisson arrivals of size_mix solves with 50 generations each
    "serve_mix_2000rps": dict(mix=True, M=256, T=196, snr_db=10.0, gens=50, E=8, p_cross=0.8,
                              p_mut=0.05, kmeans_frac=0.5, p_init=0.1, seed=1, rate=2000.0,
                              pool=64),
}
