"""Pins of the oracle's island GA (PK-means GA, Alg. 2, Sec. 4.3) on the CPU.

- C = 1 is the panmictic GA bit for bit (one island holding every position).
- The population K-means: planted clusters are recovered, the result is a
  Lloyd fixed point (labels = nearest centroid, centroids = rounded member
  means), and the farthest-point start begins at the best-ranked chromosome.
- The island step: islands are independent (changing the chromosomes of the
  other islands does not change an island's next generation), each island's
  first positions hold its best members in rank order, and without mutation a
  child's rows come from its own island's members.
"""
import numpy as np
import pytest

from paper_2511_20511_amd import scenario


def _rand_pop(rng, n, L, K):
    return np.argsort(rng.random((n, L, K)), axis=2).astype(np.uint8)


def test_one_island_is_the_panmictic_ga(oracle_mod):
    d = scenario.make_drop(7, 4, seed=3, instance_id=1)
    args = (d.beta, d.user_xy, d.bs_xy, 40, 12, 2, 0.8, 0.05, 0.5, 0.1, 9, 1)
    b, bf, tr, pop = oracle_mod.solve(*args, T=196, want_pop=True)
    ib, ibf, itr, ipop, lab = oracle_mod.island_solve(*args, C=1, recluster_every=3, T=196)
    assert np.array_equal(b, ib) and bf == ibf
    assert np.array_equal(tr, itr) and np.array_equal(pop, ipop)
    assert np.all(lab == 0)


def test_planted_clusters_recovered(oracle_mod):
    """Two groups of near-copies of two distant chromosomes: K-means with C = 2
    separates them; label 0 is the group of the best-ranked chromosome."""
    rng = np.random.default_rng(2)
    L, K = 6, 8
    base0 = np.tile(np.arange(K, dtype=np.uint8), (L, 1))
    base1 = base0[:, ::-1].copy()
    pop, group = [], []
    for i in range(30):
        g = i % 2
        c = (base0 if g == 0 else base1).copy()
        for _ in range(2):  # two swaps in random rows
            j, a, b = rng.integers(L), rng.integers(K), rng.integers(K)
            c[j, a], c[j, b] = c[j, b], c[j, a]
        pop.append(c)
        group.append(g)
    pop = np.stack(pop)
    group = np.array(group)
    fit = rng.normal(size=30)
    labels, cent, it = oracle_mod.pop_kmeans(pop, fit, 2)
    best = int(np.argmax(fit))
    assert labels[best] == 0
    want = np.where(group == group[best], 0, 1)
    assert np.array_equal(labels, want)
    assert it >= 1


@pytest.mark.parametrize("C", [2, 3, 5])
def test_kmeans_fixed_point(oracle_mod, C):
    rng = np.random.default_rng(10 + C)
    L, K, N = 5, 6, 60
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(size=N)
    labels, cent, it = oracle_mod.pop_kmeans(pop, fit, C, max_iters=100)
    assert it < 100
    X = pop.reshape(N, -1).astype(np.int64)
    Cm = cent.reshape(C, -1).astype(np.int64)
    d = ((X[:, None, :] - Cm[None, :, :]) ** 2).sum(axis=2)
    assert np.array_equal(labels, np.argmin(d, axis=1))  # argmin takes the lowest on ties
    for c in range(C):
        m = labels == c
        if m.any():
            s = X[m].sum(axis=0)
            n = m.sum()
            assert np.array_equal(Cm[c], (2 * s + n) // (2 * n))


def test_farthest_point_start(oracle_mod):
    """With one Lloyd iteration the centroids are the means of the first
    assignment, made to the farthest-point start: the best chromosome and the
    chromosome farthest from it."""
    rng = np.random.default_rng(7)
    L, K, N = 3, 5, 20
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(size=N)
    labels, cent, _ = oracle_mod.pop_kmeans(pop, fit, 2, max_iters=1)
    X = pop.reshape(N, -1).astype(np.int64)
    c0 = X[int(np.argmax(fit))]
    d0 = ((X - c0) ** 2).sum(axis=1)
    c1 = X[int(np.argmax(d0))]  # argmax takes the lowest index on ties
    d = np.stack([d0, ((X - c1) ** 2).sum(axis=1)], axis=1)
    assert np.array_equal(labels, np.argmin(d, axis=1))


def _labels(rng, N, C):
    lab = rng.integers(0, C, size=N).astype(np.int32)
    lab[:C] = np.arange(C)  # every island non-empty
    return lab


def test_islands_are_independent(oracle_mod):
    rng = np.random.default_rng(5)
    L, K, N, C, E = 6, 8, 50, 4, 4
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(size=N)
    lab = _labels(rng, N, C)
    out = oracle_mod.island_step(pop, fit, lab, C, E, 0.8, 0.1, 21, 3, 7)
    for c in range(C):
        other = lab != c
        pop2, fit2 = pop.copy(), fit.copy()
        pop2[other] = _rand_pop(rng, int(other.sum()), L, K)
        fit2[other] = rng.normal(size=int(other.sum()))
        out2 = oracle_mod.island_step(pop2, fit2, lab, C, E, 0.8, 0.1, 21, 3, 7)
        assert np.array_equal(out[lab == c], out2[lab == c])


def test_island_elites_and_parents(oracle_mod):
    rng = np.random.default_rng(6)
    L, K, N, C, E = 5, 6, 48, 3, 6
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(size=N)
    lab = _labels(rng, N, C)
    out = oracle_mod.island_step(pop, fit, lab, C, E, 1.0, 0.0, 4, 0, 2)
    assert np.all(np.sort(out, axis=-1) == np.arange(K))
    total_e = 0
    for c in range(C):
        M = np.flatnonzero(lab == c)
        n = len(M)
        Ec = max(1, min(n, (2 * E * n + N) // (2 * N)))
        total_e += Ec
        order = M[np.lexsort((M, -fit[M]))]  # fitness descending, lower index first
        for e in range(Ec):
            assert np.array_equal(out[M[e]], pop[order[e]])
        # without mutation every child row is the same row of an island member
        for s in M[Ec:]:
            for j in range(L):
                assert any(np.array_equal(out[s, j], pop[m, j]) for m in M)
    assert total_e >= C


def test_island_solve_trace_never_decreases(oracle_mod):
    d = scenario.make_drop(7, 4, seed=8, instance_id=0)
    b, bf, tr, pop, lab = oracle_mod.island_solve(d.beta, d.user_xy, d.bs_xy, 60, 15, 5, 0.8,
                                                  0.05, 0.5, 0.1, 2, 0, C=5,
                                                  recluster_every=3, T=196)
    assert np.all(np.diff(tr) >= 0)
    assert set(np.unique(lab)) <= set(range(5))
    want = oracle_mod.fitness(d.beta, b[None], T=196)[0]
    assert want == bf
