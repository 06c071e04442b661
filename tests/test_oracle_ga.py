"""Pins of the oracle's K-means seeding, initial population, genetic operators
and solve (CPU only).

K-means: a hand-worked instance, the Lloyd fixed point, the single-cluster
case (the rounded mean).  Operators: invariants (rows stay permutations,
elites are bit copies in rank order), degenerate settings with known output
(E = N, p_cross = p_mut = 0), the binary-tournament win law
P(rank r) = (2(N-r)-1)/N^2, the mutation rate, the Fisher-Yates law.
Solve: reaches the exhaustive-search optimum on small instances."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from paper_2511_20511_amd import scenario


def _is_perm_rows(pop):
    K = pop.shape[-1]
    return np.all(np.sort(pop, axis=-1) == np.arange(K))


# ---------------------------------------------------------------- K-means

def test_kmeans_hand_worked(oracle_mod):
    """Two BSs 1 km apart, two users each.  Offsets (mm) from their own BS:
    cell 0: (0,0), (100,2); cell 1: (0,2), (100,0).  Farthest-point init picks
    (100,2) then (0,0); Lloyd moves them to (100,1) and (0,1) and stops; users
    at the same relative position get the same pilot: seed [[1,0],[1,0]]."""
    bs = np.array([[0.0, 0.0], [1000.0, 0.0]])
    users = np.array([[[0.0, 0.0], [0.1, 0.002]], [[1000.0, 0.002], [1000.1, 0.0]]])
    seed, cent, labels, iters = oracle_mod.kmeans_seed(users, bs)
    assert cent.tolist() == [[100, 1], [0, 1]]
    assert labels.tolist() == [1, 0, 1, 0]
    assert iters == 1
    assert seed.tolist() == [[1, 0], [1, 0]]


@pytest.mark.parametrize("L,K", [(7, 4), (19, 16), (5, 7)])
def test_kmeans_fixed_point(oracle_mod, L, K):
    drop = scenario.make_drop(L, K, seed=5, instance_id=K)
    seed, cent, labels, iters = oracle_mod.kmeans_seed(drop.user_xy, drop.bs_xy)
    assert _is_perm_rows(seed[None])
    assert iters < 100
    off = np.rint(1000.0 * (drop.user_xy - drop.bs_xy[:, None, :])).astype(np.int64).reshape(-1, 2)
    d = ((off[:, None, :] - cent[None, :, :].astype(np.int64)) ** 2).sum(-1)
    # labels are the nearest centroid (lowest index on ties)
    assert np.array_equal(labels, np.argmin(d, axis=1))
    # centroids are the rounded (half up) means of their members
    for c in range(K):
        m = off[labels == c]
        if len(m):
            for ax in range(2):
                want = math.floor(Fraction(int(m[:, ax].sum()), len(m)) + Fraction(1, 2))
                assert cent[c, ax] == want


def test_kmeans_single_cluster_is_rounded_mean(oracle_mod):
    bs = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0]])
    users = np.array([[[-0.0015, 0.003]], [[9.999, -0.001]], [[0.0, 10.0]]])
    seed, cent, labels, _ = oracle_mod.kmeans_seed(users, bs)
    # offsets in mm (half away from zero): (-2, 3), (-1, -1), (0, 0)
    # means: x = -3/3 = -1 -> -1 ; y = 2/3 -> 1
    assert cent.tolist() == [[-1, 1]]
    assert seed.tolist() == [[0], [0], [0]]


def test_kmeans_negative_half_rounds_up(oracle_mod):
    bs = np.array([[0.0, 0.0], [10.0, 0.0]])
    users = np.array([[[-0.002, 0.0]], [[10.0 - 0.001, 0.0]]])
    _, cent, _, _ = oracle_mod.kmeans_seed(users, bs)
    assert cent.tolist() == [[-1, 0]]   # mean -1.5 -> -1 (half up)


# ---------------------------------------------------------------- population init

def test_init_population_layout(oracle_mod):
    L, K, N = 7, 4, 50
    drop = scenario.make_drop(L, K, seed=1)
    seed_chrom = oracle_mod.kmeans_seed(drop.user_xy, drop.bs_xy)[0]
    pop = oracle_mod.init_pop(L, K, N, 0.5, 0.1, 1, 0, seed_chrom)
    assert _is_perm_rows(pop)
    assert np.array_equal(pop[0], seed_chrom)
    # individuals 1..24 derive from the seed: few genes differ
    diffs = [(pop[n] != seed_chrom).sum() for n in range(1, 25)]
    assert np.mean(diffs) < 0.5 * L * K
    pop0 = oracle_mod.init_pop(L, K, N, 0.0, 0.1, 1, 0, None)
    assert _is_perm_rows(pop0)
    # random part does not depend on whether a seed exists
    assert np.array_equal(pop0[25:], pop[25:])
    # n_km = max(1, floor(frac*N + 1/2)): a tiny fraction still keeps the seed
    pop1 = oracle_mod.init_pop(L, K, N, 1e-9, 0.1, 1, 0, seed_chrom)
    assert np.array_equal(pop1[0], seed_chrom) and np.array_equal(pop1[1:], pop0[1:])


def test_fisher_yates_uniform(oracle_mod):
    K, N = 3, 6000
    pop = oracle_mod.init_pop(1, K, N, 0.0, 0.0, 77, 3, None)
    code = pop[:, 0, 0].astype(int) * 9 + pop[:, 0, 1].astype(int) * 3 + pop[:, 0, 2]
    _, counts = np.unique(code, return_counts=True)
    assert len(counts) == 6
    _, p = stats.chisquare(counts)
    assert p > 1e-4


# ---------------------------------------------------------------- GA step

def _rand_pop(rng, n, L, K):
    return np.stack([np.stack([rng.permutation(K) for _ in range(L)]) for _ in range(n)]).astype(np.uint8)


def _rank(fit):
    idx = np.arange(len(fit))
    f = np.where(np.isnan(fit), -np.inf, fit)
    nan_last = np.isnan(fit).astype(int)
    return np.lexsort((idx, -f, nan_last))


def test_ranking_rule(oracle_mod):
    fit = np.array([1.0, 3.0, np.nan, 3.0, -np.inf, np.nan, 2.0, -0.0, 0.0])
    assert oracle_mod.rank(fit).tolist() == [1, 3, 6, 0, 7, 8, 4, 2, 5]
    assert oracle_mod.rank(fit).tolist() == _rank(fit).tolist()


@pytest.mark.parametrize("L,K,N,E", [(7, 4, 50, 2), (19, 16, 64, 8), (3, 5, 9, 0), (4, 3, 10, 3)])
def test_ga_step_invariants(oracle_mod, L, K, N, E):
    rng = np.random.default_rng(N)
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(100, 5, N)
    out = oracle_mod.ga_step(pop, fit, E, 0.8, 0.05, 42, 3, 9)
    assert _is_perm_rows(out)
    order = _rank(fit)
    for e in range(E):
        assert np.array_equal(out[e], pop[order[e]])
    # deterministic and keyed by generation
    assert np.array_equal(out, oracle_mod.ga_step(pop, fit, E, 0.8, 0.05, 42, 3, 9))
    assert not np.array_equal(out[E:], oracle_mod.ga_step(pop, fit, E, 0.8, 0.05, 42, 3, 10)[E:])


def test_all_elites_is_sorted_copy(oracle_mod):
    rng = np.random.default_rng(1)
    pop = _rand_pop(rng, 12, 5, 4)
    fit = rng.normal(0, 1, 12)
    fit[3] = fit[7]
    out = oracle_mod.ga_step(pop, fit, 12, 0.8, 0.5, 1, 0, 0)
    assert np.array_equal(out, pop[_rank(fit)])


def test_no_crossover_no_mutation_copies_winners(oracle_mod):
    """With p_cross = p_mut = 0 each child is a tournament winner; the winner
    of rank r (0 = best) appears with probability (2(N-r)-1)/N^2."""
    N, L, K = 16, 3, 4
    rng = np.random.default_rng(2)
    # distinct chromosomes: encode the index in row 0
    pop = _rand_pop(rng, N, L, K)
    fit = rng.permutation(N).astype(np.float64)
    order = _rank(fit)
    rank_of = np.empty(N, dtype=int)
    rank_of[order] = np.arange(N)
    keys = {pop[i].tobytes(): i for i in range(N)}
    assert len(keys) == N
    counts = np.zeros(N, dtype=np.int64)
    for g in range(600):
        out = oracle_mod.ga_step(pop, fit, 0, 0.0, 0.0, 5, 1, g)
        for c in range(N):
            counts[rank_of[keys[out[c].tobytes()]]] += 1
    r = np.arange(N)
    expect = counts.sum() * (2 * (N - r) - 1) / N ** 2
    _, p = stats.chisquare(counts, expect)
    assert p > 1e-4


def test_crossover_single_cut_on_cells(oracle_mod):
    N, L, K = 10, 6, 5
    rng = np.random.default_rng(3)
    pop = _rand_pop(rng, N, L, K)
    fit = rng.normal(0, 1, N)
    rows = {}
    for i in range(N):
        for j in range(L):
            rows.setdefault((j, pop[i, j].tobytes()), set()).add(i)
    for g in range(20):
        out = oracle_mod.ga_step(pop, fit, 0, 1.0, 0.0, 9, 0, g)
        for a in range(0, N, 2):
            src_a = [rows[(j, out[a, j].tobytes())] for j in range(L)]
            src_b = [rows[(j, out[a + 1, j].tobytes())] for j in range(L)]
            # some cut c in 1..L-1 explains both children with two parents
            ok = False
            for c in range(1, L):
                for p1 in src_a[0]:
                    for p2 in src_b[0]:
                        if all(p1 in src_a[j] for j in range(c)) and all(p2 in src_a[j] for j in range(c, L)) \
                                and all(p2 in src_b[j] for j in range(c)) and all(p1 in src_b[j] for j in range(c, L)):
                            ok = True
            assert ok


def test_mutation_rate(oracle_mod):
    """Each gene starts a swap with probability p_mut: about 2*p_mut*L*K genes change."""
    N, L, K, pm = 40, 8, 8, 0.02
    rng = np.random.default_rng(4)
    pop = np.tile(np.arange(K, dtype=np.uint8), (N, L, 1))
    fit = np.zeros(N)
    changed = []
    for g in range(50):
        out = oracle_mod.ga_step(pop, fit, 0, 0.0, pm, 11, 0, g)
        changed.append((out != pop).sum(axis=(1, 2)))
    changed = np.concatenate(changed)
    # one swap changes two genes (rarely fewer when swaps overlap)
    assert abs(changed.mean() - 2 * pm * L * K) < 0.15
    assert _is_perm_rows(out)


def test_odd_children_and_degenerate_sizes(oracle_mod):
    rng = np.random.default_rng(5)
    pop = _rand_pop(rng, 7, 1, 1)  # L = K = 1: nothing can change
    out = oracle_mod.ga_step(pop, rng.normal(size=7), 2, 1.0, 1.0, 1, 0, 0)
    assert np.all(out == 0)
    pop = _rand_pop(rng, 8, 4, 3)
    out = oracle_mod.ga_step(pop, rng.normal(size=8), 3, 0.8, 0.1, 1, 0, 0)  # N - E = 5, odd
    assert _is_perm_rows(out)


# ---------------------------------------------------------------- solve

def test_solve_reaches_exhaustive_optimum(oracle_mod):
    """L = 3, K = 3 (36 classes): the GA with N = 50, G = 100 finds the optimum
    class on at least 99 of 100 drops."""
    hits = 0
    for inst in range(100):
        drop = scenario.make_drop(3, 3, seed=2024, instance_id=inst)
        _, opt, _ = oracle_mod.bruteforce(drop.beta)
        best, bf, trace = oracle_mod.solve(drop.beta, drop.user_xy, drop.bs_xy, 50, 100, 2,
                                           0.8, 0.05, 0.5, 0.1, 1, inst)
        assert bf <= opt * (1 + 1e-12)
        hits += bf >= opt * (1 - 1e-12)
    assert hits >= 99


def test_solve_trace_and_result(oracle_mod):
    drop = scenario.make_drop(7, 4, seed=1)
    rho = scenario.snr_to_rho(10.0)
    best, bf, trace, pop = oracle_mod.solve(drop.beta, drop.user_xy, drop.bs_xy, 50, 30, 2, 0.8,
                                            0.05, 0.5, 0.1, 1, 0, T=196, want_pop=True)
    assert np.all(np.diff(trace) >= 0)            # elitism keeps the best
    assert trace[-1] == bf
    assert oracle_mod.fitness(drop.beta, best[None], T=196)[0] == bf
    assert _is_perm_rows(pop)
    # the random-init GA (kmeans_frac = 0) needs no positions
    _, bf0, _ = oracle_mod.solve(drop.beta, None, None, 50, 30, 2, 0.8, 0.05, 0.0, 0.1, 1, 0, T=196)
    assert bf0 > 0
    # finite-M mode runs through the same loop
    _, bfm, tm = oracle_mod.solve(drop.beta, drop.user_xy, drop.bs_xy, 20, 5, 2, 0.8, 0.05, 0.5,
                                  0.1, 1, 0, T=196, se_mode=oracle_mod.SE_FINITE_M, M=128, rho=rho)
    assert np.all(np.diff(tm) >= 0) and bfm > 0


# ---------------------------------------------------------------- mutation draws

def _group_words(oracle_mod, seed, slot, gen, inst, tag, q, n=32):
    return [oracle_mod.word(seed, slot, gen, inst, tag, 32 * q + k) for k in range(n)]


@pytest.mark.parametrize("L,K", [(8, 8), (5, 7), (3, 32)])
def test_mutation_decisions_at_dyadic_rates(oracle_mod, L, K):
    """At p = 1/2, 1/4 and 3/4 the comparison 'decision word < thr' reads only
    the first one or two bits of the word, so the mutating genes of group q
    are fixed by the first words of the group: ~R0 (1/2), ~R0 & ~R1 (1/4),
    ~(R0 & R1) (3/4), bit b for gene 32q + b.  A reversed bit order, a wrong
    word index or a wrong gene-to-bit map fails this."""
    LK = L * K
    for p, rule in ((0.5, lambda r0, r1: ~r0), (0.25, lambda r0, r1: ~r0 & ~r1),
                    (0.75, lambda r0, r1: ~(r0 & r1))):
        for slot in range(3):
            codes = oracle_mod.mutation_codes(L, K, p, 77, slot, 5, 2).reshape(-1)
            for q in range((LK + 31) // 32):
                r0, r1 = _group_words(oracle_mod, 77, slot, 5, 2, oracle_mod.TAG_MUT_DECIDE, q, 2)
                m = rule(r0, r1) & 0xFFFFFFFF
                for b in range(min(32, LK - 32 * q)):
                    assert (codes[32 * q + b] != 0) == bool((m >> b) & 1), (p, slot, q, b)


def test_mutation_partners_by_hit_rank(oracle_mod):
    """The h-th mutating gene of group q swaps with the user drawn from word
    32q + h of the partner stream (r = bounded(word, K-1), k' = r + (r >= k)):
    at p = 1 every gene mutates (h = b), at p = 1/2 the hits are counted."""
    L, K = 4, 12
    for p in (1.0, 0.5):
        codes = oracle_mod.mutation_codes(L, K, p, 9, 3, 1, 0).reshape(-1)
        for q in range((L * K + 31) // 32):
            h = 0
            for b in range(min(32, L * K - 32 * q)):
                i = 32 * q + b
                if codes[i] == 0:
                    continue
                w = oracle_mod.word(9, 3, 1, 0, oracle_mod.TAG_MUT_PARTNER, 32 * q + h)
                r = oracle_mod.bounded(w, K - 1)
                k = i % K
                assert codes[i] == r + (1 if r >= k else 0) + 1
                h += 1
            if p == 1.0:
                assert h == min(32, L * K - 32 * q)


def test_mutation_law(oracle_mod):
    """The per-gene decisions are independent Bernoulli(p) events: each of the
    32 bit positions of a group mutates at rate p (chi-square), the gaps
    between consecutive mutating genes of a child follow the geometric law
    P(gap = g) = (1-p)^g p (chi-square), and neighbouring genes are
    uncorrelated."""
    L, K, p, n = 8, 8, 0.05, 6000
    hits = np.stack([oracle_mod.mutation_codes(L, K, p, 123, s, 7, 1).reshape(-1) != 0
                     for s in range(n)])
    # rate per bit position (genes b and 32 + b share bit b)
    pos = hits.reshape(n, 2, 32).sum(axis=(0, 1))
    exp = 2 * n * p
    chi = ((pos - exp) ** 2 / (exp * (1 - p))).sum()
    assert stats.chi2.sf(chi, 31) > 1e-3
    # gaps between consecutive hits inside a child
    gaps = np.concatenate([np.diff(np.flatnonzero(h)) - 1 for h in hits])
    G = 12
    obs = np.array([np.sum(gaps == g) for g in range(G)] + [np.sum(gaps >= G)])
    # the gap law conditioned on the next hit falling inside the 64 genes is
    # not exactly geometric; compare with the same statistic simulated with
    # one independent Bernoulli(p) per gene
    rng = np.random.default_rng(1)
    sim = rng.random((20 * n, L * K)) < p
    sg = np.concatenate([np.diff(np.flatnonzero(h)) - 1 for h in sim])
    ref = np.array([np.sum(sg == g) for g in range(G)] + [np.sum(sg >= G)], dtype=float)
    ref = ref / ref.sum() * obs.sum()
    chi = ((obs - ref) ** 2 / ref).sum()
    assert stats.chi2.sf(chi, G) > 1e-3
    # the geometric head of the law: P(gap = 0) / P(gap = 1) = 1 / (1 - p)
    assert abs(obs[0] / obs[1] - 1 / (1 - p)) < 0.1
    # neighbouring genes independent
    a, b = hits[:, :-1].reshape(-1), hits[:, 1:].reshape(-1)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.02
