"""FP64 CPU oracle for the K-means-seeded elitist 2D GA for pilot assignment.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(``paper_2511_20511_amd``) never does.  The oracle is plain single-threaded C
(``pa_oracle.c``) written from the paper, reached through ctypes with numpy
arrays.  It shares no code with the GPU library.

Every function below cites the passage of the paper it follows; the C source
states each reading where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "libpa_oracle.so")

SE_ASYMPTOTIC = 0
SE_FINITE_M = 1

TAG_SELECT = 0x01
TAG_MUT_DECIDE = 0x02
TAG_MUT_PARTNER = 0x03
TAG_INIT_DECIDE = 0x10
TAG_INIT_PARTNER = 0x11
TAG_INIT_SHUFFLE = 0x12


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, strict IEEE: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        f64p = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32, u32, u64, f64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.pao_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.pao_philox4x32_10.restype = None
        L.pao_word.argtypes = [u64, u32, u32, u32, u32, u32]
        L.pao_word.restype = u32
        L.pao_bounded.argtypes = [u32, u32]
        L.pao_bounded.restype = u32
        L.pao_threshold.argtypes = [f64]
        L.pao_threshold.restype = u64
        L.pao_fitness.argtypes = [i32, i32, i32, i32, f64, f64, f64p, u8p, i32, f64p]
        L.pao_fitness_obj.argtypes = [i32, i32, i32, i32, f64, f64, i32, f64p, u8p, i32, f64p]
        L.pao_se_terms.argtypes = [i32, i32, i32, f64, f64, f64p, u8p, f64p]
        L.pao_rank.argtypes = [f64p, i32, i32p]
        L.pao_kmeans_seed.argtypes = [i32, i32, f64p, f64p, u8p, i32p, i32p, i32p]
        L.pao_init_pop.argtypes = [i32, i32, i32, f64, f64, u64, u32, u8p, u8p]
        L.pao_ga_step.argtypes = [i32, i32, i32, i32, f64, f64, u64, u32, u32, u8p, f64p, u8p]
        L.pao_mutation_codes.argtypes = [i32, i32, f64, u64, u32, u32, u32, u8p]
        L.pao_pop_kmeans.argtypes = [i32, i32, i32, i32, u8p, f64p, i32, i32p, u8p, i32p]
        L.pao_island_step.argtypes = [i32, i32, i32, i32, i32, i32p, f64, f64, u64, u32, u32,
                                      u8p, f64p, u8p]
        L.pao_island_solve.argtypes = [i32, i32, i32, i32, f64, f64, f64p, f64p, f64p, i32, i32,
                                       i32, f64, f64, f64, f64, u64, u32, i32, i32, i32, u8p,
                                       f64p, f64p, u8p, i32p]
        L.pao_solve.argtypes = [i32, i32, i32, i32, f64, f64, f64p, f64p, f64p, i32, i32, i32,
                                f64, f64, f64, f64, u64, u32, u8p, f64p, f64p, u8p]
        L.pao_bruteforce.argtypes = [i32, i32, i32, i32, f64, f64, f64p, u8p, f64p, i64p]
        for name in ("pao_fitness", "pao_fitness_obj", "pao_se_terms", "pao_rank", "pao_kmeans_seed",
                     "pao_init_pop", "pao_ga_step", "pao_solve", "pao_bruteforce",
                     "pao_mutation_codes", "pao_pop_kmeans", "pao_island_step",
                     "pao_island_solve"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its input (rc={rc})")


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().pao_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def word(seed, c0, c1, c2, tag, idx):
    return int(lib().pao_word(seed, c0, c1, c2, tag, idx))


def bounded(w, n):
    return int(lib().pao_bounded(w, n))


def threshold(p):
    return int(lib().pao_threshold(p))


def fitness(beta, pop, T=0, se_mode=SE_ASYMPTOTIC, M=1, rho=1.0, objective=0):
    """Sum SE (Eq. 5-7) x pre-log (Sec. 3) of each chromosome, with objective 1
    the smallest per-user SINR (max-min SIR), with objective 2 minus the
    inter-cluster interference of Eq. 8; beta [L][L][K], pop [n][L][K]."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    L, L2, K = beta.shape
    assert L == L2
    pop = np.ascontiguousarray(pop, dtype=np.uint8).reshape(-1, L, K)
    n = pop.shape[0]
    fit = np.zeros(n, dtype=np.float64)
    rc = lib().pao_fitness_obj(L, K, T, se_mode, M, rho, int(objective),
                               _p(beta, ctypes.c_double), _p(pop, ctypes.c_uint8), n,
                               _p(fit, ctypes.c_double))
    _check(rc, "fitness")
    return fit


def se_terms(beta, chrom, se_mode=SE_ASYMPTOTIC, M=1, rho=1.0):
    """Per-user SE (Eq. 5) of one chromosome, [L][K]."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    L, _, K = beta.shape
    chrom = np.ascontiguousarray(chrom, dtype=np.uint8).reshape(L, K)
    se = np.zeros((L, K), dtype=np.float64)
    rc = lib().pao_se_terms(L, K, se_mode, M, rho, _p(beta, ctypes.c_double),
                            _p(chrom, ctypes.c_uint8), _p(se, ctypes.c_double))
    _check(rc, "se_terms")
    return se


def rank(fit):
    fit = np.ascontiguousarray(fit, dtype=np.float64)
    order = np.zeros(fit.shape[0], dtype=np.int32)
    lib().pao_rank(_p(fit, ctypes.c_double), fit.shape[0], _p(order, ctypes.c_int32))
    return order


def kmeans_seed(user_xy, bs_xy):
    """K-means seed chromosome (Sec. 4.1); returns (seed [L][K], centroids [K][2], labels [L*K], iters)."""
    user_xy = np.ascontiguousarray(user_xy, dtype=np.float64)
    bs_xy = np.ascontiguousarray(bs_xy, dtype=np.float64)
    L, K, _ = user_xy.shape
    seed = np.zeros((L, K), dtype=np.uint8)
    cent = np.zeros((K, 2), dtype=np.int32)
    labels = np.zeros(L * K, dtype=np.int32)
    iters = np.zeros(1, dtype=np.int32)
    rc = lib().pao_kmeans_seed(L, K, _p(user_xy, ctypes.c_double), _p(bs_xy, ctypes.c_double),
                               _p(seed, ctypes.c_uint8), _p(cent, ctypes.c_int32),
                               _p(labels, ctypes.c_int32), _p(iters, ctypes.c_int32))
    _check(rc, "kmeans_seed")
    return seed, cent, labels, int(iters[0])


def init_pop(L, K, N, kmeans_frac, p_init, seed, instance_id, seed_chrom=None):
    pop = np.zeros((N, L, K), dtype=np.uint8)
    sc = None if seed_chrom is None else np.ascontiguousarray(seed_chrom, dtype=np.uint8)
    rc = lib().pao_init_pop(L, K, N, kmeans_frac, p_init, seed, instance_id,
                            _p(sc, ctypes.c_uint8), _p(pop, ctypes.c_uint8))
    _check(rc, "init_pop")
    return pop


def mutation_codes(L, K, p_mut, seed, slot, gen, instance_id):
    """Mutation codes [L][K] of one child (k'+1 where gene (j, k) swaps with k', else 0):
    the per-gene mutation of the GA step (Sec. 6.1) with bit-sliced decision words."""
    out = np.zeros((L, K), dtype=np.uint8)
    rc = lib().pao_mutation_codes(L, K, float(p_mut), int(seed) & ((1 << 64) - 1),
                                  int(slot) & 0xFFFFFFFF, int(gen) & 0xFFFFFFFF,
                                  int(instance_id) & 0xFFFFFFFF, _p(out, ctypes.c_uint8))
    _check(rc, "mutation_codes")
    return out


def ga_step(pop, fit, E, p_cross, p_mut, seed, instance_id, gen):
    """One generation: elitism + tournament + row crossover + swap mutation."""
    pop = np.ascontiguousarray(pop, dtype=np.uint8)
    N, L, K = pop.shape
    fit = np.ascontiguousarray(fit, dtype=np.float64)
    out = np.zeros_like(pop)
    rc = lib().pao_ga_step(L, K, N, E, p_cross, p_mut, seed, instance_id, gen,
                           _p(pop, ctypes.c_uint8), _p(fit, ctypes.c_double),
                           _p(out, ctypes.c_uint8))
    _check(rc, "ga_step")
    return out


def solve(beta, user_xy, bs_xy, N, gens, E, p_cross, p_mut, kmeans_frac, p_init, seed,
          instance_id, T=0, se_mode=SE_ASYMPTOTIC, M=1, rho=1.0, want_pop=False):
    """Alg. 1 with a fixed number of generations; returns (best [L][K], best_fit, trace[gens+1][, pop])."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    L, _, K = beta.shape
    ux = None if user_xy is None else np.ascontiguousarray(user_xy, dtype=np.float64)
    bx = None if bs_xy is None else np.ascontiguousarray(bs_xy, dtype=np.float64)
    best = np.zeros((L, K), dtype=np.uint8)
    bf = np.zeros(1, dtype=np.float64)
    trace = np.zeros(gens + 1, dtype=np.float64)
    fpop = np.zeros((N, L, K), dtype=np.uint8) if want_pop else None
    rc = lib().pao_solve(L, K, T, se_mode, M, rho, _p(beta, ctypes.c_double),
                         _p(ux, ctypes.c_double), _p(bx, ctypes.c_double), N, gens, E,
                         p_cross, p_mut, kmeans_frac, p_init, seed, instance_id,
                         _p(best, ctypes.c_uint8), _p(bf, ctypes.c_double),
                         _p(trace, ctypes.c_double), _p(fpop, ctypes.c_uint8))
    _check(rc, "solve")
    if want_pop:
        return best, float(bf[0]), trace, fpop
    return best, float(bf[0]), trace


def pop_kmeans(pop, fit, C, max_iters=20):
    """K-means of a population into C islands (PK-means GA, Alg. 2): (labels [N],
    centroids [C][L][K], iterations)."""
    pop = np.ascontiguousarray(pop, dtype=np.uint8)
    N, L, K = pop.shape
    fit = np.ascontiguousarray(fit, dtype=np.float64)
    labels = np.zeros(N, dtype=np.int32)
    cent = np.zeros((C, L, K), dtype=np.uint8)
    it = np.zeros(1, dtype=np.int32)
    rc = lib().pao_pop_kmeans(L, K, N, C, _p(pop, ctypes.c_uint8), _p(fit, ctypes.c_double),
                              max_iters, _p(labels, ctypes.c_int32), _p(cent, ctypes.c_uint8),
                              _p(it, ctypes.c_int32))
    _check(rc, "pop_kmeans")
    return labels, cent, int(it[0])


def island_step(pop, fit, labels, C, E, p_cross, p_mut, seed, instance_id, gen):
    """One generation of every island (Alg. 2 loop body) for the given partition."""
    pop = np.ascontiguousarray(pop, dtype=np.uint8)
    N, L, K = pop.shape
    fit = np.ascontiguousarray(fit, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros_like(pop)
    rc = lib().pao_island_step(L, K, N, E, C, _p(labels, ctypes.c_int32), p_cross, p_mut,
                               int(seed) & ((1 << 64) - 1), instance_id & 0xFFFFFFFF,
                               gen & 0xFFFFFFFF, _p(pop, ctypes.c_uint8),
                               _p(fit, ctypes.c_double), _p(out, ctypes.c_uint8))
    _check(rc, "island_step")
    return out


def island_solve(beta, user_xy, bs_xy, N, gens, E, p_cross, p_mut, kmeans_frac, p_init, seed,
                 instance_id, C, recluster_every, max_iters=20, T=0, se_mode=SE_ASYMPTOTIC,
                 M=1, rho=1.0):
    """PK-means GA (Alg. 2): (best, best_fit, trace, final_pop, final_labels)."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    L, _, K = beta.shape
    ux = None if user_xy is None else np.ascontiguousarray(user_xy, dtype=np.float64)
    bx = None if bs_xy is None else np.ascontiguousarray(bs_xy, dtype=np.float64)
    best = np.zeros((L, K), dtype=np.uint8)
    bf = np.zeros(1, dtype=np.float64)
    trace = np.zeros(gens + 1, dtype=np.float64)
    fpop = np.zeros((N, L, K), dtype=np.uint8)
    flab = np.zeros(N, dtype=np.int32)
    rc = lib().pao_island_solve(L, K, T, se_mode, M, rho, _p(beta, ctypes.c_double),
                                _p(ux, ctypes.c_double), _p(bx, ctypes.c_double), N, gens, E,
                                p_cross, p_mut, kmeans_frac, p_init, seed, instance_id, C,
                                recluster_every, max_iters, _p(best, ctypes.c_uint8),
                                _p(bf, ctypes.c_double), _p(trace, ctypes.c_double),
                                _p(fpop, ctypes.c_uint8), _p(flab, ctypes.c_int32))
    _check(rc, "island_solve")
    return best, float(bf[0]), trace, fpop, flab


def bruteforce(beta, T=0, se_mode=SE_ASYMPTOTIC, M=1, rho=1.0):
    """Exhaustive search (EX-PA) over the K!^(L-1) classes; returns (best, best_fit, count)."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    L, _, K = beta.shape
    best = np.zeros((L, K), dtype=np.uint8)
    bf = np.zeros(1, dtype=np.float64)
    cnt = np.zeros(1, dtype=np.int64)
    rc = lib().pao_bruteforce(L, K, T, se_mode, M, rho, _p(beta, ctypes.c_double),
                              _p(best, ctypes.c_uint8), _p(bf, ctypes.c_double),
                              _p(cnt, ctypes.c_int64))
    _check(rc, "bruteforce")
    return best, float(bf[0]), int(cnt[0])
