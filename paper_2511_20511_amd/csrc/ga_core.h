// ga_core.h -- device code of the genetic operators (Alg. 1 loop body):
// elitism, binary-tournament selection, single-point crossover on the cell
// axis, per-gene swap mutation.  Every random decision is a Philox word
// keyed by (seed; slot, generation, instance, stream tag), so a child depends
// only on (parents' bits, fitness ranking, seed, instance, generation, slot).
#pragma once
#include "pa_dev.h"
#include "pa_internal.h"

namespace pa {

// Swap mutation of the rows held in `buf` (LDS, row-major L x K bytes): gene
// i = j*K + k mutates when decision word i is below thr and then swaps with
// user k' != k of the same row, k' from partner word i.  Rows are processed
// one lane each, genes of a row in increasing k against the current row.
__device__ __forceinline__ void mutate_rows(uint8_t *buf, int L, int K, const Stream &dec,
                                            const Stream &par, uint64_t thr, int lane) {
  if (K < 2 || thr == 0) return;
  for (int j = lane; j < L; j += kWave) {
    uint8_t *row = buf + j * K;
    uint32_t cur = 0xFFFFFFFFu;
    Words4 wb{0, 0, 0, 0};
    for (int k = 0; k < K; ++k) {
      const uint32_t i = (uint32_t)(j * K + k);
      if ((i >> 2) != cur) {
        cur = i >> 2;
        wb = dec.block(cur);
      }
      if (hit(pick(wb, i & 3u), thr)) {
        const uint32_t r = bounded(par.word(i), (uint32_t)(K - 1));
        const int kp = (int)r + ((int)r >= k ? 1 : 0);
        const uint8_t t = row[k];
        row[k] = row[kp];
        row[kp] = t;
      }
    }
  }
}

// Fisher-Yates shuffle from the identity of every row, one lane per row:
// for k = K-1 .. 1, r = bounded(word[j*K + k], k + 1), swap(row[k], row[r]).
__device__ __forceinline__ void shuffle_rows(uint8_t *buf, int L, int K, const Stream &shf,
                                             int lane) {
  for (int j = lane; j < L; j += kWave) {
    uint8_t *row = buf + j * K;
    for (int k = 0; k < K; ++k) row[k] = (uint8_t)k;
    uint32_t cur = 0xFFFFFFFFu;
    Words4 wb{0, 0, 0, 0};
    for (int k = K - 1; k >= 1; --k) {
      const uint32_t i = (uint32_t)(j * K + k);
      if ((i >> 2) != cur) {
        cur = i >> 2;
        wb = shf.block(cur);
      }
      const int r = (int)bounded(pick(wb, i & 3u), (uint32_t)(k + 1));
      const uint8_t t = row[k];
      row[k] = row[r];
      row[r] = t;
    }
  }
}

// Parents and cut of the child in slot s (pairs (a, a+1) share their six
// SELECT words, keyed by slot a).  Lanes 0 and 1 compute the two Philox
// blocks, every lane gets all words.
struct Pairing {
  uint32_t p1, p2;  // parents: child a takes rows [0, cut) of p1, the rest of p2
  int cut;          // L when there is no crossover
};

__device__ __forceinline__ Pairing select_parents(const float *__restrict__ fin, int N, int L,
                                                  const DevGa &ga, uint32_t gen, int pair_a,
                                                  int lane) {
  const Stream sel{ga.seed_lo, ga.seed_hi, (uint32_t)pair_a, gen, ga.instance_id, kTagSelect};
  const Words4 b = sel.block((uint32_t)(lane & 1));
  const uint32_t w0 = __shfl(b.x, 0), w1 = __shfl(b.y, 0), w2 = __shfl(b.z, 0),
                 w3 = __shfl(b.w, 0), w4 = __shfl(b.x, 1), w5 = __shfl(b.y, 1);
  const uint32_t u0 = bounded(w0, (uint32_t)N), v0 = bounded(w1, (uint32_t)N);
  const uint32_t u1 = bounded(w2, (uint32_t)N), v1 = bounded(w3, (uint32_t)N);
  const uint32_t ku0 = rank_key(fin[u0]), kv0 = rank_key(fin[v0]);
  const uint32_t ku1 = rank_key(fin[u1]), kv1 = rank_key(fin[v1]);
  Pairing pr;
  pr.p1 = beats(kv0, v0, ku0, u0) ? v0 : u0;
  pr.p2 = beats(kv1, v1, ku1, u1) ? v1 : u1;
  const bool cross = L >= 2 && hit(w4, ga.thr_cross);
  pr.cut = cross ? 1 + (int)bounded(w5, (uint32_t)(L - 1)) : L;
  return pr;
}

// Indices of the E best (E <= 64) into idx[0..E) by repeated arg-max over keys
// strictly below the previous maximum (keys are unique: they embed the index).
__device__ __forceinline__ void top_e_wave(const float *__restrict__ fin, int N, int E,
                                           int32_t *idx, int lane) {
  uint64_t prev = ~0ull;
  for (int e = 0; e < E; ++e) {
    uint64_t best = 0;
    for (int i = lane; i < N; i += kWave) {
      const uint64_t k = full_key(fin[i], (uint32_t)i);
      if (k < prev && k > best) best = k;
    }
    best = wave_max_u64(best);
    if (lane == 0) idx[e] = (int32_t)key_index(best);
    prev = best;
  }
}

// Rank of chromosome i = number of chromosomes that beat it (E > 64 path).
__device__ __forceinline__ int rank_of(const float *__restrict__ fin, int N, int i) {
  const uint32_t ki = rank_key(fin[i]);
  int r = 0;
  for (int m = 0; m < N; ++m) {
    const uint32_t km = rank_key(fin[m]);
    r += beats(km, (uint32_t)m, ki, (uint32_t)i) ? 1 : 0;
  }
  return r;
}

}  // namespace pa
