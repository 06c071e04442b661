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
// Populations up to 2048 keep their keys in registers (32 per lane).
__device__ __forceinline__ void top_e_wave(const float *__restrict__ fin, int N, int E,
                                           int32_t *idx, int lane) {
  constexpr int kCached = 32;
  if (N <= kCached * kWave) {
    uint32_t kk[kCached];
#pragma unroll
    for (int u = 0; u < kCached; ++u) {
      const int i = lane + u * kWave;
      kk[u] = i < N ? rank_key(fin[i]) : 0u;
    }
    uint64_t prev = ~0ull;
    for (int e = 0; e < E; ++e) {
      uint64_t best = 0;
#pragma unroll
      for (int u = 0; u < kCached; ++u) {
        const int i = lane + u * kWave;
        const uint64_t k = ((uint64_t)kk[u] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
        if (i < N && k < prev && k > best) best = k;
      }
      best = wave_max_u64(best);
      if (lane == 0) idx[e] = (int32_t)key_index(best);
      prev = best;
    }
    return;
  }
  uint64_t prev = ~0ull;
  for (int e = 0; e < E; ++e) {
    uint64_t best = 0;
    for (int i0 = lane; i0 < N; i0 += 8 * kWave) {
      float f[8];  // eight loads in flight per lane
#pragma unroll
      for (int u = 0; u < 8; ++u) f[u] = fin[min(i0 + u * kWave, N - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u * kWave;
        const uint64_t k = full_key(f[u], (uint32_t)i);
        if (i < N && k < prev && k > best) best = k;
      }
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

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Builds the child of slot `slot` (generation `gen`) in the wave's LDS buffer
// `child` (L*K bytes), using `hit` (L*K bytes of LDS) for the mutation
// decisions: lanes over genes copy the parents' rows, all lanes draw the
// decision words (4 genes per Philox block), then one lane per row applies
// the swaps in increasing k.  Ends with the child complete in LDS.
__device__ __forceinline__ void build_child(const uint8_t *__restrict__ pin,
                                            const float *__restrict__ fin, int N, int E, int L,
                                            int K, const DevGa &ga, uint32_t gen, int slot,
                                            uint8_t *child, uint8_t *hits, int lane) {
  const int LK = L * K;
  const int pair_a = E + ((slot - E) & ~1);
  const bool second = ((slot - E) & 1) != 0;
  const Pairing pr = select_parents(fin, N, L, ga, gen, pair_a, lane);
  const uint8_t *first = pin + (size_t)(second ? pr.p2 : pr.p1) * LK;
  const uint8_t *rest = pin + (size_t)(second ? pr.p1 : pr.p2) * LK;
  const int cutg = pr.cut * K;
  for (int i = lane; i < LK; i += kWave) child[i] = i < cutg ? first[i] : rest[i];
  const bool mutate = K >= 2 && ga.thr_mut != 0;
  if (mutate) {
    const Stream dec{ga.seed_lo, ga.seed_hi, (uint32_t)slot, gen, ga.instance_id, kTagMutDecide};
    const int nb = (LK + 3) >> 2;
    for (int b = lane; b < nb; b += kWave) {
      const Words4 w = dec.block((uint32_t)b);
      const int i = 4 * b;
      hits[i] = hit(w.x, ga.thr_mut);
      if (i + 1 < LK) hits[i + 1] = hit(w.y, ga.thr_mut);
      if (i + 2 < LK) hits[i + 2] = hit(w.z, ga.thr_mut);
      if (i + 3 < LK) hits[i + 3] = hit(w.w, ga.thr_mut);
    }
  }
  wave_sync();
  if (mutate) {
    const Stream par{ga.seed_lo, ga.seed_hi, (uint32_t)slot, gen, ga.instance_id, kTagMutPartner};
    for (int j = lane; j < L; j += kWave) {
      uint8_t *row = child + j * K;
      const uint8_t *h = hits + j * K;
      uint32_t cur = 0xFFFFFFFFu;
      Words4 wb{0, 0, 0, 0};
      for (int k = 0; k < K; ++k) {
        if (!h[k]) continue;
        const uint32_t i = (uint32_t)(j * K + k);
        if ((i >> 2) != cur) {
          cur = i >> 2;
          wb = par.block(cur);
        }
        const uint32_t r = bounded(pick(wb, i & 3u), (uint32_t)(K - 1));
        const int kp = (int)r + ((int)r >= k ? 1 : 0);
        const uint8_t t = row[k];
        row[k] = row[kp];
        row[kp] = t;
      }
    }
  }
  wave_sync();
}

// Elitism by one wave: slots 0..E-1 of pout receive the E best chromosomes
// of pin in rank order (and fout their fitness, when given); trace (when
// given) receives the best fitness at index gen.  idx: 64 ints of LDS.
__device__ __forceinline__ void copy_elites(const uint8_t *__restrict__ pin,
                                            const float *__restrict__ fin, int N, int E, int LK,
                                            uint8_t *__restrict__ pout, float *fout, float *trace,
                                            int gen, int32_t *idx, int lane) {
  if (E < 64) {
    const int Ek = E > 1 ? E : 1;
    top_e_wave(fin, N, Ek, idx, lane);
    wave_sync();
    if (trace && lane == 0) trace[gen] = fin[idx[0]];
    for (int e = 0; e < E; ++e) {
      const int src = idx[e];
      for (int i = lane; i < LK; i += kWave) pout[(size_t)e * LK + i] = pin[(size_t)src * LK + i];
      if (fout && lane == 0) fout[e] = fin[src];
    }
  } else {
    // E >= 64: every lane ranks its chromosomes by counting who beats them
    for (int i = lane; i < N; i += kWave) {
      const int r = rank_of(fin, N, i);
      if (r == 0 && trace) trace[gen] = fin[i];
      if (r < E) {
        for (int g = 0; g < LK; ++g) pout[(size_t)r * LK + g] = pin[(size_t)i * LK + g];
        if (fout) fout[r] = fin[i];
      }
    }
  }
}

// Builds the children of slots [s0, s0 + nc) in LDS (child c at child +
// c*L*K) with the whole workgroup, in phases separated by barriers:
//   1. one thread per child: its pair's six SELECT words, two tournaments,
//      crossover decision and cut;
//   2. all threads over all genes: copy from the parents;
//      all threads over all (child, Philox block): mutation decisions;
//   3. one thread per (child, row): the swaps, in increasing k.
// Each phase costs about one global-memory round trip however many children
// the workgroup builds.  sSel: 2 ints per child.  Ends with a barrier.
__device__ __forceinline__ void build_children_block(const uint8_t *__restrict__ pin,
                                                     const float *__restrict__ fin, int N, int E,
                                                     int L, int K, const DevGa &ga, uint32_t gen,
                                                     int s0, int nc, uint8_t *child,
                                                     uint8_t *hits, int32_t *sSel, int block) {
  const int LK = L * K;
  const int tid = threadIdx.x;
  for (int c = tid; c < nc; c += block) {
    const int slot = s0 + c;
    const int pair_a = E + ((slot - E) & ~1);
    const bool second = ((slot - E) & 1) != 0;
    const Stream sel{ga.seed_lo, ga.seed_hi, (uint32_t)pair_a, gen, ga.instance_id, kTagSelect};
    const Words4 b0 = sel.block(0u), b1 = sel.block(1u);
    const uint32_t u0 = bounded(b0.x, (uint32_t)N), v0 = bounded(b0.y, (uint32_t)N);
    const uint32_t u1 = bounded(b0.z, (uint32_t)N), v1 = bounded(b0.w, (uint32_t)N);
    const uint32_t p1 = beats(rank_key(fin[v0]), v0, rank_key(fin[u0]), u0) ? v0 : u0;
    const uint32_t p2 = beats(rank_key(fin[v1]), v1, rank_key(fin[u1]), u1) ? v1 : u1;
    const bool cross = L >= 2 && hit(b1.x, ga.thr_cross);
    const int cut = cross ? 1 + (int)bounded(b1.y, (uint32_t)(L - 1)) : L;
    const uint32_t first = second ? p2 : p1, rest = second ? p1 : p2;
    sSel[2 * c] = (int32_t)(first | (rest << 16));
    sSel[2 * c + 1] = cut * K;
  }
  __syncthreads();
  // child c = first parent's genes [0, cut) + second's [cut, LK): two byte
  // ranges per child, moved as aligned words, several loads in flight
  {
    const int ws = (LK >> 2) + 2;  // words of a range, upper bound
    const int items = nc * 2 * ws;
    for (int i0 = tid; i0 < items; i0 += kCopyBatch * block) {
      uint32_t v[kCopyBatch];
#pragma unroll
      for (int u = 0; u < kCopyBatch; ++u) {
        const int i = i0 + u * block;
        const int c = i / (2 * ws), rr = (i / ws) & 1, w = i % ws;
        const uint32_t pr = (uint32_t)sSel[2 * (c < nc ? c : 0)];
        const int cutg = sSel[2 * (c < nc ? c : 0) + 1];
        const ByteRange r = rr == 0 ? ByteRange{pin + (size_t)(pr & 0xFFFFu) * LK, cutg}
                                    : ByteRange{pin + (size_t)(pr >> 16) * LK + cutg, LK - cutg};
        const bool ok = i < items && r.n > 0 && w < r.words();
        v[u] = ok ? r.load(w) : 0u;
      }
#pragma unroll
      for (int u = 0; u < kCopyBatch; ++u) {
        const int i = i0 + u * block;
        const int c = i / (2 * ws), rr = (i / ws) & 1, w = i % ws;
        if (i < items) {
          const uint32_t pr = (uint32_t)sSel[2 * c];
          const int cutg = sSel[2 * c + 1];
          const ByteRange r = rr == 0 ? ByteRange{pin + (size_t)(pr & 0xFFFFu) * LK, cutg}
                                      : ByteRange{pin + (size_t)(pr >> 16) * LK + cutg, LK - cutg};
          uint8_t *dst = child + c * LK + (rr == 0 ? 0 : cutg);
          if (r.n > 0 && w < r.words()) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int g = r.pos(w, b);
              if (g >= 0 && g < r.n) dst[g] = (uint8_t)(v[u] >> (8 * b));
            }
          }
        }
      }
    }
  }
  const bool mutate = K >= 2 && ga.thr_mut != 0;
  if (mutate) {
    const int nb = (LK + 3) >> 2;
    for (int i = tid; i < nc * nb; i += block) {
      const int c = i / nb, b = i - c * nb;
      const Stream dec{ga.seed_lo, ga.seed_hi, (uint32_t)(s0 + c), gen, ga.instance_id,
                       kTagMutDecide};
      const Words4 w = dec.block((uint32_t)b);
      uint8_t *h = hits + c * LK + 4 * b;
      const int g = 4 * b;
      h[0] = hit(w.x, ga.thr_mut);
      if (g + 1 < LK) h[1] = hit(w.y, ga.thr_mut);
      if (g + 2 < LK) h[2] = hit(w.z, ga.thr_mut);
      if (g + 3 < LK) h[3] = hit(w.w, ga.thr_mut);
    }
  }
  __syncthreads();
  if (mutate) {
    for (int i = tid; i < nc * L; i += block) {
      const int c = i / L, j = i - c * L;
      const Stream par{ga.seed_lo, ga.seed_hi, (uint32_t)(s0 + c), gen, ga.instance_id,
                       kTagMutPartner};
      uint8_t *row = child + c * LK + j * K;
      const uint8_t *h = hits + c * LK + j * K;
      uint32_t cur = 0xFFFFFFFFu;
      Words4 wb{0, 0, 0, 0};
      for (int k = 0; k < K; ++k) {
        if (!h[k]) continue;
        const uint32_t gi = (uint32_t)(j * K + k);
        if ((gi >> 2) != cur) {
          cur = gi >> 2;
          wb = par.block(cur);
        }
        const uint32_t r = bounded(pick(wb, gi & 3u), (uint32_t)(K - 1));
        const int kp = (int)r + ((int)r >= k ? 1 : 0);
        const uint8_t t = row[k];
        row[k] = row[kp];
        row[kp] = t;
      }
    }
  }
  __syncthreads();
}

// Elitism by a whole workgroup: wave 0 ranks, then every thread helps copy
// the E best chromosomes (rank order) into slots 0..E-1 of pout, fout[e]
// their fitness (when given), trace[gen] the best fitness (when given).
// idx: 64 ints of LDS.  Every thread must call it; ends with a barrier.
__device__ __forceinline__ void copy_elites_block(const uint8_t *__restrict__ pin,
                                                  const float *__restrict__ fin, int N, int E,
                                                  int LK, uint8_t *pout, float *fout,
                                                  float *trace, int gen, int32_t *idx) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (E >= 64) {  // rare: rank by counting, one wave
    if (wave == 0) copy_elites(pin, fin, N, E, LK, pout, fout, trace, gen, idx, lane);
    __syncthreads();
    return;
  }
  if (wave == 0) top_e_wave(fin, N, E > 1 ? E : 1, idx, lane);
  __syncthreads();
  if (threadIdx.x == 0 && trace) trace[gen] = fin[idx[0]];
  if (fout && (int)threadIdx.x < E) fout[threadIdx.x] = fin[idx[threadIdx.x]];
  const int ws = (LK >> 2) + 2;
  const int items = E * ws;
  const int step = (int)blockDim.x;
  for (int i0 = threadIdx.x; i0 < items; i0 += kCopyBatch * step) {
    uint32_t v[kCopyBatch];
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int i = i0 + u * step;
      const int e = i / ws, w = i % ws;
      const ByteRange r{pin + (size_t)idx[e < E ? e : 0] * LK, LK};
      v[u] = (i < items && w < r.words()) ? r.load(w) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int i = i0 + u * step;
      const int e = i / ws, w = i % ws;
      if (i < items) {
        const ByteRange r{pin + (size_t)idx[e] * LK, LK};
        if (w < r.words()) {
          uint8_t *dst = pout + (size_t)e * LK;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int g = r.pos(w, b);
            if (g >= 0 && g < LK) dst[g] = (uint8_t)(v[u] >> (8 * b));
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace pa
