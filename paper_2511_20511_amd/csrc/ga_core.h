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

// Indices of the E best (E <= 64) into idx[0..E) by repeated arg-max over keys
// strictly below the previous maximum (keys are unique: they embed the index).
// Populations up to 64*C keep their keys in registers (C per lane).
template <int C>
__device__ __forceinline__ void top_e_cached(const float *__restrict__ fin, int N, int E,
                                             int32_t *idx, int lane) {
  uint32_t kk[C];
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int i = lane + u * kWave;
    kk[u] = i < N ? rank_key(gp(fin)[i]) : 0u;
  }
  uint64_t prev = ~0ull;
  for (int e = 0; e < E; ++e) {
    uint64_t best = 0;
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int i = lane + u * kWave;
      const uint64_t k = ((uint64_t)kk[u] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
      if (i < N && k < prev && k > best) best = k;
    }
    best = wave_max_u64(best);
    if (lane == 0) idx[e] = (int32_t)key_index(best);
    prev = best;
  }
}

__device__ __forceinline__ void top_e_wave(const float *__restrict__ fin, int N, int E,
                                           int32_t *idx, int lane) {
  if (N <= 1 * kWave) return top_e_cached<1>(fin, N, E, idx, lane);
  if (N <= 2 * kWave) return top_e_cached<2>(fin, N, E, idx, lane);
  if (N <= 4 * kWave) return top_e_cached<4>(fin, N, E, idx, lane);
  if (N <= 8 * kWave) return top_e_cached<8>(fin, N, E, idx, lane);
  if (N <= 16 * kWave) return top_e_cached<16>(fin, N, E, idx, lane);
  if (N <= 32 * kWave) return top_e_cached<32>(fin, N, E, idx, lane);
  uint64_t prev = ~0ull;
  for (int e = 0; e < E; ++e) {
    uint64_t best = 0;
    for (int i0 = lane; i0 < N; i0 += 8 * kWave) {
      float f[8];  // eight loads in flight per lane
#pragma unroll
      for (int u = 0; u < 8; ++u) f[u] = gp(fin)[min(i0 + u * kWave, N - 1)];
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
  const uint32_t ki = rank_key(gp(fin)[i]);
  int r = 0;
  for (int m = 0; m < N; ++m) {
    const uint32_t km = rank_key(gp(fin)[m]);
    r += beats(km, (uint32_t)m, ki, (uint32_t)i) ? 1 : 0;
  }
  return r;
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
    if (trace && lane == 0) gp(trace)[gen] = gp(fin)[idx[0]];
    for (int e = 0; e < E; ++e) {
      const int src = idx[e];
      for (int i = lane; i < LK; i += kWave)
        gp(pout)[(size_t)e * LK + i] = gp(pin)[(size_t)src * LK + i];
      if (fout && lane == 0) gp(fout)[e] = gp(fin)[src];
    }
  } else {
    // E >= 64: every lane ranks its chromosomes by counting who beats them
    for (int i = lane; i < N; i += kWave) {
      const int r = rank_of(fin, N, i);
      if (r == 0 && trace) gp(trace)[gen] = gp(fin)[i];
      if (r < E) {
        for (int g = 0; g < LK; ++g) gp(pout)[(size_t)r * LK + g] = gp(pin)[(size_t)i * LK + g];
        if (fout) gp(fout)[r] = gp(fin)[i];
      }
    }
  }
}

// Stores the code word of genes 4b .. 4b+3 of a child whose codes start at
// `dst` (byte-aligned when LK is not a multiple of 4).
__device__ __forceinline__ void store_code_word(uint8_t *codes, int LK, int b, uint32_t v) {
  uint8_t *dst = codes + 4 * b;
  if ((LK & 3) == 0 && ((uintptr_t)codes & 3u) == 0) {
    *reinterpret_cast<uint32_t *>(dst) = v;
  } else {
    const int n = LK - 4 * b < 4 ? LK - 4 * b : 4;
    for (int u = 0; u < n; ++u) dst[u] = (uint8_t)(v >> (8 * u));
  }
}

// Mutation codes of group q (genes 32q .. 32q+31, row-major i = j*K + k) of
// the child in `slot`: byte code[b] = k' + 1 when gene 32q + b mutates and
// swaps with user k' of its cell, 0 otherwise (in out[b / 4], byte b % 4).
// The decision word of gene 32q + b has as its bit 31 - k the bit b of word
// 32q + k of the MUT_DECIDE stream, and the gene mutates when that word is
// below thr: the comparison runs from the most significant bit, one stream
// word (one bit of every gene of the group) at a time -- where thr's bit is 1
// a 0 bit decides "below", where it is 0 a 1 bit decides "not below" -- and
// stops drawing Philox blocks once every gene is decided.  The h-th mutating
// gene takes its partner from word 32q + h of the MUT_PARTNER stream.  boff is
// or-ed into the block counter (the island streams of the island GA).
// Returns the mask of the group's mutating genes (bit b: gene 32q + b).
__device__ __forceinline__ uint32_t group_codes(int q, int LK, int K, const DevGa &ga,
                                                uint32_t gen, uint32_t slot, uint32_t (&out)[8],
                                                uint32_t boff = 0u) {
#pragma unroll
  for (int w = 0; w < 8; ++w) out[w] = 0u;
  const int g0 = 32 * q;
  const int n = LK - g0 < 32 ? LK - g0 : 32;
  const uint32_t valid = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
  uint32_t hitm = 0u;
  if (ga.thr_mut >= (1ull << 32)) {
    hitm = valid;
  } else {
    const uint32_t th = (uint32_t)ga.thr_mut;
    const Stream dec{ga.seed_lo, ga.seed_hi, slot, gen, ga.instance_id, kTagMutDecide};
    uint32_t und = valid;
    for (int k4 = 0; k4 < 8 && und != 0u; ++k4) {
      const Words4 wb = dec.block(boff | (uint32_t)(8 * q + k4));
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t R = pick(wb, (uint32_t)u);
        if ((th >> (31 - (4 * k4 + u))) & 1u) {
          hitm |= und & ~R;
          und &= R;
        } else {
          und &= ~R;
        }
      }
    }
  }
  if (hitm == 0u) return 0u;
  const uint32_t hits = hitm;
  const Stream par{ga.seed_lo, ga.seed_hi, slot, gen, ga.instance_id, kTagMutPartner};
  Words4 pw{0u, 0u, 0u, 0u};
  int h = 0;
  while (hitm != 0u) {
    const int b = __builtin_ctz(hitm);
    hitm &= hitm - 1u;
    if ((h & 3) == 0) pw = par.block(boff | (uint32_t)(8 * q + (h >> 2)));
    const int k = (g0 + b) % K;
    const uint32_t r = bounded(pick(pw, (uint32_t)(h & 3)), (uint32_t)(K - 1));
    const uint32_t code = r + ((int)r >= k ? 1u : 0u) + 1u;
    // b is lane-varying: select the word without dynamic register indexing
#pragma unroll
    for (int w = 0; w < 8; ++w)
      if ((b >> 2) == w) out[w] |= code << (8 * (b & 3));
    ++h;
  }
  return hits;
}

// Byte b (0..31) of a group's codes, selected without dynamic register
// indexing.
__device__ __forceinline__ uint32_t code_byte(const uint32_t (&code)[8], int b) {
  const int w = b >> 2;
  uint32_t x = code[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) x = w == i ? code[i] : x;
  return (x >> (8 * (b & 3))) & 0xFFu;
}

// The latency form of group_codes: eight lanes (u = 0..7, consecutive lanes
// of one wave) per group, lane u drawing the decision block 8q + u (bits 4u ..
// 4u+3 of every gene's word, most significant first) at once.  Each lane
// compares its four bits ("below", "equal so far" masks), the lanes combine
// in order of significance (a more significant segment decides unless it is
// equal: below = below_a | (equal_a & below_b), equal = equal_a & equal_b) with
// three shuffle steps, and lane u writes the codes of genes 4u .. 4u+3 (their
// partner words by hit rank, as in group_codes).  Same codes as group_codes;
// more Philox blocks (all eight), far shorter dependence chains.  Every lane
// of the wave must call it (inactive ones with act = false).
__device__ __forceinline__ uint32_t group_codes_x8(bool act, int q, int u, int LK, int K,
                                                   const DevGa &ga, uint32_t gen, uint32_t slot) {
  const int g0 = 32 * q;
  const int n = LK - g0 < 32 ? (LK - g0 < 0 ? 0 : LK - g0) : 32;
  const uint32_t valid = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
  uint32_t lt = 0u, eq = valid;
  const bool all = ga.thr_mut >= (1ull << 32);
  if (act && !all) {
    const uint32_t th = (uint32_t)ga.thr_mut;
    const Stream dec{ga.seed_lo, ga.seed_hi, slot, gen, ga.instance_id, kTagMutDecide};
    const Words4 wb = dec.block((uint32_t)(8 * q + u));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t R = pick(wb, (uint32_t)v);
      if ((th >> (31 - (4 * u + v))) & 1u) {
        lt |= eq & ~R;
        eq &= R;
      } else {
        eq &= ~R;
      }
    }
  }
  const int lane = (int)(threadIdx.x & (kWave - 1));
#pragma unroll
  for (int st = 1; st < 8; st <<= 1) {
    const bool has = u + st < 8;
    const uint32_t lt2 = (uint32_t)__shfl((int)lt, has ? lane + st : lane);
    const uint32_t eq2 = (uint32_t)__shfl((int)eq, has ? lane + st : lane);
    if (has) {
      lt = lt | (eq & lt2);
      eq = eq & eq2;
    }
  }
  uint32_t hitm = (uint32_t)__shfl((int)lt, lane - u);  // the group's lane 0 holds all bits
  if (all) hitm = valid;
  if (!act) return 0u;
  uint32_t out = 0u;
  const uint32_t mine = hitm & (0xFu << (4 * u));
  if (mine != 0u) {
    const Stream par{ga.seed_lo, ga.seed_hi, slot, gen, ga.instance_id, kTagMutPartner};
    int hb = -1;
    Words4 pw{0u, 0u, 0u, 0u};
    for (uint32_t m = mine; m != 0u; m &= m - 1u) {
      const int b = __builtin_ctz(m);
      const int h = __builtin_popcount(hitm & ((1u << b) - 1u));
      if ((h >> 2) != hb) {
        hb = h >> 2;
        pw = par.block((uint32_t)(8 * q + hb));
      }
      const int k = (g0 + b) % K;
      const uint32_t r = bounded(pick(pw, (uint32_t)(h & 3)), (uint32_t)(K - 1));
      out |= (r + ((int)r >= k ? 1u : 0u) + 1u) << (8 * (b & 3));
    }
  }
  return out;
}

// Mutation codes of the children of slots [s0, s0 + nc) into `codes` (child c
// at byte c*LK) with the workgroup's threads from `base` (a multiple of the
// wave size) on: eight lanes per group of 32 genes (group_codes_x8: all eight
// decision blocks at once, short dependence chains) when the groups fit
// those threads in at most x8_passes passes, else one thread per (child,
// group) (the early-stopping group_codes: fewer Philox blocks, longer
// chains).  Threads below base return at once.  No barrier: the caller's next
// one publishes the codes.
__device__ __forceinline__ void mutation_codes_block(uint8_t *codes, int nc, int LK, int K,
                                                     const DevGa &ga, uint32_t gen, int s0,
                                                     int block, int base = 0,
                                                     int x8_passes = 1) {
  const int t0 = (int)threadIdx.x - base, avail = block - base;
  if (t0 < 0) return;
  const int ng = (LK + 31) >> 5;
  const int total = nc * ng;
  if (8 * total <= avail * x8_passes) {
    // every lane of a participating wave runs every pass (the eight lanes of
    // a group shuffle with each other)
    for (int p0 = 0; p0 < total; p0 += avail >> 3) {
      const int t = p0 + (t0 >> 3), u = t0 & 7;
      const bool act = t < total;
      const int c = act ? t / ng : 0, q = act ? t - c * ng : 0;
      const uint32_t v = group_codes_x8(act, q, u, LK, K, ga, gen, (uint32_t)(s0 + c));
      if (act && 32 * q + 4 * u < LK) store_code_word(codes + (size_t)c * LK, LK, 8 * q + u, v);
    }
    return;
  }
  for (int t = t0; t < total; t += avail) {
    const int c = t / ng, q = t - c * ng;
    uint32_t out[8];
    group_codes(q, LK, K, ga, gen, (uint32_t)(s0 + c), out);
    uint8_t *dst = codes + (size_t)c * LK;
#pragma unroll
    for (int w = 0; w < 8; ++w)
      if (32 * q + 4 * w < LK) store_code_word(dst, LK, 8 * q + w, out[w]);
  }
}

// Applies the swaps of one row (bytes row[0..K) in LDS) given its codes, in
// increasing k against the current row.  `codes` and `row` sit at the same
// offset `off` from 4-byte aligned bases, so the codes are read as aligned
// 32-bit words and only mutating genes touch the row.
__device__ __forceinline__ void apply_swaps(uint8_t *row, const uint8_t *codes, int off, int K) {
  const int mis = off & 3;
  const uint32_t *cw = reinterpret_cast<const uint32_t *>(codes - mis);
  const int nw = (mis + K + 3) >> 2;
  uint64_t m = 0;
#pragma unroll 4
  for (int w = 0; w < nw; ++w) {
    const uint32_t v = cw[w];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * w + b - mis;
      if (k >= 0 && k < K && ((v >> (8 * b)) & 0xFFu) != 0u) m |= 1ull << k;
    }
  }
  while (m != 0ull) {
    const int k = __builtin_ctzll(m);
    m &= m - 1ull;
    const int kp = (int)codes[k] - 1;
    const uint8_t t = row[k];
    row[k] = row[kp];
    row[kp] = t;
  }
}

// Copies the byte range r into LDS at dst + off (dst 4-byte aligned) with a
// team of tpr threads (this thread is member `sub`): aligned 32-bit loads, up
// to kCopyBatch in flight; whole words are stored as words when source and
// destination share their alignment, bytes otherwise.
__device__ __forceinline__ void gather_range(const ByteRange &r, uint8_t *dst, int off, int sub,
                                             int tpr) {
  if (r.n <= 0) return;
  const int nw = r.words();
  const int smis = (int)((uintptr_t)r.src & 3u);
  const bool same = ((off - smis) & 3) == 0;
  for (int w0 = sub; w0 < nw; w0 += kCopyBatch * tpr) {
    uint32_t v[kCopyBatch];
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) v[u] = r.load(min(w0 + u * tpr, nw - 1));
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int w = w0 + u * tpr;
      if (w < nw) {
        const int g0 = 4 * w - smis;  // range offset of the word's first byte
        if (same && g0 >= 0 && g0 + 4 <= r.n) {
          *reinterpret_cast<uint32_t *>(dst + off + g0) = v[u];
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int g = g0 + b;
            if (g >= 0 && g < r.n) dst[off + g] = (uint8_t)(v[u] >> (8 * b));
          }
        }
      }
    }
  }
}

enum : int { kBuildSelect = 0, kBuildGather = 1, kBuildAll = 2 };

// Builds the children of slots [s0, s0 + nc) in LDS (child c at child +
// c*L*K) with the whole workgroup (nc <= block), in phases separated by
// barriers:
//   1. thread c < nc: its pair's six SELECT words and the four fitness loads
//      of its tournaments; meanwhile the workgroup draws the mutation codes
//      into `codes`; then thread c resolves the tournaments, crossover
//      decision and cut;
//   2. all threads over all genes: copy from the parents (aligned words,
//      several loads in flight);
//   3. one thread per (child, row): the swaps, in increasing k.
// `upto` stops after phase 1 (kBuildSelect: parents and cut in sSel) or
// phase 2 (kBuildGather: children without their swaps).
// `child` and `codes` are 4-byte aligned LDS buffers of nc*L*K bytes; sSel:
// 2 ints per child.  Ends with a barrier.
__device__ __forceinline__ void build_children_block(const uint8_t *__restrict__ pin,
                                                     const float *__restrict__ fin, int N, int E,
                                                     int L, int K, const DevGa &ga, uint32_t gen,
                                                     int s0, int nc, uint8_t *child,
                                                     uint8_t *codes, int32_t *sSel, int block,
                                                     int upto = kBuildAll) {
  const int LK = L * K;
  const int tid = threadIdx.x;
  const bool sel = tid < nc;
  const int slot = s0 + tid;
  uint32_t u0 = 0, v0 = 0, u1 = 0, v1 = 0;
  float fu0 = 0.0f, fv0 = 0.0f, fu1 = 0.0f, fv1 = 0.0f;
  Words4 b1{0, 0, 0, 0};
  if (sel) {
    const int pair_a = E + ((slot - E) & ~1);
    const Stream st{ga.seed_lo, ga.seed_hi, (uint32_t)pair_a, gen, ga.instance_id, kTagSelect};
    const Words4 b0 = st.block(0u);
    b1 = st.block(1u);
    u0 = bounded(b0.x, (uint32_t)N);
    v0 = bounded(b0.y, (uint32_t)N);
    u1 = bounded(b0.z, (uint32_t)N);
    v1 = bounded(b0.w, (uint32_t)N);
    fu0 = gp(fin)[u0];
    fv0 = gp(fin)[v0];
    fu1 = gp(fin)[u1];
    fv1 = gp(fin)[v1];
  }
  const bool mutate = K >= 2 && ga.thr_mut != 0;
  if (mutate) mutation_codes_block(codes, nc, LK, K, ga, gen, s0, block);
  if (sel) {
    const bool second = ((slot - E) & 1) != 0;
    const uint32_t p1 = beats(rank_key(fv0), v0, rank_key(fu0), u0) ? v0 : u0;
    const uint32_t p2 = beats(rank_key(fv1), v1, rank_key(fu1), u1) ? v1 : u1;
    const bool cross = L >= 2 && hit(b1.x, ga.thr_cross);
    const int cut = cross ? 1 + (int)bounded(b1.y, (uint32_t)(L - 1)) : L;
    const uint32_t first = second ? p2 : p1, rest = second ? p1 : p2;
    sSel[2 * tid] = (int32_t)(first | (rest << 16));
    sSel[2 * tid + 1] = cut * K;
  }
  __syncthreads();
  if (upto == kBuildSelect) return;
  // child c = first parent's genes [0, cut) + second's [cut, LK): two byte
  // ranges per child; a power-of-two team of threads per range moves it as
  // aligned words, several loads in flight per thread
  {
    const int nr = 2 * nc;
    int lg = 0;
    while ((2 << lg) * nr <= block) ++lg;
    const int tpr = 1 << lg;  // threads per range
    const int sub = tid & (tpr - 1);
    for (int r0 = tid >> lg; r0 < nr; r0 += block >> lg) {
      const int c = r0 >> 1;
      const uint32_t pr = (uint32_t)sSel[2 * c];
      const int cutg = sSel[2 * c + 1];
      if ((r0 & 1) == 0)
        gather_range(ByteRange{pin + (size_t)(pr & 0xFFFFu) * LK, cutg}, child, c * LK, sub, tpr);
      else
        gather_range(ByteRange{pin + (size_t)(pr >> 16) * LK + cutg, LK - cutg}, child,
                     c * LK + cutg, sub, tpr);
    }
  }
  __syncthreads();
  if (mutate && upto == kBuildAll) {
    for (int r = tid; r < nc * L; r += block) {
      const int off = r * K;  // (c*L + j)*K
      apply_swaps(child + off, codes + off, off, K);
    }
    __syncthreads();
  }
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
  if (threadIdx.x == 0 && trace) gp(trace)[gen] = gp(fin)[idx[0]];
  if (fout && (int)threadIdx.x < E) gp(fout)[threadIdx.x] = gp(fin)[idx[threadIdx.x]];
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
            if (g >= 0 && g < LK) gp(dst)[g] = (uint8_t)(v[u] >> (8 * b));
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace pa
