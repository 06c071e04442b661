// k_island.hip -- the parallel K-means GA (PK-means GA, Alg. 2, Sec. 4.3):
// the population is partitioned by K-means into C clusters (islands) that
// evolve on their own, and K-means is applied again every few generations
// (three in Sec. 6.1).  The reading (the paper fixes neither the feature
// space nor the per-island operators):
//   - a chromosome is the point (g_0, .., g_{LK-1}) of Z^{LK}, squared
//     Euclidean distance in integers (exact: at most 63^2 x 4096 < 2^31);
//   - farthest-point start from the best-ranked chromosome (ties to the lowest
//     index), then Lloyd iterations: assign to the nearest centroid (ties to
//     the lowest cluster), centroid = per-gene rounded mean
//     floor((2 s + n) / (2 n)) (an empty cluster keeps its centroid), until no
//     label changes or max_iters;
//   - island c holds the positions labelled c until the next clustering; its
//     next generation: E_c = 0 if E = 0, else min(n_c, max(1, floor(E n_c / N
//     + 1/2))) elites (its best, in rank order) in its first E_c positions,
//     children in pairs over its following positions, tournament candidates
//     among its members, crossover and mutation as in the panmictic step;
//   - the random streams are those of the panmictic step with the island
//     index in bits 16..23 of the block counter, so C = 1 is the panmictic GA.
// Kernels: k_pop_kmeans / k_pop_kmeans_lds (one workgroup per population; the
// second with the population resident in LDS), k_island_plan (one
// workgroup per island, the processing unit of an island in Sec. 5) and
// k_island_build (the positions of all islands in chunks).
#include <algorithm>
#include <cstring>
#include <vector>

#include "fitness_core.h"
#include "ga_core.h"
#include "pa_host.h"

namespace pa {
namespace {

constexpr int kIslandMaxN = 4096;
constexpr int kIslandMaxC = 16;
constexpr int kKmThreads = 1024;

// ---------------------------------------------------------------- K-means
//
// LDS: centroids [C][LK] bytes | labels [N] | nearest distances [N] | small
// scratch.  The population stays in global memory (each chromosome read once
// per assignment pass by its thread, each gene column once per update pass).
struct PopKmArgs {
  const uint8_t *pop;
  const float *fit;
  int N, LK, C, max_iters;
  int32_t *labels;  // out [N]
  int32_t *iters;   // out [1] (may be null)
};

// squared distance of chromosome row (global, 4-byte aligned when LK % 4 == 0)
// to centroid cent (LDS)
__device__ __forceinline__ int32_t km_dist(const uint8_t *row, const uint8_t *cent, int LK) {
  int32_t d = 0;
  if ((LK & 3) == 0) {
    const gptr<const uint32_t> r = gp(reinterpret_cast<const uint32_t *>(row));
    const uint32_t *c = reinterpret_cast<const uint32_t *>(cent);
    for (int w = 0; w < (LK >> 2); ++w) {
      const uint32_t a = r[w], b = c[w];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t t = (int32_t)((a >> (8 * k)) & 0xFFu) - (int32_t)((b >> (8 * k)) & 0xFFu);
        d += t * t;
      }
    }
  } else {
    for (int i = 0; i < LK; ++i) {
      const int32_t t = (int32_t)gp(row)[i] - (int32_t)cent[i];
      d += t * t;
    }
  }
  return d;
}

// Block-wide arg-max of a 64-bit key over threads (lowest index wins through
// the key's low half); returns it in every thread.
__device__ __forceinline__ uint64_t block_max_u64(uint64_t k, uint64_t *sRed) {
  k = wave_max_u64(k);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) sRed[wave] = k;
  __syncthreads();
  uint64_t m = 0;
  const int nw = (int)blockDim.x / kWave;
  for (int w = 0; w < nw; ++w) m = sRed[w] > m ? sRed[w] : m;
  return m;
}

__global__ __launch_bounds__(kKmThreads) void k_pop_kmeans(PopKmArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int N = a.N, LK = a.LK, C = a.C;
  const int cent_bytes = (C * LK + 15) / 16 * 16;
  uint8_t *sCent = smem;
  int32_t *sLab = reinterpret_cast<int32_t *>(smem + cent_bytes);
  int32_t *sDmin = sLab + N;
  uint64_t *sRed = reinterpret_cast<uint64_t *>(sDmin + N);  // 8 N bytes after sLab: aligned
  int32_t *sFlag = reinterpret_cast<int32_t *>(sRed + kKmThreads / kWave);
  int32_t *sCnt = sFlag + 2;
  const int tid = threadIdx.x, T = blockDim.x;
  // centroid 0: the best-ranked chromosome (fitness descending, lower index
  // first, NaN last: the rank key)
  uint64_t bk = 0;
  for (int n = tid; n < N; n += T) {
    const uint64_t k = full_key(gp(a.fit)[n], (uint32_t)n);
    bk = k > bk ? k : bk;
  }
  int pick = (int)key_index(block_max_u64(bk, sRed));
  for (int m = 0; m < C; ++m) {
    for (int i = tid; i < LK; i += T) sCent[m * LK + i] = gp(a.pop)[(size_t)pick * LK + i];
    __syncthreads();
    if (m + 1 == C) break;
    // nearest-centroid distance of every chromosome, updated with centroid m;
    // the next centroid is the farthest (ties to the lowest index)
    uint64_t fk = 0;
    for (int n = tid; n < N; n += T) {
      const int32_t d = km_dist(a.pop + (size_t)n * LK, sCent + m * LK, LK);
      const int32_t dm = m == 0 ? d : min(sDmin[n], d);
      sDmin[n] = dm;
      const uint64_t k = ((uint64_t)(uint32_t)dm << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)n);
      fk = k > fk ? k : fk;
    }
    pick = (int)key_index(block_max_u64(fk, sRed));
  }
  for (int n = tid; n < N; n += T) sLab[n] = -1;
  int it = 0;
  for (; it < a.max_iters; ++it) {
    if (tid == 0) sFlag[0] = 0;
    __syncthreads();
    // assignment: nearest centroid, ties to the lowest cluster
    for (int n = tid; n < N; n += T) {
      int best = 0;
      int32_t bd = 0x7FFFFFFF;
      for (int c = 0; c < C; ++c) {
        const int32_t d = km_dist(a.pop + (size_t)n * LK, sCent + c * LK, LK);
        if (d < bd) {
          bd = d;
          best = c;
        }
      }
      if (sLab[n] != best) {
        sLab[n] = best;
        sFlag[0] = 1;
      }
    }
    __syncthreads();
    if (sFlag[0] == 0) break;
    // update: per gene, the member sums of every cluster (then counts)
    if (tid < C) sCnt[tid] = 0;
    __syncthreads();
    for (int n = tid; n < N; n += T) atomicAdd(&sCnt[sLab[n]], 1);
    __syncthreads();
    for (int i = tid; i < LK; i += T) {
      int32_t s[kIslandMaxC];
#pragma unroll
      for (int c = 0; c < kIslandMaxC; ++c) s[c] = 0;
      for (int n = 0; n < N; ++n) {
        const int32_t g = gp(a.pop)[(size_t)n * LK + i];
        const int lab = sLab[n];
#pragma unroll
        for (int c = 0; c < kIslandMaxC; ++c) s[c] += lab == c ? g : 0;
      }
#pragma unroll
      for (int c = 0; c < kIslandMaxC; ++c) {
        if (c < C && sCnt[c] > 0)
          sCent[c * LK + i] = (uint8_t)((2 * s[c] + sCnt[c]) / (2 * sCnt[c]));
      }
    }
    __syncthreads();
  }
  for (int n = tid; n < N; n += T) gp(a.labels)[n] = sLab[n];
  if (tid == 0 && a.iters) *gp(a.iters) = it;
}

// The same clustering with the population resident in LDS (rows padded with
// zero genes to LKP bytes, a multiple of 16), for populations that fit.  Gene
// values are below 64, so the squared distance is |a|^2 + |b|^2 - 2 a.b,
// exact in 32 bits; a chromosome's nearest centroid minimises |c|^2 - 2 a.c.
// The products a.c of the assignment and of the farthest-point passes are
// int8 matrix products (km_tile_dots: 16 chromosomes x 16 centroids per
// tile); |a|^2 uses v_dot4_u32_u8.  Update: the members of each cluster
// listed by a counting sort, then threads per (cluster, 4-gene word) sum
// their members' genes in two packed 16-bit accumulators (flushed every 256
// members).
constexpr int kKmPad = 16;

__device__ __forceinline__ int km_lkp(int LK) { return (LK + kKmPad - 1) / kKmPad * kKmPad; }

struct KmLds {
  uint8_t *pop, *cent;
  int32_t *a2, *lab, *dmin, *mem, *b2, *cnt, *off, *pos, *flag, *pk;
  uint64_t *red, *far;
  uint32_t *part;  // [kKmThreads][4] partial member sums of the update
};

__device__ __forceinline__ KmLds km_lds_layout(unsigned char *smem, int N, int LKP, int C) {
  KmLds m;
  m.pop = smem;
  m.cent = smem + (size_t)N * LKP;
  int32_t *w = reinterpret_cast<int32_t *>(m.cent + (size_t)C * LKP);
  m.a2 = w;
  m.lab = w + N;
  m.dmin = w + 2 * N;
  m.mem = w + 3 * N;
  m.b2 = w + 4 * N;
  m.cnt = m.b2 + kIslandMaxC;      // two sets, by pass parity
  m.off = m.cnt + 2 * kIslandMaxC;
  m.pos = m.off + kIslandMaxC;
  m.flag = m.pos + kIslandMaxC;    // two, by pass parity (+ 2 unused)
  m.pk = m.flag + 4;               // the farthest-point picks
  m.red = reinterpret_cast<uint64_t *>(m.pk + kIslandMaxC);  // 8-byte aligned: N, LKP multiples of 4
  m.far = m.red + kKmThreads / kWave;                         // three rotating maxima
  m.part = reinterpret_cast<uint32_t *>(m.far + 4);           // 16-byte aligned
  return m;
}

int kmeans_lds_resident(int N, int LK, int C) {
  const int LKP = (LK + kKmPad - 1) / kKmPad * kKmPad;
  return N * LKP + C * LKP + 16 * N + 4 * (6 * kIslandMaxC + 4) +
         8 * (kKmThreads / kWave + 4) + 16 * kKmThreads;
}

// Lanes per chromosome in the distance passes: the largest power of two (at
// most 16) with N x S within the workgroup, so small populations still fill
// it; a chromosome's S lanes are consecutive and each takes every S-th
// 16-byte chunk of the row.
__device__ __forceinline__ int km_split(int N, int T) {
  int S = 1;
  while (S < 16 && N * (2 * S) <= T) S <<= 1;
  return S;
}

// a.b over chunks q, q + S, .. of a row and a centroid (LDS)
__device__ __forceinline__ uint32_t km_dot_part(const uint8_t *x, const uint8_t *y, int LKP, int q,
                                                int S) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  uint32_t d = 0u;
  for (int o = 16 * q; o < LKP; o += 16 * S) {
    const u4 a = *reinterpret_cast<const u4 *>(x + o), b = *reinterpret_cast<const u4 *>(y + o);
    d = __builtin_amdgcn_udot4(a.x, b.x, d, false);
    d = __builtin_amdgcn_udot4(a.y, b.y, d, false);
    d = __builtin_amdgcn_udot4(a.z, b.z, d, false);
    d = __builtin_amdgcn_udot4(a.w, b.w, d, false);
  }
  return d;
}

// sum over the S consecutive lanes of a group (every lane of the wave calls it)
__device__ __forceinline__ uint32_t km_group_sum(uint32_t v, int S) {
  for (int m = 1; m < S; m <<= 1) v += (uint32_t)__shfl_xor((int)v, m);
  return v;
}

typedef int km_v4i __attribute__((ext_vector_type(4)));

// The products a.c of the 16 chromosomes of tile t (rows 16 t .. 16 t + 15 of
// the population in LDS) with 16 centroid rows (column j: row cent + j *
// cstride, zero for j >= ncent), as an int8 matrix product in steps of 64
// genes (gene values are below 64, so the int8 operands are exact and the
// int32 sums too).  Lane l gives row l % 16 and column l % 16 the same 16
// genes of each step (bytes 16 (l / 16) of it; zeros past the padded row
// end), so the order of the product's k slots does not matter.  Lane l
// receives rows 4 (l / 16) + r, column l % 16 in element r.  Every lane of the
// wave calls it.
__device__ __forceinline__ km_v4i km_tile_dots(const uint8_t *pop, int N, int LKP, int t,
                                               const uint8_t *cent, int ncent, int cstride) {
  const int lane = (int)(threadIdx.x & 63), i = lane & 15, g = lane >> 4;
  const int n = 16 * t + i;
  const uint8_t *ra = pop + (size_t)n * LKP;
  const uint8_t *rb = cent + (size_t)i * cstride;
  km_v4i d = {0, 0, 0, 0};
  for (int o = 16 * g; o - 16 * g < LKP; o += 64) {
    const bool in = o < LKP;
    const km_v4i zero = {0, 0, 0, 0};
    const km_v4i x = (in && n < N) ? *reinterpret_cast<const km_v4i *>(ra + o) : zero;
    const km_v4i y = (in && i < ncent) ? *reinterpret_cast<const km_v4i *>(rb + o) : zero;
    d = __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, d, 0, 0, 0);
  }
  return d;
}

__global__ __launch_bounds__(kKmThreads) void k_pop_kmeans_lds(PopKmArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  const int N = a.N, LK = a.LK, C = a.C, LKP = km_lkp(LK), W = LKP / 4;
  const KmLds m = km_lds_layout(smem, N, LKP, C);
  const int tid = threadIdx.x, T = blockDim.x;
  const int wave = tid / kWave, lane = tid % kWave, nw = T / kWave;
  // the population into LDS, zero genes past LK: rows of whole 16-byte
  // chunks as one flat copy (four chunks in flight per thread), others one
  // wave per row
  if (LK == LKP && (reinterpret_cast<uintptr_t>(a.pop) & 15) == 0) {
    const gptr<const u4> src = gp(reinterpret_cast<const u4 *>(a.pop));
    u4 *dst = reinterpret_cast<u4 *>(m.pop);
    const int total = N * (LKP / 16);
#pragma unroll 4
    for (int i = tid; i < total; i += T) dst[i] = src[i];
  } else {
    for (int n = wave; n < N; n += nw) {
      uint32_t *dst = reinterpret_cast<uint32_t *>(m.pop + (size_t)n * LKP);
      if ((LK & 3) == 0) {
        const gptr<const uint32_t> src =
            gp(reinterpret_cast<const uint32_t *>(a.pop + (size_t)n * LK));
        for (int w = lane; w < W; w += kWave) dst[w] = w < (LK >> 2) ? src[w] : 0u;
      } else {
        for (int i = lane; i < LKP; i += kWave)
          m.pop[(size_t)n * LKP + i] = i < LK ? gp(a.pop)[(size_t)n * LK + i] : (uint8_t)0;
      }
    }
  }
  __syncthreads();
  const int S = km_split(N, T);
  // |row|^2 of every chromosome; centroid 0 the best-ranked chromosome
  uint64_t bk = 0;
  for (int n = tid; n < N; n += T) {
    const uint64_t k = full_key(gp(a.fit)[n], (uint32_t)n);
    bk = k > bk ? k : bk;
  }
  for (int b0 = 0; b0 < N * S; b0 += T) {
    const int n = (b0 + tid) / S, q = (b0 + tid) % S;
    const uint8_t *row = m.pop + (size_t)min(n, N - 1) * LKP;
    const uint32_t d = km_group_sum(n < N ? km_dot_part(row, row, LKP, q, S) : 0u, S);
    if (n < N && q == 0) m.a2[n] = (int32_t)d;
  }
  if (tid < 3) m.far[tid] = 0;  // (published by the barriers of the next reduction)
  int pick = (int)key_index(block_max_u64(bk, m.red));  // (its barriers publish a2)
  // farthest-point start: centroid c is population row pk[c] (compared in
  // place); each pass updates every chromosome's nearest distance and takes
  // the farthest through an LDS maximum (three slots in rotation, each reset
  // a pass before its next use)
  for (int c = 0; c + 1 < C; ++c) {
    if (tid == 0) {
      m.pk[c] = pick;
      m.far[(c + 1) % 3] = 0;
    }
    const uint8_t *cr = m.pop + (size_t)pick * LKP;
    const int32_t bc = m.a2[pick];
    uint64_t fk = 0;
    for (int t = wave; 16 * t < N; t += nw) {
      // the picked row in every column; lanes of column 0 take the results
      const km_v4i dot = km_tile_dots(m.pop, N, LKP, t, cr, 16, 0);
      if ((lane & 15) == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = 16 * t + 4 * (lane >> 4) + r;
          if (n < N) {
            const int32_t d = m.a2[n] + bc - 2 * dot[r];
            const int32_t dm = c == 0 ? d : min(m.dmin[n], d);
            m.dmin[n] = dm;
            const uint64_t k =
                ((uint64_t)(uint32_t)dm << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)n);
            fk = k > fk ? k : fk;
          }
        }
      }
    }
    fk = wave_max_u64(fk);
    if (lane == 0) atomicMax(reinterpret_cast<unsigned long long *>(&m.far[c % 3]),
                             (unsigned long long)fk);
    __syncthreads();
    pick = (int)key_index(m.far[c % 3]);
  }
  if (tid == 0) {
    m.pk[C - 1] = pick;
    m.flag[0] = 0;
  }
  if (tid < kIslandMaxC) m.cnt[tid] = 0;
  __syncthreads();
  // the centroids: copies of the picked rows
  for (int i = tid; i < C * (LKP / 16); i += T) {
    const int c = i / (LKP / 16), o = i - c * (LKP / 16);
    reinterpret_cast<u4 *>(m.cent + (size_t)c * LKP)[o] =
        reinterpret_cast<const u4 *>(m.pop + (size_t)m.pk[c] * LKP)[o];
  }
  if (tid < C) m.b2[tid] = m.a2[m.pk[tid]];
  for (int n = tid; n < N; n += T) m.lab[n] = -1;
  __syncthreads();
  const int CW = C * W;
  const int S2 = max(1, T / CW);  // threads per (cluster, word) in the update
  int it = 0;
  for (; it < a.max_iters; ++it) {
    // counts and the change flag alternate by pass parity: this pass clears
    // the other set, last read before the previous pass's final barrier
    const int par = it & 1;
    int32_t *cnt = m.cnt + par * kIslandMaxC;
    if (tid == 0) m.flag[par ^ 1] = 0;
    if (tid < kIslandMaxC) m.cnt[(par ^ 1) * kIslandMaxC + tid] = 0;
    // assignment: the centroid minimising |c|^2 - 2 a.c, ties to the lowest,
    // by tiles of 16 chromosomes x 16 centroids; each cluster's members counted
    for (int t = wave; 16 * t < N; t += nw) {
      const km_v4i dot = km_tile_dots(m.pop, N, LKP, t, m.cent, C, LKP);
      const int j = lane & 15;
      const int32_t bj = j < C ? m.b2[j] : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // key (|c|^2 - 2 a.c + 2^25) << 5 | c: |c|^2 and a.c stay below 4096 x 63^2
        // < 2^24, so the offset distance fits 26 bits and the minimum key is the
        // nearest centroid, the lowest on ties
        uint32_t key = j < C ? ((uint32_t)(bj - 2 * dot[r] + (1 << 25)) << 5) | (uint32_t)j
                             : 0xFFFFFFFFu;
#pragma unroll
        for (int x = 1; x < 16; x <<= 1) {
          const uint32_t o = (uint32_t)__shfl_xor((int)key, x);
          key = o < key ? o : key;
        }
        const int n = 16 * t + 4 * (lane >> 4) + r;
        if (j == 0 && n < N) {
          const int best = (int)(key & 31u);
          if (m.lab[n] != best) {
            m.lab[n] = best;
            m.flag[par] = 1;
          }
          atomicAdd(&cnt[best], 1);
        }
      }
    }
    __syncthreads();
    if (m.flag[par] == 0) break;
    // members of each cluster, listed by a counting sort (the order inside
    // a cluster is free: the sums are exact)
    if (tid == 0) {
      int o = 0;
      for (int c = 0; c < C; ++c) {
        m.off[c] = o;
        m.pos[c] = o;
        o += cnt[c];
      }
    }
    if (tid < C && cnt[tid] > 0) m.b2[tid] = 0;  // recomputed below with the new centroid
    __syncthreads();
    for (int n = tid; n < N; n += T) m.mem[atomicAdd(&m.pos[m.lab[n]], 1)] = n;
    __syncthreads();
    // new centroids: the members' gene sums per (cluster, word of 4 genes),
    // over S2 slices of the member list when threads are left over
    for (int t = tid; t < CW * S2; t += T) {
      const int h = t / CW, cw = t - h * CW;
      const int c = cw / W, w = cw - c * W;
      const int n_c = cnt[c];
      if (n_c == 0) continue;
      uint32_t sum[4] = {0u, 0u, 0u, 0u};
      const int32_t *mem = m.mem + m.off[c];
      const uint32_t *pw = reinterpret_cast<const uint32_t *>(m.pop) + w;
      const int ka = (int)((int64_t)h * n_c / S2), kb = (int)((int64_t)(h + 1) * n_c / S2);
      for (int k0 = ka; k0 < kb; k0 += 256) {
        uint32_t ev = 0u, od = 0u;  // genes 0, 2 and 1, 3 of the word in 16-bit halves
        const int k1 = min(kb, k0 + 256);
        int k = k0;
        for (; k + 8 <= k1; k += 8) {  // eight members' loads in flight
          uint32_t x[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) x[j] = pw[(size_t)mem[k + j] * W];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            ev += x[j] & 0x00FF00FFu;
            od += (x[j] >> 8) & 0x00FF00FFu;
          }
        }
        for (; k < k1; ++k) {
          const uint32_t x = pw[(size_t)mem[k] * W];
          ev += x & 0x00FF00FFu;
          od += (x >> 8) & 0x00FF00FFu;
        }
        sum[0] += ev & 0xFFFFu;
        sum[1] += od & 0xFFFFu;
        sum[2] += ev >> 16;
        sum[3] += od >> 16;
      }
      if (S2 > 1) {
#pragma unroll
        for (int b = 0; b < 4; ++b) m.part[4 * t + b] = sum[b];
        continue;
      }
      uint32_t word = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        word |= ((2u * sum[b] + (uint32_t)n_c) / (2u * (uint32_t)n_c)) << (8 * b);
      reinterpret_cast<uint32_t *>(m.cent + (size_t)c * LKP)[w] = word;
      atomicAdd(&m.b2[c], (int32_t)__builtin_amdgcn_udot4(word, word, 0u, false));
    }
    if (S2 > 1) {
      __syncthreads();
      for (int cw = tid; cw < CW; cw += T) {
        const int c = cw / W, w = cw - c * W;
        const int n_c = cnt[c];
        if (n_c == 0) continue;
        uint32_t word = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          uint32_t sb = 0u;
          for (int h = 0; h < S2; ++h) sb += m.part[4 * (h * CW + cw) + b];
          word |= ((2u * sb + (uint32_t)n_c) / (2u * (uint32_t)n_c)) << (8 * b);
        }
        reinterpret_cast<uint32_t *>(m.cent + (size_t)c * LKP)[w] = word;
        atomicAdd(&m.b2[c], (int32_t)__builtin_amdgcn_udot4(word, word, 0u, false));
      }
    }
    __syncthreads();
  }
  for (int n = tid; n < N; n += T) gp(a.labels)[n] = m.lab[n];
  if (tid == 0 && a.iters) *gp(a.iters) = it;
}

// ---------------------------------------------------------------- island step
//
// Two kernels: k_island_plan (one workgroup per island) finds the island's
// members, its elites and each child's tournaments and cut, and writes one
// record per position; k_island_build (positions in chunks, many workgroups)
// builds every position from its record: rows from the parents (word
// gathers), mutation codes drawn per (child, group of 32 genes) with the
// island's block offset, swaps per row.
struct IslandArgs {
  const uint8_t *pin;
  const float *fin;
  uint8_t *pout;
  const int32_t *labels;
  int N, E, L, K, C;
  uint32_t gen;
  DevGa ga;
  float *trace_g;  // null, or the trace entry that receives the best of fin
};

// What position s of the next generation is built from: rows [0, cutg / K)
// from `first`, the others from `rest` (packed first | rest << 16); `island`
// its island; elite != 0: a copy of `first`, no mutation.
struct IslandRec {
  int32_t parents, cutg, island, elite;
};

constexpr int kIslandThreads = 256;

__global__ __launch_bounds__(kIslandThreads) void k_island_plan(IslandArgs a, IslandRec *rec) {
  __shared__ int32_t sM[kIslandMaxN];
  __shared__ uint64_t sRed[kIslandThreads / kWave];
  __shared__ int32_t sCount[kIslandThreads / kWave + 1];
  const int c = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const int N = a.N, L = a.L, K = a.K, LK = L * K;
  if (c == a.C) {
    // the extra workgroup: a position whose label names no island is a copy
    // of itself (no island writes its record), and the best of the input
    // population goes to the trace
    uint64_t bk = 0;
    for (int n = tid; n < N; n += T) {
      const int lab = gp(a.labels)[n];
      if (lab < 0 || lab >= a.C) rec[n] = IslandRec{n | (n << 16), LK, 0, 1};
      const uint64_t k = full_key(gp(a.fin)[n], (uint32_t)n);
      bk = k > bk ? k : bk;
    }
    if (a.trace_g) {
      bk = block_max_u64(bk, sRed);
      if (tid == 0) *gp(a.trace_g) = gp(a.fin)[key_index(bk)];
    }
    return;
  }
  // members of island c, in increasing position: a block prefix over the labels
  int base = 0;
  for (int n0 = 0; n0 < N; n0 += T) {
    const int n = n0 + tid;
    const bool mine = n < N && gp(a.labels)[n] == c;
    const uint64_t ballot = __ballot(mine);
    const int wave = tid / kWave, lane = tid % kWave;
    const int before = __popcll(ballot & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) sCount[wave] = __popcll(ballot);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wave; ++w) off += sCount[w];
    if (mine) sM[off + before] = n;
    int total = 0;
    for (int w = 0; w < T / kWave; ++w) total += sCount[w];
    __syncthreads();
    base += total;
  }
  const int n = base;
  if (n == 0) return;
  int Ec = 0;
  if (a.E > 0) {
    Ec = (int)((2 * (int64_t)a.E * n + N) / (2 * (int64_t)N));
    Ec = Ec < 1 ? 1 : (Ec > n ? n : Ec);
  }
  // elites: the island's Ec best in rank order (repeated arg-max over keys
  // below the previous maximum; keys embed the position, so they are unique)
  uint64_t prev = ~0ull;
  for (int e = 0; e < Ec; ++e) {
    uint64_t best = 0;
    for (int t = tid; t < n; t += T) {
      const int m = sM[t];
      const uint64_t k = full_key(gp(a.fin)[m], (uint32_t)m);
      if (k < prev && k > best) best = k;
    }
    best = block_max_u64(best, sRed);
    prev = best;
    if (tid == 0) {
      const int src = (int)key_index(best);
      rec[sM[e]] = IslandRec{src | (src << 16), LK, c, 1};
    }
  }
  // children, one thread each: pair (first, first + 1) of island positions
  // t >= Ec; selection words keyed by the pair's first slot
  const uint32_t boff = (uint32_t)c << 16;
  for (int t = Ec + tid; t < n; t += T) {
    const int first = Ec + ((t - Ec) & ~1);
    const bool second = ((t - Ec) & 1) != 0;
    const uint32_t slot_a = (uint32_t)sM[first];
    const Stream st{a.ga.seed_lo, a.ga.seed_hi, slot_a, a.gen, a.ga.instance_id, kTagSelect};
    const Words4 b0 = st.block(boff | 0u), b1 = st.block(boff | 1u);
    const int u0 = sM[bounded(b0.x, (uint32_t)n)], v0 = sM[bounded(b0.y, (uint32_t)n)];
    const int u1 = sM[bounded(b0.z, (uint32_t)n)], v1 = sM[bounded(b0.w, (uint32_t)n)];
    const int p1 = beats(rank_key(gp(a.fin)[v0]), (uint32_t)v0, rank_key(gp(a.fin)[u0]),
                         (uint32_t)u0)
                       ? v0
                       : u0;
    const int p2 = beats(rank_key(gp(a.fin)[v1]), (uint32_t)v1, rank_key(gp(a.fin)[u1]),
                         (uint32_t)u1)
                       ? v1
                       : u1;
    const bool cross = L >= 2 && hit(b1.x, a.ga.thr_cross);
    const int cut = cross ? 1 + (int)bounded(b1.y, (uint32_t)(L - 1)) : L;
    const int pf = second ? p2 : p1, pr = second ? p1 : p2;
    rec[sM[t]] = IslandRec{pf | (pr << 16), cut * K, c, 0};
  }
}

// Positions per build workgroup for N chromosomes of LK genes: enough
// workgroups for the population to spread over 128 of them, at most 64
// positions and two 16 KB buffers of them in LDS.
int island_chunk(int LK, int N) {
  return std::max(1, std::min({64, 16384 / LK, (N + 127) / 128}));
}

// The positions [blockIdx.x cpw, ..) built from their records into LDS (smem:
// child rows | codes | selections) and stored; the rows stay in LDS.
__device__ __forceinline__ void island_build_chunk(const IslandArgs &a, const IslandRec *rec,
                                                   int cpw, unsigned char *smem) {
  const int L = a.L, K = a.K, LK = L * K, tid = threadIdx.x, block = blockDim.x;
  const int s0 = blockIdx.x * cpw, nc = min(cpw, a.N - s0);
  const int cb = (cpw * LK + 15) / 16 * 16;
  uint8_t *child = smem;
  uint8_t *codes = smem + cb;
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + 2 * cb);  // parents, cutg per position
  int32_t *sIsl = sSel + 2 * cpw;                                // island, or -1 for an elite
  if (tid < nc) {
    const IslandRec r = rec[s0 + tid];
    sSel[2 * tid] = r.parents;
    sSel[2 * tid + 1] = r.cutg;
    sIsl[tid] = r.elite ? -1 : r.island;
  }
  __syncthreads();
  const bool mutate = K >= 2 && a.ga.thr_mut != 0;
  // mutation codes of the children (not of the elites), one thread per
  // (position, group of 32 genes), the island index in the block counter
  if (mutate) {
    const int ng = (LK + 31) >> 5;
    for (int t = tid; t < nc * ng; t += block) {
      const int cpos = t / ng, q = t - cpos * ng;
      const int isl = sIsl[cpos];
      if (isl < 0) continue;
      uint32_t out[8];
      group_codes(q, LK, K, a.ga, a.gen, (uint32_t)(s0 + cpos), out, (uint32_t)isl << 16);
      uint8_t *dst = codes + (size_t)cpos * LK;
#pragma unroll
      for (int w = 0; w < 8; ++w)
        if (32 * q + 4 * w < LK) store_code_word(dst, LK, 8 * q + w, out[w]);
    }
  }
  // rows [0, cut) from the first parent and [cut, L) from the other: two
  // byte ranges per position, a team of threads per range
  {
    const int nr = 2 * nc;
    int lg = 0;
    while ((2 << lg) * nr <= block) ++lg;
    const int tpr = 1 << lg;
    const int sub = tid & (tpr - 1);
    for (int r0 = tid >> lg; r0 < nr; r0 += block >> lg) {
      const int cpos = r0 >> 1;
      const uint32_t pr = (uint32_t)sSel[2 * cpos];
      const int cutg = sSel[2 * cpos + 1];
      if ((r0 & 1) == 0)
        gather_range(ByteRange{a.pin + (size_t)(pr & 0xFFFFu) * LK, cutg}, child, cpos * LK, sub,
                     tpr);
      else
        gather_range(ByteRange{a.pin + (size_t)(pr >> 16) * LK + cutg, LK - cutg}, child,
                     cpos * LK + cutg, sub, tpr);
    }
  }
  __syncthreads();
  if (mutate) {
    for (int r = tid; r < nc * L; r += block) {
      if (sIsl[r / L] < 0) continue;
      const int off = r * K;
      apply_swaps(child + off, codes + off, off, K);
    }
    __syncthreads();
  }
  store_bytes(a.pout + (size_t)s0 * LK, child, nc * LK);
}

// LDS bytes of island_build_chunk for cpw positions of LK genes.
__host__ __device__ inline int island_build_lds(int cpw, int LK) {
  const int cb = (cpw * LK + 15) / 16 * 16;
  return 2 * cb + (3 * (int)sizeof(int32_t) * cpw + 15) / 16 * 16;
}

__global__ __launch_bounds__(kIslandThreads) void k_island_build(IslandArgs a,
                                                                 const IslandRec *rec,
                                                                 int cpw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  island_build_chunk(a, rec, cpw, smem);
}

// The fitness of the new population, when the build evaluates it too.
struct IslandFit {
  const float *T2;  // the instance's table [L][L][TP] (asymptotic SE)
  float *fit_out;   // [N]
  float prelog;
  int objective;
};

// Build and fitness in one launch for tables that fit LDS in the quad layout
// (asymptotic SE, L of 7 or 19): the table is staged while the chunk is
// built, then the chunk's rows (still in LDS) are inverted and evaluated by
// the fitness kernels' own quad sums and pilot reduction, so every position
// gets the bits pa_fitness would give it.  cpw * K <= the workgroup size.
template <int LT, int TPT>
__global__ __launch_bounds__(kIslandThreads) void k_island_build_fit(IslandArgs a,
                                                                     const IslandRec *rec,
                                                                     int cpw, IslandFit f) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int LP = quad_rows<LT>();
  constexpr int kQuadBytes = LT * TPT * LP * 4;
  float *sQ = reinterpret_cast<float *>(smem);
  load_quad(f.T2, LT, TPT, 0, LT, LP, sQ);  // published by the build's barriers
  unsigned char *b = smem + kQuadBytes;
  island_build_chunk(a, rec, cpw, b);      // ends with the final rows in LDS, after a barrier
  const int K = a.K, block = (int)blockDim.x, q = (int)threadIdx.x;
  const int s0 = blockIdx.x * cpw, nc = min(cpw, a.N - s0);
  const uint8_t *child = b;
  uint8_t *sInv = b + island_build_lds(cpw, LT * K);
  float *sE = reinterpret_cast<float *>(sInv + (block * LT + 15) / 16 * 16);
  build_inverse(child, nc * LT, LT, K, sInv);
  __syncthreads();
  const bool active = q / K < nc;
  const float acc = lane_sum_quad<LT, TPT>(sInv + q * LT, active, sQ, f.objective);
  reduce_round(sE, acc, active, nc, K, f.prelog, f.fit_out + s0, f.objective);
}

template <int LT, int TPT>
hipError_t launch_build_fit(const IslandArgs &a, const IslandRec *rec, int cpw,
                            const IslandFit &f, hipStream_t s) {
  const int LK = LT * a.K;
  const int lds = LT * TPT * quad_rows<LT>() * 4 + island_build_lds(cpw, LK) +
                  (kIslandThreads * LT + 15) / 16 * 16 + kIslandThreads * 4;
  static LdsAttr attr;
  const hipError_t ae =
      allow_lds_once(attr, reinterpret_cast<const void *>(k_island_build_fit<LT, TPT>), kLdsBytes);
  hipLaunchKernelGGL((k_island_build_fit<LT, TPT>), dim3((a.N + cpw - 1) / cpw),
                     dim3(kIslandThreads), lds, s, a, rec, cpw, f);
  return launch_status(ae);
}

__global__ void k_trace_best(const float *fit, int N, float *trace_g) {
  // best fitness of a population into one trace entry (one wave)
  uint64_t b = 0;
  for (int n = threadIdx.x; n < N; n += kWave) {
    const uint64_t k = full_key(gp(fit)[n], (uint32_t)n);
    b = k > b ? k : b;
  }
  b = wave_max_u64(b);
  if (threadIdx.x == 0) *gp(trace_g) = gp(fit)[key_index(b)];
}

hipError_t launch_trace_best(const float *fit, int N, float *trace_g, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_best, dim3(1), dim3(kWave), 0, s, fit, N, trace_g);
  return hipGetLastError();
}

int kmeans_lds(int N, int LK, int C) {
  return (C * LK + 15) / 16 * 16 + 8 * N + 8 * (kKmThreads / kWave) + 4 * (2 + kIslandMaxC);
}

hipError_t launch_pop_kmeans(const uint8_t *pop, const float *fit, int N, int LK, int C,
                             int max_iters, int32_t *labels, int32_t *iters, hipStream_t s) {
  PopKmArgs a{pop, fit, N, LK, C, max_iters, labels, iters};
  const int resident = kmeans_lds_resident(N, LK, C);
  if (resident <= kLdsBytes) {
    static LdsAttr attr_r;
    const hipError_t ae =
        allow_lds_once(attr_r, reinterpret_cast<const void *>(k_pop_kmeans_lds), kLdsBytes);
    hipLaunchKernelGGL(k_pop_kmeans_lds, dim3(1), dim3(kKmThreads), resident, s, a);
    return launch_status(ae);
  }
  static LdsAttr attr;
  const int lds = kmeans_lds(N, LK, C);
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(k_pop_kmeans), kLdsBytes);
  hipLaunchKernelGGL(k_pop_kmeans, dim3(1), dim3(kKmThreads), lds, s, a);
  return launch_status(ae);
}

// One generation of every island: plan (one workgroup per island, and one
// for the positions of no island and, with trace_g, the trace entry), then
// build (positions in chunks).  rec: N records of device scratch.  With
// fit_out, the build also evaluates the new population when the table fits
// the fused form (*evaluated set to true; else the caller evaluates it).
hipError_t launch_island_step(const DevProblem &p, const DevGa &ga, int C, uint32_t gen,
                              const int32_t *labels, const uint8_t *pin, const float *fin,
                              uint8_t *pout, IslandRec *rec, hipStream_t s,
                              float *trace_g = nullptr, float *fit_out = nullptr,
                              bool *evaluated = nullptr) {
  IslandArgs a{pin, fin, pout, labels, ga.N, ga.E, p.L, p.K, C, gen, ga, trace_g};
  if (evaluated) *evaluated = false;
  hipLaunchKernelGGL(k_island_plan, dim3(C + 1), dim3(kIslandThreads), 0, s, a, rec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int LK = p.L * p.K, cpw = island_chunk(LK, ga.N);
  if (fit_out && p.se_mode == 0 && (p.L == 7 || p.L == 19) && p.TP <= 32) {
    const int cpf = std::max(1, std::min(cpw, kIslandThreads / p.K));
    const IslandFit f{p.T2, fit_out, p.prelog, p.objective};
    hipError_t ef = hipErrorInvalidValue;
#define PA_BUILD_FIT(LV, TV) \
  if (p.L == LV && p.TP == TV) ef = launch_build_fit<LV, TV>(a, rec, cpf, f, s);
    PA_BUILD_FIT(7, 4) PA_BUILD_FIT(7, 8) PA_BUILD_FIT(7, 16) PA_BUILD_FIT(7, 32)
    PA_BUILD_FIT(19, 4) PA_BUILD_FIT(19, 8) PA_BUILD_FIT(19, 16) PA_BUILD_FIT(19, 32)
#undef PA_BUILD_FIT
    if (ef == hipSuccess && evaluated) *evaluated = true;
    return ef;
  }
  hipLaunchKernelGGL(k_island_build, dim3((ga.N + cpw - 1) / cpw), dim3(kIslandThreads),
                     island_build_lds(cpw, LK), s, a, rec, cpw);
  return hipGetLastError();
}

pa_status island_check(const pa_instance *in, int N, int C, int max_iters) {
  if (C < 1 || C > kIslandMaxC) return set_error(PA_EINVAL, "clusters=%d outside [1, %d]", C, kIslandMaxC);
  if (N > kIslandMaxN) return set_error(PA_EINVAL, "island GA: pop=%d above %d", N, kIslandMaxN);
  if (C > N) return set_error(PA_EINVAL, "clusters=%d above pop=%d", C, N);
  if (max_iters < 1) return set_error(PA_EINVAL, "kmeans_iters=%d must be >= 1", max_iters);
  if (kmeans_lds(N, in->p.L * in->p.K, C) > kLdsBytes)
    return set_error(PA_EUNSUPPORTED, "population K-means does not fit LDS");
  return PA_OK;
}

#define ITRY(call, what)                              \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_population_kmeans(pa_instance *in, int32_t clusters, int32_t kmeans_iters,
                               const uint8_t *d_pop, const float *d_fit, int32_t n,
                               int32_t *d_labels, void *stream) {
  if (!in || !d_pop || !d_fit || !d_labels) return set_error(PA_EINVAL, "NULL argument");
  if (n < 1) return set_error(PA_EINVAL, "n=%d must be >= 1", n);
  pa_status st = island_check(in, n, clusters, kmeans_iters);
  if (st != PA_OK) return st;
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  ITRY(launch_pop_kmeans(d_pop, d_fit, n, in->p.L * in->p.K, clusters, kmeans_iters, d_labels,
                         nullptr, (hipStream_t)stream),
       "pa_population_kmeans");
  return PA_OK;
}

pa_status pa_island_step(pa_instance *in, const pa_ga_params *g, int32_t clusters, int32_t gen,
                         const int32_t *d_labels, const uint8_t *d_pop_in, const float *d_fit_in,
                         uint8_t *d_pop_out, void *stream) {
  if (!in || !d_labels || !d_pop_in || !d_fit_in || !d_pop_out)
    return set_error(PA_EINVAL, "NULL argument");
  if (d_pop_in == d_pop_out) return set_error(PA_EINVAL, "d_pop_in and d_pop_out must differ");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if ((st = island_check(in, g->pop, clusters, 1)) != PA_OK) return st;
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  IslandRec *rec = nullptr;
  ITRY(hipMallocAsync(reinterpret_cast<void **>(&rec), sizeof(IslandRec) * g->pop, s),
       "pa_island_step scratch");
  const hipError_t e = launch_island_step(in->p, ga_from_params(g), clusters, (uint32_t)gen,
                                          d_labels, d_pop_in, d_fit_in, d_pop_out, rec, s);
  const hipError_t ef = hipFreeAsync(rec, s);
  ITRY(e, "pa_island_step");
  ITRY(ef, "pa_island_step scratch");
  return PA_OK;
}

pa_status pa_island_solve(pa_instance *in, const pa_ga_params *g, int32_t clusters,
                          int32_t recluster_every, int32_t kmeans_iters, pa_result *out,
                          int32_t *labels, void *stream) {
  if (in && g && g->pop < 1) return set_error(PA_EINVAL, "pop=%d must be >= 1", g->pop);
  if (!in || !out) return set_error(PA_EINVAL, "instance or result is NULL");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if ((st = island_check(in, g->pop, clusters, kmeans_iters)) != PA_OK) return st;
  if (recluster_every < 0) return set_error(PA_EINVAL, "recluster_every=%d < 0", recluster_every);
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  const int N = g->pop, G = g->gens, LK = in->p.L * in->p.K;
  hipStream_t s = (hipStream_t)stream;
  // work buffers: two populations, two fitness arrays, labels, trace, best
  uint8_t *pop[2] = {nullptr, nullptr};
  float *fit[2] = {nullptr, nullptr};
  int32_t *lab = nullptr, *bidx = nullptr;
  float *trace = nullptr, *bfit = nullptr;
  IslandRec *rec = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    for (void *p : {(void *)pop[0], (void *)pop[1], (void *)fit[0], (void *)fit[1], (void *)lab,
                    (void *)bidx, (void *)trace, (void *)bfit, (void *)rec})
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipMalloc(&pop[b], (size_t)LK * N);
    if (e == hipSuccess) e = hipMalloc(&fit[b], sizeof(float) * N);
  }
  if (e == hipSuccess) e = hipMalloc(&lab, sizeof(int32_t) * N);
  if (e == hipSuccess) e = hipMalloc(&bidx, sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&trace, sizeof(float) * (G + 1));
  if (e == hipSuccess) e = hipMalloc(&bfit, sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&rec, sizeof(IslandRec) * N);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(lab, 0, sizeof(int32_t) * N, s);
  const DevGa ga = ga_from_params(g);
  FitShape fs;
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess && ga.n_km > 0) e = launch_kmeans_seed(in->p, s);
  if (e == hipSuccess) e = launch_init_pop(in->p, ga, pop[0], s);
  if (e == hipSuccess) e = launch_fitness(in->p, pop[0], N, fit[0], fs, in->ctx->info, s);
  for (int gen = 0; gen < G && e == hipSuccess; ++gen) {
    const int a = gen & 1, b = 1 - a;
    // Alg. 2: apply K-means (at 0, then every recluster_every generations)
    if (clusters > 1 &&
        (gen == 0 || (recluster_every > 0 && gen % recluster_every == 0)))
      e = launch_pop_kmeans(pop[a], fit[a], N, LK, clusters, kmeans_iters, lab, nullptr, s);
    bool evaluated = false;
    if (e == hipSuccess)
      e = launch_island_step(in->p, ga, clusters, (uint32_t)gen, lab, pop[a], fit[a], pop[b], rec,
                             s, trace + gen, fit[b], &evaluated);
    if (e == hipSuccess && !evaluated)
      e = launch_fitness(in->p, pop[b], N, fit[b], fs, in->ctx->info, s);
  }
  const int fin = G & 1;
  if (e == hipSuccess) e = launch_trace_best(fit[fin], N, trace + G, s);
  if (e == hipSuccess) e = launch_best(fit[fin], N, bidx, bfit, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  int32_t hidx = 0;
  float hfit = 0.0f;
  std::vector<float> htrace(G + 1);
  if (e == hipSuccess) e = hipMemcpyAsync(&hidx, bidx, sizeof hidx, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hfit, bfit, sizeof hfit, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(htrace.data(), trace, sizeof(float) * (G + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && out->best)
    e = hipMemcpy(out->best, pop[fin] + (size_t)hidx * LK, LK, hipMemcpyDeviceToHost);
  if (e == hipSuccess && labels)
    e = hipMemcpy(labels, lab, sizeof(int32_t) * N, hipMemcpyDeviceToHost);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  release();
  if (e != hipSuccess) return hip_error(e, "pa_island_solve");
  out->best_fit = hfit;
  out->best_index = hidx;
  if (out->trace) std::memcpy(out->trace, htrace.data(), sizeof(float) * (G + 1));
  out->device_ms = ms;
  return PA_OK;
}

}  // extern "C"
