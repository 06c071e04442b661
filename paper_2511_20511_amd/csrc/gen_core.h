// gen_core.h -- the fused generation kernel: one launch runs a whole GA
// generation (Alg. 1 loop body: select and evolve, then evaluate) for every
// task of a class of instances.  A workgroup takes a contiguous chunk of
// tasks; per child task it
//   1. builds up to CPR = block/K children in LDS with the whole workgroup
//      (tournaments, cell-axis crossover, swap mutation; ga_core.h),
//   2. writes them to the output population and inverts their rows in LDS,
//   3. evaluates them against the LDS-staged table (fitness_core.h),
// so a child never goes back to HBM before its fitness is known.  The elite
// task of an instance copies its E best chromosomes and their fitness.
#pragma once
#include "fitness_core.h"
#include "ga_core.h"

namespace pa {

struct GenArgs {
  const GenInst *insts;
  const GenTask *tasks;
  const int32_t *bounds;  // null: runs of equal task counts (see task_range)
  int ntasks;
  int gen;             // -1: fitness of the initial populations
  const int32_t *gens; // non-null: a task's generation is gens[task.inst] (gen ignored)
};

// The range of tasks of this workgroup in a launch of `ntasks` tasks: the
// tasks are cut into gridDim.x contiguous runs, [bounds[r], bounds[r + 1])
// when bounds is given (cut by the host by task cost), else runs whose
// lengths differ by at most one, and the runs are dealt so that the
// workgroups of one XCD take neighbouring runs.  Workgroup b is dispatched to
// XCD b % 8, so the workgroups of an XCD share the instances (tables,
// populations) of a contiguous 1/8 of the task list, and its L2 serves them.
constexpr int kXcds = 8;
__device__ __forceinline__ void task_range(int ntasks, const int32_t *bounds, int &t0, int &t1) {
  const int b = blockIdx.x, G = gridDim.x;
  const int x = b % kXcds, r = b / kXcds, per = G / kXcds, rem = G % kXcds;
  const int run = x * per + min(x, rem) + r;  // a bijection of [0, G)
  if (bounds) {
    t0 = __builtin_amdgcn_readfirstlane(gp(bounds)[run]);
    t1 = __builtin_amdgcn_readfirstlane(gp(bounds)[run + 1]);
    return;
  }
  t0 = (int)(((int64_t)run * ntasks) / G);
  t1 = (int)(((int64_t)(run + 1) * ntasks) / G);
}

// LDS plan: table tile | children (<= block*L) | inverse rows (<= block*L) |
// sums (block*4) | elite indices (64 ints) |
// own-cell squares | parents and cut per child | with PF (persistent form) the
// tournament candidates of the task's pairs (4 chromosomes per pair; reused
// for the per-row SE terms of the split lane sum), their selection words (6
// ints per pair) and their outcome (4 ints per pair) | the children's
// mutation codes (<= block*L).
template <int LT, int TPT, int MODE, int BLOCK, bool PF = false>
struct GenPlan {
  static constexpr int kChildBytes = ((BLOCK * LT) + 15) / 16 * 16;
  static constexpr int kInvBytes = kChildBytes;
  static constexpr int kEBytes = BLOCK * 4;
  static constexpr int kIdxBytes = 256;
  static constexpr int kOwnBytes = LT * TPT * 4;  // own-cell squares (tiled tables)
  static constexpr int kSelBytes = BLOCK * 8;     // parents and cut per child
  static constexpr int kMaxPairs = BLOCK / 2 + 2;
  static constexpr int kCandBytes = PF ? (2 * BLOCK * LT + 6 * LT * TPT + 15) / 16 * 16 : 0;
  static constexpr int kPairBytes = PF ? kMaxPairs * 24 : 0;
  static constexpr int kResBytes = PF ? kMaxPairs * 16 : 0;
  static constexpr int kCodeBytes = kChildBytes;  // mutation codes
  using T = TilePlan<LT, TPT, MODE,
                     kChildBytes + kInvBytes + kEBytes + kIdxBytes + kOwnBytes + kSelBytes +
                         kCandBytes + kPairBytes + kResBytes + kCodeBytes>;
  static constexpr int kTiles = T::kTiles;
  static constexpr int kTileRows = T::kTileRows;
  // an asymptotic-SE table that fits whole in its quad layout is staged that
  // way (four BS rows per 16-byte gather)
  static constexpr int kQuadBytes = LT * TPT * quad_rows<LT>() * 4;
  static constexpr bool kQuad = MODE == 0 && kTiles == 1 && kQuadBytes <= T::kBudget;
  static constexpr int kChildOff = kQuad ? kQuadBytes : T::kTableBytes;
  static constexpr int kInvOff = kChildOff + kChildBytes;
  static constexpr int kEOff = kInvOff + kInvBytes;
  static constexpr int kIdxOff = kEOff + kEBytes;
  static constexpr int kOwnOff = kIdxOff + kIdxBytes;
  static constexpr int kSelOff = kOwnOff + kOwnBytes;
  static constexpr int kCandOff = kSelOff + kSelBytes;
  static constexpr int kPairOff = kCandOff + kCandBytes;
  static constexpr int kResOff = kPairOff + kPairBytes;
  static constexpr int kCodeOff = kResOff + kResBytes;
  static constexpr int kTotal = kCodeOff + kCodeBytes;
  static_assert(kTotal <= kLdsBytes, "LDS plan too large");
};

// A task read with scalar loads (task lists are read-only while a launch
// runs); t must be wave-uniform.
__device__ __forceinline__ GenTask load_task(const GenTask *tasks, int t) {
  typedef __attribute__((address_space(4))) const int32_t *cwords;
  const cwords p = (cwords)reinterpret_cast<const int32_t *>(tasks + __builtin_amdgcn_readfirstlane(t));
  return GenTask{p[0], p[1], p[2], p[3]};
}

// A finished child row of K bytes (K % 16 == 0, n16 = K / 16) from LDS
// (rowb) to the output population (gdst) as whole 16-byte words, and its
// inverse entries: dst[t * L] = the position of pilot t in the row.  Both
// rows are 16-byte aligned (LDS rows and population rows of a multiple of 16
// bytes).
__device__ __forceinline__ void store_row_inverse16(const uint8_t *rowb, uint8_t *gdst,
                                                    uint8_t *dst, int n16, int K, int L) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 *row = reinterpret_cast<const u32x4 *>(rowb);
  gptr<u32x4> gw = gp(reinterpret_cast<u32x4 *>(gdst));
  for (int h = 0; h < n16; ++h) {
    const u32x4 x4 = row[h];
    gw[h] = x4;
    const uint32_t xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int t = (int)((xs[w] >> (8 * b)) & 0xFFu);
        if (t < K) dst[t * L] = (uint8_t)(16 * h + 4 * w + b);
      }
  }
}

// The children's rows straight from their parents (K % 4 == 0, K <= 32;
// parents and cut in sSel as build_children_block leaves them), one thread
// per row (c, j), the loads of two rows in flight per thread: the crossover
// cuts between rows, so row j comes whole from the first parent when j < cut
// and from the second otherwise; then the row's swaps, its write-out and its
// inverse entries.  Ends with a barrier.
__device__ __forceinline__ void rows_from_parents(const uint8_t *__restrict__ pin,
                                                  const int32_t *sSel, const uint8_t *sCode,
                                                  int nc, int L, int K, bool mutate,
                                                  uint8_t *sChild, uint8_t *pout, uint8_t *sInv,
                                                  int block) {
  const int LK = L * K, nw = K >> 2, rows = nc * L;
  for (int r = threadIdx.x; r < rows; r += 2 * block) {
    uint32_t v[2][8];  // K <= 32
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = min(r + h * block, rows - 1);  // clamped: every load is in bounds
      const int c = q / L, j = q - c * L;
      const uint32_t pr = (uint32_t)sSel[2 * c];
      const uint32_t par = j * K < sSel[2 * c + 1] ? (pr & 0xFFFFu) : (pr >> 16);
      const gptr<const uint32_t> src =
          gp(reinterpret_cast<const uint32_t *>(pin + (size_t)par * LK + j * K));
#pragma unroll
      for (int w = 0; w < 8; ++w) v[h][w] = w < nw ? src[w] : 0u;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = r + h * block;
      if (q < rows) {
        const int c = q / L, j = q - c * L;
        uint32_t *row = reinterpret_cast<uint32_t *>(sChild + q * K);
#pragma unroll
        for (int w = 0; w < 8; ++w)
          if (w < nw) row[w] = v[h][w];
        if (mutate) apply_swaps(sChild + q * K, sCode + q * K, q * K, K);
        uint8_t *dst = sInv + c * K * L + j;
        if ((K & 15) == 0) {
          store_row_inverse16(sChild + q * K, pout + (size_t)q * K, dst, K >> 4, K, L);
          continue;
        }
        gptr<uint32_t> gw = gp(reinterpret_cast<uint32_t *>(pout + (size_t)q * K));
        for (int w = 0; w < nw; ++w) {
          const uint32_t x = row[w];
          gw[w] = x;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int t = (int)((x >> (8 * b)) & 0xFFu);
            if (t < K) dst[t * L] = (uint8_t)(4 * w + b);
          }
        }
      }
    }
  }
  __syncthreads();
}

// Everything of a task but the fitness evaluation; returns the number of
// chromosomes to evaluate (0 for an elite task or a finished instance).
// Leaves their inverse rows in sInv and ends with a barrier.  sCode: the
// mutation codes (may alias sInv; apart from it, and with K % 4 == 0, the
// rows are taken from the parents, swapped, written out and inverted in one
// pass).
__device__ __forceinline__ int gen_prepare(const GenInst &I, const GenTask &task, int gen,
                                           uint8_t *sChild, uint8_t *sInv, uint8_t *sCode,
                                           int32_t *sIdx, int32_t *sSel, int block) {
  const int L = I.L, K = I.K, LK = L * K;
  const int in = gen < 0 ? 0 : (gen & 1);
  const int out = gen < 0 ? 0 : 1 - in;
  if (task.kind == kTaskElite) {
    copy_elites_block(pop_buf(I, in), fit_buf(I, in), I.N, I.E, LK, pop_buf(I, out),
                      fit_buf(I, out), I.trace, gen, sIdx);
    return 0;
  }
  const int nc = task.s1 - task.s0;
  if (task.kind == kTaskChild) {
    const bool merged = sCode != sInv && (K & 3) == 0 && K <= 32;
    build_children_block(pop_buf(I, in), fit_buf(I, in), I.N, I.E, L, K, I.ga, (uint32_t)gen,
                         task.s0, nc, sChild, sCode, sSel, block,
                         merged ? kBuildSelect : kBuildAll);
    if (merged) {
      rows_from_parents(pop_buf(I, in), sSel, sCode, nc, L, K, K >= 2 && I.ga.thr_mut != 0,
                        sChild, pop_buf(I, out) + (size_t)task.s0 * LK, sInv, block);
      return nc;
    }
    store_bytes(pop_buf(I, out) + (size_t)task.s0 * LK, sChild, nc * LK);
    build_inverse(sChild, nc * L, L, K, sInv);
  } else {
    copy_bytes(pop_buf(I, in) + (size_t)task.s0 * LK, nc * LK, sChild);
    __syncthreads();
    build_inverse(sChild, nc * L, L, K, sInv);
  }
  __syncthreads();
  return nc;
}

// ---- persistent form: a child task prepared ahead ----------------------
//
// Everything of a child task that depends only on (seed, slots, generation)
// -- its pairs' SELECT words and its children's mutation codes -- is
// computed before the grid barrier that precedes the generation; after the
// barrier one round trip fetches the fitness of the tournament candidates
// together with the candidates' chromosomes (4 per pair), and the children
// are assembled from LDS.  Same draws, same children as gen_prepare.

struct PairSpan {
  int pa0, np;  // first pair index (slot E + 2*pa0) and pairs of the task
};
__device__ __forceinline__ PairSpan pair_span(const GenInst &I, const GenTask &task) {
  const int pa0 = (task.s0 - I.E) >> 1;
  return PairSpan{pa0, ((task.s1 - 1 - I.E) >> 1) - pa0 + 1};
}

// SELECT words of the task's pairs into sPair (6 per pair: u0, v0, u1, v1,
// crossover word, cut word) and mutation codes of its children into codes.
// Every thread must call it; no barrier (the caller's next one publishes the
// results: a workgroup barrier here, ahead of the grid barrier, measurably
// lengthens every generation).
__device__ __forceinline__ void pf_precompute(const GenInst &I, const GenTask &task, int gen,
                                              uint8_t *codes, int32_t *sPair, int block) {
  const int N = I.N, K = I.K, LK = I.L * K;
  const PairSpan ps = pair_span(I, task);
  const int tid = threadIdx.x;
  const DevGa &ga = I.ga;
  if (tid < ps.np) {
    const uint32_t a = (uint32_t)(I.E + 2 * (ps.pa0 + tid));
    const Stream st{ga.seed_lo, ga.seed_hi, a, (uint32_t)gen, ga.instance_id, kTagSelect};
    const Words4 b0 = st.block(0u), b1 = st.block(1u);
    int32_t *w = sPair + 6 * tid;
    w[0] = (int32_t)bounded(b0.x, (uint32_t)N);
    w[1] = (int32_t)bounded(b0.y, (uint32_t)N);
    w[2] = (int32_t)bounded(b0.z, (uint32_t)N);
    w[3] = (int32_t)bounded(b0.w, (uint32_t)N);
    w[4] = (int32_t)b1.x;
    w[5] = (int32_t)b1.y;
  }
  if (K >= 2 && ga.thr_mut != 0)
    mutation_codes_block(codes, task.s1 - task.s0, LK, K, ga, (uint32_t)gen, task.s0, block);
}

// The children of a prepared task (pf_precompute of this generation done and
// followed by a barrier; codes in sCode): tournaments, crossover and swaps,
// write-out and inverse rows; returns the number of children.  Ends with a
// barrier.
__device__ __forceinline__ int pf_build(const GenInst &I, const GenTask &task, int gen,
                                        uint8_t *sChild, uint8_t *sInv, uint8_t *sCand,
                                        const int32_t *sPair, int32_t *sRes,
                                        const uint8_t *sCode, int block) {
  const int L = I.L, K = I.K, LK = L * K, E = I.E;
  const int in = gen & 1, out = 1 - in;
  const uint8_t *pin = pop_buf(I, in);
  const float *fin = fit_buf(I, in);
  const PairSpan ps = pair_span(I, task);
  const int nc = task.s1 - task.s0;
  const int tid = threadIdx.x;
  // 1. one round trip: the candidates' fitness and chromosomes
  float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, f3 = 0.0f;
  if (tid < ps.np) {
    const int32_t *w = sPair + 6 * tid;
    f0 = gp(fin)[w[0]];
    f1 = gp(fin)[w[1]];
    f2 = gp(fin)[w[2]];
    f3 = gp(fin)[w[3]];
  }
  {
    const int nr = 4 * ps.np;
    int lg = 0;
    while ((2 << lg) * nr <= block) ++lg;
    const int tpr = 1 << lg;
    const int sub = tid & (tpr - 1);
    for (int r = tid >> lg; r < nr; r += block >> lg) {
      const int idx = sPair[6 * (r >> 2) + (r & 3)];
      gather_range(ByteRange{pin + (size_t)idx * LK, LK}, sCand, r * LK, sub, tpr);
    }
  }
  if (tid < ps.np) {
    const int32_t *w = sPair + 6 * tid;
    const uint32_t u0 = (uint32_t)w[0], v0 = (uint32_t)w[1];
    const uint32_t u1 = (uint32_t)w[2], v1 = (uint32_t)w[3];
    const bool c1 = beats(rank_key(f1), v0, rank_key(f0), u0);
    const bool c2 = beats(rank_key(f3), v1, rank_key(f2), u1);
    const bool cross = L >= 2 && hit((uint32_t)w[4], I.ga.thr_cross);
    const int cut = cross ? 1 + (int)bounded((uint32_t)w[5], (uint32_t)(L - 1)) : L;
    sRes[4 * tid] = c1 ? 1 : 0;      // candidate slot of parent 1
    sRes[4 * tid + 1] = c2 ? 3 : 2;  // candidate slot of parent 2
    sRes[4 * tid + 2] = cut * K;
  }
  __syncthreads();
  const bool mutate = K >= 2 && I.ga.thr_mut != 0;
  uint8_t *pout = pop_buf(I, out) + (size_t)task.s0 * LK;
  if ((K & 3) == 0) {
    // 2+3. one thread per row (c, j), rows whole aligned words: the crossover
    // cuts between rows, so the row is copied whole from its parent (rows
    // before the cut from the first, the others from the second), then its
    // swaps, its write-out and its inverse entries
    for (int r = tid; r < nc * L; r += block) {
      const int c = r / L, j = r - c * L;
      const int slot = task.s0 + c;
      const int lp = ((slot - E) >> 1) - ps.pa0;
      const bool second = ((slot - E) & 1) != 0;
      const int32_t *res = sRes + 4 * lp;
      const int fs = second ? res[1] : res[0], rs = second ? res[0] : res[1];
      const int src = j * K < res[2] ? fs : rs;
      const uint32_t *from = reinterpret_cast<const uint32_t *>(sCand + (4 * lp + src) * LK + j * K);
      uint32_t *row = reinterpret_cast<uint32_t *>(sChild + r * K);
      for (int w = 0; w < (K >> 2); ++w) row[w] = from[w];
      if (mutate) apply_swaps(sChild + r * K, sCode + r * K, r * K, K);
      gptr<uint32_t> gw = gp(reinterpret_cast<uint32_t *>(pout + (size_t)r * K));
      uint8_t *dst = sInv + c * K * L + j;
      for (int w = 0; w < (K >> 2); ++w) {
        const uint32_t v = row[w];
        gw[w] = v;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int t = (int)((v >> (8 * b)) & 0xFFu);
          if (t < K) dst[t * L] = (uint8_t)(4 * w + b);
        }
      }
    }
    __syncthreads();
    return nc;
  }
  // 2. child c = first parent's genes [0, cut) + second's [cut, LK), one
  // power-of-two team of threads per child, 32-bit words when LK % 4 == 0
  {
    int lg = 0;
    while ((2 << lg) * nc <= block) ++lg;
    const int tpr = 1 << lg, sub = tid & (tpr - 1);
    for (int c = tid >> lg; c < nc; c += block >> lg) {
      const int slot = task.s0 + c;
      const int lp = ((slot - E) >> 1) - ps.pa0;
      const bool second = ((slot - E) & 1) != 0;
      const int32_t *res = sRes + 4 * lp;
      const int r0 = res[0], r1 = res[1], cutg = res[2];
      const int fs = second ? r1 : r0, rs = second ? r0 : r1;
      const uint8_t *cf = sCand + (4 * lp + fs) * LK, *cr = sCand + (4 * lp + rs) * LK;
      uint8_t *dst = sChild + c * LK;
      if ((LK & 3) == 0) {
        for (int w = sub; w < (LK >> 2); w += tpr) {
          const int g = 4 * w;
          uint32_t v;
          if (g + 4 <= cutg) {
            v = *reinterpret_cast<const uint32_t *>(cf + g);
          } else if (g >= cutg) {
            v = *reinterpret_cast<const uint32_t *>(cr + g);
          } else {
            const uint32_t a = *reinterpret_cast<const uint32_t *>(cf + g);
            const uint32_t b = *reinterpret_cast<const uint32_t *>(cr + g);
            const uint32_t m = 0xFFFFFFFFu >> (8 * (4 - (cutg - g)));  // bytes below cutg
            v = (a & m) | (b & ~m);
          }
          *reinterpret_cast<uint32_t *>(dst + g) = v;
        }
      } else {
        for (int g = sub; g < LK; g += tpr) dst[g] = g < cutg ? cf[g] : cr[g];
      }
    }
  }
  __syncthreads();
  // 3. the swaps (K % 4 != 0)
  if (mutate) {
    for (int r = tid; r < nc * L; r += block) apply_swaps(sChild + r * K, sCode + r * K, r * K, K);
  }
  __syncthreads();
  // 4. write-out and inverse rows
  store_bytes(pout, sChild, nc * LK);
  build_inverse(sChild, nc * L, L, K, sInv);
  __syncthreads();
  return nc;
}

// What a workgroup's LDS holds between tasks: the instance whose table (or,
// tiled, whose own-cell squares) it holds, and with tiled tables which tile.
struct LdsState {
  int inst = -1;
  int tile = -1;
};

// One task of one generation for a workgroup of the unrolled kernel.  I is a
// copy of the instance descriptor in registers, read before the task's first
// global store: a descriptor field loaded after a store would make its wait
// (the vector-memory counter is in order) wait for the store as well.
// `prepared`: the child task's draws were made ahead (persistent form).
// KIND >= 0: the task is known to be of that kind (only its code is built).
template <int LT, int TPT, int MODE, int BLOCK, bool PF = false, int KIND = -1>
__device__ __forceinline__ void run_task(const GenInst &I, const GenTask &task_in, int gen,
                                         unsigned char *smem, LdsState &st, bool prepared) {
  GenTask task = task_in;
  if constexpr (KIND >= 0) task.kind = KIND;
  using P = GenPlan<LT, TPT, MODE, BLOCK, PF>;
  constexpr int NT = P::kTiles;
  constexpr int TR = P::kTileRows;
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sChild = smem + P::kChildOff;
  uint8_t *sInv = smem + P::kInvOff;
  float *sE = reinterpret_cast<float *>(smem + P::kEOff);
  int32_t *sIdx = reinterpret_cast<int32_t *>(smem + P::kIdxOff);
  float *sOwn = reinterpret_cast<float *>(smem + P::kOwnOff);
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + P::kSelOff);
  uint8_t *sCode = smem + P::kCodeOff;
  if (gen >= I.G) return;  // this instance has finished its generations
  const int out = gen < 0 ? 0 : 1 - (gen & 1);
  float *const fit_out = fit_buf(I, out) + task.s0;
  const float prelog = I.prelog;
  const int mn = I.objective;
  if (task.kind != kTaskElite && task.inst != st.inst) {
    // every thread passed a barrier since the tables were last read
    if constexpr (P::kQuad)
      load_quad(I.T2, LT, TPT, 0, LT, quad_rows<LT>(), sT);
    else if constexpr (NT == 1)
      load_tile<MODE>(I.T2, I.T1, LT, TPT, 0, LT, TR, sT);
    else
      load_own(I.Town, LT, TPT, sOwn);
    st.inst = task.inst;
    st.tile = -1;
  }
  int nc;
  if constexpr (PF) {
    if (task.kind == kTaskChild) {
      int32_t *sPair = reinterpret_cast<int32_t *>(smem + P::kPairOff);
      if (!prepared) {
        pf_precompute(I, task, gen, sCode, sPair, BLOCK);
        __syncthreads();
      }
      nc = pf_build(I, task, gen, sChild, sInv, smem + P::kCandOff, sPair,
                    reinterpret_cast<int32_t *>(smem + P::kResOff), sCode, BLOCK);
    } else {
      nc = gen_prepare(I, task, gen, sChild, sInv, sCode, sIdx, sSel, BLOCK);
    }
  } else {
    nc = gen_prepare(I, task, gen, sChild, sInv, sCode, sIdx, sSel, BLOCK);
  }
  if (nc == 0) return;
  const int K = I.K;
  const int q = threadIdx.x;
  if constexpr (PF && NT == 1) {
    // few chromosomes (persistent tasks): split the BS rows over all waves
    const int lanes = nc * K;
    int GS = kWave;
    while (GS < lanes) GS <<= 1;
    if (GS < BLOCK) {
      const int rg = __builtin_amdgcn_readfirstlane(q / GS);
      const int ql = q - rg * GS;
      const bool act = ql < lanes;
      float acc;
      if constexpr (P::kQuad)
        acc = lane_sum_split_quad<LT, TPT>(sInv, ql, act, rg, BLOCK / GS, sT,
                                           reinterpret_cast<float *>(smem + P::kCandOff), mn);
      else
        acc = lane_sum_split<LT, TPT, MODE>(
            sInv, ql, act, rg, BLOCK / GS, sT, reinterpret_cast<float *>(smem + P::kCandOff),
            I.lconst, mn);
      reduce_round(sE, acc, act && rg == 0, nc, K, prelog, fit_out, mn);
      return;
    }
  }
  const bool active = q / K < nc;
  float acc;
  if constexpr (P::kQuad)
    acc = lane_sum_quad<LT, TPT>(sInv + q * LT, active, sT, mn);
  else if constexpr (NT == 1)
    acc = lane_sum_exact<LT, TPT, MODE, TR, 1>(sInv + q * LT, active, sT, I.T2, I.T1, I.lconst,
                                               mn);
  else
    acc = lane_sum_tiled<LT, TPT, MODE, TR>(sInv + q * LT, active, sT, sOwn, I.T2z, I.T1,
                                            I.lconst, st.tile, mn);
  reduce_round(sE, acc, active, nc, K, prelog, fit_out, mn);
}

// Tasks [t0, t1) of one generation for a workgroup (gens: per-instance
// generations, or null for `gen`).
template <int LT, int TPT, int MODE, int BLOCK, bool PF = false, int KIND = -1>
__device__ __forceinline__ void gen_tasks_exact(const GenInst *insts, const GenTask *tasks,
                                                int t0, int t1, int gen, unsigned char *smem,
                                                LdsState &st, const int32_t *gens = nullptr) {
  for (int t = t0; t < t1; ++t) {
    const GenTask task = load_task(tasks, t);
    const GenInst I = load_inst(insts, task.inst);
    const int g = gens ? gp(gens)[task.inst] : gen;
    run_task<LT, TPT, MODE, BLOCK, PF, KIND>(I, task, g, smem, st, false);
  }
}

// ---- batch form with tiled tables: the next child task prepared during the
// current one's gathers
//
// A child task's preparation is latency: the tournament candidates' fitness,
// the parents' rows (global memory) and the mutation draws (Philox chains).
// When the next task of a workgroup's run is a child task of the same
// instance, these move into the current task's lane sum: its SELECT words and
// candidate fitness loads are issued before the first tile's gathers, the
// tournaments are resolved and the children's source rows (one parent row
// each: the crossover cuts between rows) fetched into sChild around the load
// of the last tile, and the mutation codes drawn after the last tile's
// gathers.  The task then starts with its rows in LDS: swaps, write-out and
// inverse rows.  Same draws, same children, same bits.  With K = 32 a row is
// one group of 32 genes, and the row's thread draws its codes itself
// (group_codes), with no code buffer.

// Selection of one child (thread c < nc of the task): the pair's SELECT words
// and the four candidates' fitness, in registers.
struct SelRegs {
  uint32_t u0, v0, u1, v1, w4, w5;
  float f0, f1, f2, f3;
};

__device__ __forceinline__ SelRegs sel_issue(const GenInst &I, const GenTask &task, int gen) {
  SelRegs r{0u, 0u, 0u, 0u, 0u, 0u, 0.0f, 0.0f, 0.0f, 0.0f};
  const int nc = task.s1 - task.s0;
  const int tid = threadIdx.x;
  if (tid < nc) {
    const int slot = task.s0 + tid;
    const int pair_a = I.E + ((slot - I.E) & ~1);
    const Stream st{I.ga.seed_lo, I.ga.seed_hi, (uint32_t)pair_a, (uint32_t)gen,
                    I.ga.instance_id, kTagSelect};
    const Words4 b0 = st.block(0u), b1 = st.block(1u);
    const uint32_t N = (uint32_t)I.N;
    r.u0 = bounded(b0.x, N);
    r.v0 = bounded(b0.y, N);
    r.u1 = bounded(b0.z, N);
    r.v1 = bounded(b0.w, N);
    r.w4 = b1.x;
    r.w5 = b1.y;
    const float *fin = fit_buf(I, gen & 1);
    r.f0 = gp(fin)[r.u0];
    r.f1 = gp(fin)[r.v0];
    r.f2 = gp(fin)[r.u1];
    r.f3 = gp(fin)[r.v1];
  }
  return r;
}

// Tournaments, crossover decision and cut of thread c's child into sSel (as
// build_children_block leaves them).  No barrier.
__device__ __forceinline__ void sel_resolve(const GenInst &I, const GenTask &task,
                                            const SelRegs &r, int32_t *sSel) {
  const int nc = task.s1 - task.s0;
  const int tid = threadIdx.x;
  if (tid < nc) {
    const int slot = task.s0 + tid;
    const bool second = ((slot - I.E) & 1) != 0;
    const uint32_t p1 = beats(rank_key(r.f1), r.v0, rank_key(r.f0), r.u0) ? r.v0 : r.u0;
    const uint32_t p2 = beats(rank_key(r.f3), r.v1, rank_key(r.f2), r.u1) ? r.v1 : r.u1;
    const bool cross = I.L >= 2 && hit(r.w4, I.ga.thr_cross);
    const int cut = cross ? 1 + (int)bounded(r.w5, (uint32_t)(I.L - 1)) : I.L;
    const uint32_t first = second ? p2 : p1, rest = second ? p1 : p2;
    sSel[2 * tid] = (int32_t)(first | (rest << 16));
    sSel[2 * tid + 1] = cut * I.K;
  }
}

// The source rows of a task's children into sChild (row (c, j) from the
// first parent when j < cut, else from the second; K % 4 == 0, K <= 32) by
// global_load_lds: 16 bytes per lane when K % 16 == 0, else 4.  Issues only:
// wait_vmem() and a barrier publish the rows.
__device__ __forceinline__ void dma_rows(const GenInst &I, const GenTask &task, int gen,
                                         const int32_t *sSel, uint8_t *sChild) {
  const int L = I.L, K = I.K, LK = L * K;
  const int total = (task.s1 - task.s0) * LK;
  const uint8_t *pin = pop_buf(I, gen & 1);
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int nw = (int)(blockDim.x >> 6);
  const bool wide = (K & 15) == 0;
  const int span = wide ? 1024 : 256;
  const int chunks = (total + span - 1) / span;
  for (int k = wave; k < chunks; k += nw) {
    const int o = k * span + lane * (wide ? 16 : 4);
    if (o < total) {
      const int q = o / K, w = o - q * K;
      const int c = q / L, j = q - c * L;
      const uint32_t pr = (uint32_t)sSel[2 * c];
      const uint32_t par = j * K < sSel[2 * c + 1] ? (pr & 0xFFFFu) : (pr >> 16);
      const uint8_t *src = pin + (size_t)par * LK + j * K + w;
      uint8_t *dst = sChild + (size_t)__builtin_amdgcn_readfirstlane(k) * span;
      if (wide)
        lds_dma<16>(src, dst);
      else
        lds_dma<4>(src, dst);
    }
  }
}

// The children of a task from their source rows in sChild: each row's swaps
// (codes from sCode, or with K = 32 drawn here), its write-out and its inverse
// entries.  Ends with a barrier.
__device__ __forceinline__ void rows_finish(const GenInst &I, const GenTask &task, int gen,
                                            uint8_t *sChild, const uint8_t *sCode, uint8_t *sInv,
                                            int block) {
  const int L = I.L, K = I.K, LK = L * K, nw = K >> 2;
  const int nc = task.s1 - task.s0, rows = nc * L;
  const bool mutate = K >= 2 && I.ga.thr_mut != 0;
  uint8_t *pout = pop_buf(I, gen < 0 ? 0 : 1 - (gen & 1)) + (size_t)task.s0 * LK;
  for (int q = threadIdx.x; q < rows; q += block) {
    const int c = q / L, j = q - c * L;
    uint8_t *rowb = sChild + q * K;
    if (mutate) {
      if (K == 32) {
        uint32_t code[8];
        // the row's swaps in increasing gene order, over this row's hits only
        // (a loop over all 32 positions runs nearly every one for some lane
        // of the wave)
        uint32_t hits =
            group_codes(j, LK, K, I.ga, (uint32_t)gen, (uint32_t)(task.s0 + c), code);
        while (hits != 0u) {
          const int k = __builtin_ctz(hits);
          hits &= hits - 1u;
          const int kp = (int)code_byte(code, k) - 1;
          const uint8_t t = rowb[k];
          rowb[k] = rowb[kp];
          rowb[kp] = t;
        }
      } else {
        apply_swaps(rowb, sCode + q * K, q * K, K);
      }
    }
    uint8_t *dst = sInv + c * K * L + j;
    if (K == 32) {
      store_row_inverse16(rowb, pout + (size_t)q * K, dst, 2, K, L);
      continue;
    }
    const uint32_t *row = reinterpret_cast<const uint32_t *>(rowb);
    gptr<uint32_t> gw = gp(reinterpret_cast<uint32_t *>(pout + (size_t)q * K));
    for (int w = 0; w < nw; ++w) {
      const uint32_t x = row[w];
      gw[w] = x;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int t = (int)((x >> (8 * b)) & 0xFFu);
        if (t < K) dst[t * L] = (uint8_t)(4 * w + b);
      }
    }
  }
  __syncthreads();
}

// Whether the children of a task can be built by this path (rows whole
// aligned words) and whether it draws the K = 32 codes in the row pass.
__device__ __forceinline__ bool rows_path(const GenInst &I) { return (I.K & 3) == 0 && I.K <= 32; }

// Hook around the last tile load of the current task: resolves the next
// task's tournaments, then fetches its source rows along with the tile.
struct PrepHook {
  const GenInst *I;
  const GenTask *next;
  int gen;
  const SelRegs *sel;
  int32_t *sSel;
  uint8_t *sChild;
  __device__ __forceinline__ void before_load() { sel_resolve(*I, *next, *sel, sSel); }
  __device__ __forceinline__ void issue() { dma_rows(*I, *next, gen, sSel, sChild); }
};

template <int LT, int TPT, int MODE, int BLOCK>
__device__ __forceinline__ void gen_tasks_tiled(const GenInst *insts, const GenTask *tasks,
                                                int t0, int t1, int gen_arg, unsigned char *smem,
                                                const int32_t *gens) {
  using P = GenPlan<LT, TPT, MODE, BLOCK>;
  constexpr int TR = P::kTileRows;
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sChild = smem + P::kChildOff;
  uint8_t *sInv = smem + P::kInvOff;
  float *sE = reinterpret_cast<float *>(smem + P::kEOff);
  float *sOwn = reinterpret_cast<float *>(smem + P::kOwnOff);
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + P::kSelOff);
  uint8_t *sCode = smem + P::kCodeOff;
  LdsState st;
  bool ready = false;  // this task's source rows are in sChild (and its codes in sCode)
  GenTask task = t0 < t1 ? load_task(tasks, t0) : GenTask{0, kTaskElite, 0, 0};
  for (int t = t0; t < t1; ++t) {
    const GenInst I = load_inst(insts, task.inst);
    const int g = gens ? gp(gens)[task.inst] : gen_arg;
    const GenTask next = t + 1 < t1 ? load_task(tasks, t + 1) : GenTask{0, kTaskElite, 0, 0};
    const bool child = task.kind == kTaskChild && g >= 0 && g < I.G && rows_path(I);
    if (!child) {
      run_task<LT, TPT, MODE, BLOCK>(I, task, g, smem, st, false);
      ready = false;
      task = next;
      continue;
    }
    if (task.inst != st.inst) {
      load_own(I.Town, LT, TPT, sOwn);
      st.inst = task.inst;
      st.tile = -1;
    }
    const int nc = task.s1 - task.s0;
    const bool mutate = I.K >= 2 && I.ga.thr_mut != 0;
    if (!ready) {
      // cold start: this task's selection, codes and rows now
      const SelRegs r = sel_issue(I, task, g);
      if (mutate && I.K != 32)
        mutation_codes_block(sCode, nc, I.L * I.K, I.K, I.ga, (uint32_t)g, task.s0, BLOCK);
      sel_resolve(I, task, r, sSel);
      __syncthreads();
      dma_rows(I, task, g, sSel, sChild);
      wait_vmem();
      __syncthreads();
    }
    rows_finish(I, task, g, sChild, sCode, sInv, BLOCK);
    // the next task is prepared inside this one's lane sum when it is a child
    // task of the same instance at the same generation
    const bool pipe = next.kind == kTaskChild && next.inst == task.inst;
    const int q = threadIdx.x;
    const bool active = q / I.K < nc;
    float acc;
    if (pipe) {
      const SelRegs r = sel_issue(I, next, g);
      PrepHook hook{&I, &next, g, &r, sSel, sChild};
      acc = lane_sum_tiled_hook<LT, TPT, MODE, TR>(sInv + q * LT, active, sT, sOwn, I.T2z,
                                                   I.T1, I.lconst, st.tile, I.objective,
                                                   hook);
      if (mutate && I.K != 32)
        mutation_codes_block(sCode, next.s1 - next.s0, I.L * I.K, I.K, I.ga, (uint32_t)g,
                             next.s0, BLOCK);
    } else {
      NoTileHook hook;
      acc = lane_sum_tiled_hook<LT, TPT, MODE, TR>(sInv + q * LT, active, sT, sOwn, I.T2z,
                                                   I.T1, I.lconst, st.tile, I.objective,
                                                   hook);
    }
    float *const fit_out = fit_buf(I, 1 - (g & 1)) + task.s0;
    reduce_round(sE, acc, active, nc, I.K, I.prelog, fit_out, I.objective);
    ready = pipe;
    task = next;
  }
}

template <int LT, int TPT, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_gen_exact(GenArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int t0, t1;
  task_range(a.ntasks, a.bounds, t0, t1);
  if constexpr (GenPlan<LT, TPT, MODE, BLOCK>::kTiles > 1) {
    if (a.gen >= 0 || a.gens) {
      gen_tasks_tiled<LT, TPT, MODE, BLOCK>(a.insts, a.tasks, t0, t1, a.gen, smem, a.gens);
      return;
    }
  }
  LdsState st;
  gen_tasks_exact<LT, TPT, MODE, BLOCK>(a.insts, a.tasks, t0, t1, a.gen, smem, st, a.gens);
}

// ---- persistent form: generations [g0, g1) in one launch, grid barriers ------
//
// Every workgroup keeps the same chunk of tasks in every generation (so the
// table of its instance stays in LDS) and the generations are separated by a
// grid barrier: a monotonic arrival counter (zeroed before the launch) that
// the barrier b waits to reach b * gridDim.x.  Global writes are released at
// agent scope before the arrival and acquired after it.  A wait that exceeds
// kBarrierSpins polls sets *err and every workgroup returns at its next
// barrier, so the grid always drains.
struct PersistArgs {
  const GenInst *insts;
  const GenTask *tasks;
  int ntasks, chunk;
  const GenTask *evals;
  int neval, echunk;
  int g0, g1;  // generations to run; g0 = -1 starts with the initial fitness
  int best;    // nonzero: finish with the best of each instance's last population
  int ninst;
  uint32_t *bar;
  int32_t *err;
};

constexpr uint32_t kBarrierSpins = 1u << 21;

// The grid barrier in two halves, so that a workgroup can do work that
// needs nothing from the others (the next generation's draws) between its
// arrival and its wait.  Arrival: every wave waits until its global writes
// have completed (reached the L2 the workgroup's CU shares), the workgroup
// barrier orders them before thread 0, whose agent-scope release (a write-back
// of that L2, which holds every wave's writes) precedes the arrival.
__device__ __forceinline__ void grid_arrive(uint32_t *bar) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt not waited on
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait until `target` arrivals (bounded, see above); thread 0 acquires at
// agent scope (invalidating the caches of the workgroup's CU) before the
// workgroup barrier, so every wave's later reads see what other workgroups
// wrote before arriving.
__device__ __forceinline__ bool grid_wait(uint32_t *bar, uint32_t target, int32_t *err,
                                          int32_t *sFlag) {
  if (threadIdx.x == 0) {
    int good = 1;
    for (uint32_t spins = 0;; ++spins) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (spins >= kBarrierSpins ||
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *sFlag = good;
  }
  __syncthreads();
  return *sFlag != 0;
}

// Best chromosome of an instance's population after its last generation
// (the whole workgroup; closes the trace).  idx: LDS.
__device__ __forceinline__ void best_block(const GenInst &I, int32_t *idx) {
  const float *fit = fit_buf(I, I.G & 1);
  if (threadIdx.x < kWave) top_e_wave(fit, I.N, 1, idx, threadIdx.x);
  __syncthreads();
  const int b = idx[0];
  if (threadIdx.x == 0) {
    *gp(I.best_idx) = b;
    *gp(I.best_fit) = gp(fit)[b];
    gp(I.trace)[I.G] = gp(fit)[b];
  }
  const int LK = I.L * I.K;
  const uint8_t *src = pop_buf(I, I.G & 1) + (size_t)b * LK;
  for (int i = threadIdx.x; i < LK; i += blockDim.x) gp(I.best_out)[i] = gp(src)[i];
  __syncthreads();
}

// Prefetching child tasks when the plan with their regions keeps the whole
// table in LDS.
template <int LT, int TPT, int MODE, int BLOCK>
constexpr bool persist_prefetch() {
  return GenPlan<LT, TPT, MODE, BLOCK, true>::kTiles == 1;
}
template <int LT, int TPT, int MODE, int BLOCK>
using PersistPlan = GenPlan<LT, TPT, MODE, BLOCK, persist_prefetch<LT, TPT, MODE, BLOCK>()>;

template <int LT, int TPT, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_gen_persist(PersistArgs a) {
  constexpr bool PF = persist_prefetch<LT, TPT, MODE, BLOCK>();
  using P = PersistPlan<LT, TPT, MODE, BLOCK>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int32_t *sIdx = reinterpret_cast<int32_t *>(smem + P::kIdxOff);
  LdsState st;
  uint32_t nbar = 0;
  // with one task per workgroup (the persistent plans), the workgroup's
  // generation task and its descriptor are read once, into registers
  const bool fixed = a.chunk == 1 && (int)blockIdx.x < a.ntasks;
  GenTask mt{0, kTaskElite, 0, 0};
  if (fixed) mt = load_task(a.tasks, blockIdx.x);
  const GenInst mI = load_inst(a.insts, mt.inst);
  bool prepared = false;  // the child task of `gen` is prepared
  for (int gen = a.g0; gen < a.g1; ++gen) {
    if (gen < 0) {
      const int t0 = blockIdx.x * a.echunk, t1 = min(a.neval, t0 + a.echunk);
      gen_tasks_exact<LT, TPT, MODE, BLOCK, PF, kTaskEval>(a.insts, a.evals, t0, t1, gen, smem,
                                                           st);
    } else {
      // one inlined copy of the task code for both forms keeps the kernel's
      // per-generation code compact
      const int t0 = fixed ? 0 : blockIdx.x * a.chunk;
      const int t1 = fixed ? 1 : min(a.ntasks, t0 + a.chunk);
      for (int t = t0; t < t1; ++t) {
        const GenTask task = fixed ? mt : load_task(a.tasks, t);
        const GenInst I = fixed ? mI : load_inst(a.insts, task.inst);
        run_task<LT, TPT, MODE, BLOCK, PF>(I, task, gen, smem, st, prepared);
      }
    }
    prepared = false;
    grid_arrive(a.bar);
    if constexpr (PF) {
      // prepare the next generation's child task (LDS only, nothing from the
      // other workgroups) while they finish this one
      if (fixed && gen + 1 < a.g1 && mt.kind == kTaskChild && gen + 1 < mI.G) {
        pf_precompute(mI, mt, gen + 1, smem + P::kCodeOff,
                      reinterpret_cast<int32_t *>(smem + P::kPairOff), BLOCK);
        prepared = true;
      }
    }
    // sIdx[63] is free here: elite tasks use sIdx[0 .. E) with E < 64
    if (!grid_wait(a.bar, ++nbar * gridDim.x, a.err, sIdx + 63)) return;
  }
  if (a.best)
    for (int i = blockIdx.x; i < a.ninst; i += gridDim.x) best_block(a.insts[i], sIdx);
}

// Runtime-L variant: L <= LMAX, any TP; the LDS plan comes from the host.
struct GenGenericPlan {
  int tile_rows, child_off, inv_off, e_off, idx_off, sel_off;
};

template <int LMAX, int MODE>
__global__ __launch_bounds__(1024) void k_gen_generic(GenArgs a, GenGenericPlan pl) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sChild = smem + pl.child_off;
  uint8_t *sInv = smem + pl.inv_off;
  float *sE = reinterpret_cast<float *>(smem + pl.e_off);
  int32_t *sIdx = reinterpret_cast<int32_t *>(smem + pl.idx_off);
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + pl.sel_off);
  int t0, t1;
  task_range(a.ntasks, a.bounds, t0, t1);
  int loaded = -1;
  for (int t = t0; t < t1; ++t) {
    const GenTask task = load_task(a.tasks, t);
    const GenInst I = load_inst(a.insts, task.inst);
    const int gen = a.gens ? gp(a.gens)[task.inst] : a.gen;
    if (gen >= I.G) continue;
    const int L = I.L, TP = I.TP, TR = pl.tile_rows;
    if (TR >= L && task.kind != kTaskElite && task.inst != loaded) {
      __syncthreads();
      load_tile<MODE>(I.T2, I.T1, L, TP, 0, L, TR, sT);
      loaded = task.inst;
    }
    const int nc = gen_prepare(I, task, gen, sChild, sInv, sInv, sIdx, sSel, (int)blockDim.x);
    if (nc == 0) continue;
    const int K = I.K;
    const int q = threadIdx.x;
    const bool active = q / K < nc;
    const float acc =
        lane_sum_generic<LMAX, MODE>(sInv + q * L, active, L, TP, TR, sT, I.T2, I.T1, I.lconst,
                                     I.objective);
    const int out = gen < 0 ? 0 : 1 - (gen & 1);
    reduce_round(sE, acc, active, nc, K, I.prelog, fit_buf(I, out) + task.s0, I.objective);
  }
}

}  // namespace pa

// ---------------------------------------------------------------- host side
namespace pa {

inline GenArgs gen_args(const GenInst *insts, const GenClass &c, int gen) {
  GenArgs a;
  a.insts = insts;
  a.gen = gen;
  a.gens = c.gens;
  a.tasks = (gen < 0 && !c.gens) ? c.eval_tasks : c.tasks;
  a.ntasks = (gen < 0 && !c.gens) ? c.neval : c.ntasks;
  a.bounds = (gen < 0 && !c.gens) ? nullptr : c.bounds;
  return a;
}

// Workgroups of `kern` (block threads, lds bytes of dynamic LDS) one CU holds.
inline hipError_t per_cu_query(const void *kern, int block, int lds, int *out) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, block, lds);
  *out = e == hipSuccess ? nb : 0;
  return e;
}

template <int LT, int TPT, int MODE, int BLOCK>
hipError_t gen_launch_exact(const GenInst *insts, const GenClass &c, int gen, hipStream_t s) {
  using P = GenPlan<LT, TPT, MODE, BLOCK>;
  auto kern = k_gen_exact<LT, TPT, MODE, BLOCK>;
  static LdsAttr attr;
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(kern), P::kTotal);
  if (c.query_per_cu) return per_cu_query(reinterpret_cast<const void *>(kern), BLOCK, P::kTotal,
                                          c.query_per_cu);
  const int n = gen < 0 ? c.neval : c.ntasks;
  if (n <= 0) return hipSuccess;
  const int grid = c.grid < 1 ? 1 : (c.grid > n ? n : c.grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), P::kTotal, s, gen_args(insts, c, gen));
  return launch_status(ae);
}

// A persistent launch of a class (PersistArgs with the grid), or, when
// `capacity` is set, only the query of the largest co-resident grid of the
// class's persistent kernel.
struct PersistCall {
  PersistArgs args;
  int grid;
  int cus;
  int *capacity;
};

// The persistent kernel is an ordinary launch whose grid is at most the
// number of its workgroups the device holds at once (the occupancy query
// below; plans never ask for more).  On a device that runs nothing else all
// of them are then resident together; if other streams keep CUs busy, the
// late workgroups start as those kernels end, and a grid-barrier wait that
// exceeds its bound makes the solve report PA_EINTERNAL instead of hanging.
// (The cooperative-launch API is not used: the runtime serves it from an
// internal device queue that lives until the process tears the runtime
// down.)
template <int LT, int TPT, int MODE, int BLOCK>
hipError_t gen_persist_exact(const PersistCall &pc, hipStream_t s) {
  using P = PersistPlan<LT, TPT, MODE, BLOCK>;
  auto kern = k_gen_persist<LT, TPT, MODE, BLOCK>;
  static LdsAttr attr;
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(kern), P::kTotal);
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, reinterpret_cast<const void *>(kern), BLOCK, P::kTotal);
  if (e != hipSuccess) return e;
  if (pc.capacity) {
    *pc.capacity = nb * pc.cus;
    return hipSuccess;
  }
  if (pc.grid < 1 || pc.grid > nb * pc.cus) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(kern, dim3(pc.grid), dim3(BLOCK), P::kTotal, s, pc.args);
  return launch_status(ae);
}

template <int LT, int TPT, int MODE, bool PERSIST>
hipError_t gen_dispatch_block(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                              bool *handled, const PersistCall *pc) {
  *handled = true;
  switch (c.block) {
    case 256:
      if constexpr (PERSIST) return gen_persist_exact<LT, TPT, MODE, 256>(*pc, s);
      else return gen_launch_exact<LT, TPT, MODE, 256>(insts, c, gen, s);
    case 512:
      if constexpr (PERSIST) return gen_persist_exact<LT, TPT, MODE, 512>(*pc, s);
      else return gen_launch_exact<LT, TPT, MODE, 512>(insts, c, gen, s);
    default: *handled = false; return hipSuccess;
  }
}

// Launches the unrolled generation kernel of cell count LT and SE mode MODE
// (its persistent form when PERSIST, with pc set); *handled = false when no
// unrolled variant serves (L, mode, TP, block).
template <int LT, int MODE, bool PERSIST>
hipError_t gen_dispatch_unrolled(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                                 bool *handled, const PersistCall *pc) {
  *handled = false;
  if (c.L != LT || c.mode != MODE || (pc != nullptr) != PERSIST) return hipSuccess;
  switch (c.TP) {
    case 4: return gen_dispatch_block<LT, 4, MODE, PERSIST>(insts, c, gen, s, handled, pc);
    case 8: return gen_dispatch_block<LT, 8, MODE, PERSIST>(insts, c, gen, s, handled, pc);
    case 16: return gen_dispatch_block<LT, 16, MODE, PERSIST>(insts, c, gen, s, handled, pc);
    case 32: return gen_dispatch_block<LT, 32, MODE, PERSIST>(insts, c, gen, s, handled, pc);
    default: return hipSuccess;
  }
}

// One dispatch function per (L, SE mode, form), each defined by its own
// compile unit of k_gen_unrolled.hip (x: per-generation, p: persistent).
using GenDispatchFn = hipError_t (*)(const GenInst *, const GenClass &, int, hipStream_t, bool *,
                                     const PersistCall *);
#define PA_GEN_DECL(LV, MV, FV)                                                                \
  hipError_t gen_dispatch_L##LV##_m##MV##_##FV(const GenInst *, const GenClass &, int,         \
                                               hipStream_t, bool *, const PersistCall *);
PA_GEN_DECL(7, 0, x) PA_GEN_DECL(7, 0, p) PA_GEN_DECL(7, 1, x) PA_GEN_DECL(7, 1, p)
PA_GEN_DECL(19, 0, x) PA_GEN_DECL(19, 0, p) PA_GEN_DECL(19, 1, x) PA_GEN_DECL(19, 1, p)
PA_GEN_DECL(37, 0, x) PA_GEN_DECL(37, 0, p) PA_GEN_DECL(37, 1, x) PA_GEN_DECL(37, 1, p)
#undef PA_GEN_DECL
hipError_t gen_dispatch_generic(const GenInst *, const GenClass &, int, hipStream_t);

}  // namespace pa
