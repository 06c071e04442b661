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
  int ntasks;
  int chunk;  // tasks per workgroup
  int gen;    // -1: fitness of the initial populations
};

// LDS plan: table tile | children (<= block*L) | inverse rows, aliased by the
// mutation flags while children are built (<= block*L) | sums (block*4) |
// elite indices (64 ints).
template <int LT, int TPT, int MODE, int BLOCK>
struct GenPlan {
  static constexpr int kChildBytes = ((BLOCK * LT) + 15) / 16 * 16;
  static constexpr int kInvBytes = kChildBytes;
  static constexpr int kEBytes = BLOCK * 4;
  static constexpr int kIdxBytes = 256;
  static constexpr int kOwnBytes = LT * TPT * 4;  // own-cell squares (tiled tables)
  static constexpr int kSelBytes = BLOCK * 8;     // parents and cut per child
  using T = TilePlan<LT, TPT, MODE,
                     kChildBytes + kInvBytes + kEBytes + kIdxBytes + kOwnBytes + kSelBytes>;
  static constexpr int kTiles = T::kTiles;
  static constexpr int kTileRows = T::kTileRows;
  static constexpr int kChildOff = T::kTableBytes;
  static constexpr int kInvOff = kChildOff + kChildBytes;
  static constexpr int kEOff = kInvOff + kInvBytes;
  static constexpr int kIdxOff = kEOff + kEBytes;
  static constexpr int kOwnOff = kIdxOff + kIdxBytes;
  static constexpr int kSelOff = kOwnOff + kOwnBytes;
  static constexpr int kTotal = kSelOff + kSelBytes;
  static_assert(kTotal <= kLdsBytes, "LDS plan too large");
};

// Everything of a task but the fitness evaluation; returns the number of
// chromosomes to evaluate (0 for an elite task or a finished instance).
// Leaves their inverse rows in sInv and ends with a barrier.
__device__ __forceinline__ int gen_prepare(const GenInst &I, const GenTask &task, int gen,
                                           uint8_t *sChild, uint8_t *sInv, int32_t *sIdx,
                                           int32_t *sSel, int block) {
  const int L = I.L, K = I.K, LK = L * K;
  const int in = gen < 0 ? 0 : (gen & 1);
  const int out = gen < 0 ? 0 : 1 - in;
  if (task.kind == kTaskElite) {
    copy_elites_block(I.pop[in], I.fit[in], I.N, I.E, LK, I.pop[out], I.fit[out], I.trace, gen,
                      sIdx);
    return 0;
  }
  const int nc = task.s1 - task.s0;
  if (task.kind == kTaskChild) {
    build_children_block(I.pop[in], I.fit[in], I.N, I.E, L, K, I.ga, (uint32_t)gen, task.s0, nc,
                         sChild, sInv, sSel, block);
    uint8_t *dst = I.pop[out] + (size_t)task.s0 * LK;
    for (int i = threadIdx.x; i < nc * LK; i += block) dst[i] = sChild[i];
    build_inverse(sChild, nc * L, L, K, sInv);
  } else {
    copy_bytes(I.pop[in] + (size_t)task.s0 * LK, nc * LK, sChild);
    __syncthreads();
    build_inverse(sChild, nc * L, L, K, sInv);
  }
  __syncthreads();
  return nc;
}

template <int LT, int TPT, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_gen_exact(GenArgs a) {
  using P = GenPlan<LT, TPT, MODE, BLOCK>;
  constexpr int NT = P::kTiles;
  constexpr int TR = P::kTileRows;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sChild = smem + P::kChildOff;
  uint8_t *sInv = smem + P::kInvOff;
  float *sE = reinterpret_cast<float *>(smem + P::kEOff);
  int32_t *sIdx = reinterpret_cast<int32_t *>(smem + P::kIdxOff);
  float *sOwn = reinterpret_cast<float *>(smem + P::kOwnOff);
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + P::kSelOff);
  const int t0 = blockIdx.x * a.chunk;
  const int t1 = min(a.ntasks, t0 + a.chunk);
  int loaded = -1;
  for (int t = t0; t < t1; ++t) {
    const GenTask task = a.tasks[t];
    const GenInst &I = a.insts[task.inst];
    if (a.gen >= I.G) continue;  // this instance has finished its generations
    if (task.kind != kTaskElite && task.inst != loaded) {
      // every thread passed a barrier since the tables were last read
      if constexpr (NT == 1)
        load_tile<MODE>(I.T2, I.T1, LT, TPT, 0, LT, TR, sT);
      else
        load_own(I.Town, LT, TPT, sOwn);
      loaded = task.inst;
    }
    const int nc = gen_prepare(I, task, a.gen, sChild, sInv, sIdx, sSel, BLOCK);
    if (nc == 0) continue;
    const int K = I.K;
    const int q = threadIdx.x;
    const bool active = q / K < nc;
    float acc;
    if constexpr (NT == 1)
      acc = lane_sum_exact<LT, TPT, MODE, TR, 1>(sInv + q * LT, active, sT, I.T2, I.T1, I.lconst);
    else
      acc = lane_sum_tiled<LT, TPT, MODE, TR>(sInv + q * LT, active, sT, sOwn, I.T2z, I.T1,
                                              I.lconst);
    const int out = a.gen < 0 ? 0 : 1 - (a.gen & 1);
    reduce_round(sE, acc, active, nc, K, I.prelog, I.fit[out] + task.s0);
  }
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
  const int t0 = blockIdx.x * a.chunk;
  const int t1 = min(a.ntasks, t0 + a.chunk);
  int loaded = -1;
  for (int t = t0; t < t1; ++t) {
    const GenTask task = a.tasks[t];
    const GenInst &I = a.insts[task.inst];
    if (a.gen >= I.G) continue;
    const int L = I.L, TP = I.TP, TR = pl.tile_rows;
    if (TR >= L && task.kind != kTaskElite && task.inst != loaded) {
      __syncthreads();
      load_tile<MODE>(I.T2, I.T1, L, TP, 0, L, TR, sT);
      loaded = task.inst;
    }
    const int nc = gen_prepare(I, task, a.gen, sChild, sInv, sIdx, sSel, (int)blockDim.x);
    if (nc == 0) continue;
    const int K = I.K;
    const int q = threadIdx.x;
    const bool active = q / K < nc;
    const float acc =
        lane_sum_generic<LMAX, MODE>(sInv + q * L, active, L, TP, TR, sT, I.T2, I.T1, I.lconst);
    const int out = a.gen < 0 ? 0 : 1 - (a.gen & 1);
    reduce_round(sE, acc, active, nc, K, I.prelog, I.fit[out] + task.s0);
  }
}

}  // namespace pa

// ---------------------------------------------------------------- host side
namespace pa {

inline void gen_allow_lds(const void *kern, int bytes) {
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    (void)hipGetLastError();
}

inline GenArgs gen_args(const GenInst *insts, const GenClass &c, int gen, int grid) {
  GenArgs a;
  a.insts = insts;
  a.gen = gen;
  a.tasks = gen < 0 ? c.eval_tasks : c.tasks;
  a.ntasks = gen < 0 ? c.neval : c.ntasks;
  a.chunk = (a.ntasks + grid - 1) / grid;
  return a;
}

template <int LT, int TPT, int MODE, int BLOCK>
hipError_t gen_launch_exact(const GenInst *insts, const GenClass &c, int gen, hipStream_t s) {
  using P = GenPlan<LT, TPT, MODE, BLOCK>;
  auto kern = k_gen_exact<LT, TPT, MODE, BLOCK>;
  static bool attr = false;
  if (!attr) {
    gen_allow_lds(reinterpret_cast<const void *>(kern), P::kTotal);
    attr = true;
  }
  const int n = gen < 0 ? c.neval : c.ntasks;
  if (n <= 0) return hipSuccess;
  const int grid = c.grid < 1 ? 1 : (c.grid > n ? n : c.grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), P::kTotal, s, gen_args(insts, c, gen, grid));
  return hipGetLastError();
}

template <int LT, int TPT, int MODE>
hipError_t gen_dispatch_block(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                              bool *handled) {
  *handled = true;
  switch (c.block) {
    case 64: return gen_launch_exact<LT, TPT, MODE, 64>(insts, c, gen, s);
    case 256: return gen_launch_exact<LT, TPT, MODE, 256>(insts, c, gen, s);
    case 512: return gen_launch_exact<LT, TPT, MODE, 512>(insts, c, gen, s);
    default: *handled = false; return hipSuccess;
  }
}

// Launches the unrolled generation kernel of cell count LT; *handled = false
// when no unrolled variant serves (TP, mode, block).
template <int LT>
hipError_t gen_dispatch_L(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                          bool *handled) {
  *handled = false;
  if (c.L != LT) return hipSuccess;
  if (c.mode == 0) {
    switch (c.TP) {
      case 4: return gen_dispatch_block<LT, 4, 0>(insts, c, gen, s, handled);
      case 8: return gen_dispatch_block<LT, 8, 0>(insts, c, gen, s, handled);
      case 16: return gen_dispatch_block<LT, 16, 0>(insts, c, gen, s, handled);
      case 32: return gen_dispatch_block<LT, 32, 0>(insts, c, gen, s, handled);
      default: return hipSuccess;
    }
  }
  switch (c.TP) {
    case 4: return gen_dispatch_block<LT, 4, 1>(insts, c, gen, s, handled);
    case 8: return gen_dispatch_block<LT, 8, 1>(insts, c, gen, s, handled);
    case 16: return gen_dispatch_block<LT, 16, 1>(insts, c, gen, s, handled);
    case 32: return gen_dispatch_block<LT, 32, 1>(insts, c, gen, s, handled);
    default: return hipSuccess;
  }
}

hipError_t gen_dispatch_L7(const GenInst *, const GenClass &, int, hipStream_t, bool *);
hipError_t gen_dispatch_L19(const GenInst *, const GenClass &, int, hipStream_t, bool *);
hipError_t gen_dispatch_L37(const GenInst *, const GenClass &, int, hipStream_t, bool *);
hipError_t gen_dispatch_generic(const GenInst *, const GenClass &, int, hipStream_t);

}  // namespace pa
