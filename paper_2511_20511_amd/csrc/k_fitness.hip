// k_fitness.hip -- population fitness (uplink sum SE, Sec. 3.2 Eq. 5-6).
//
// A workgroup stages the FP32 table of the problem in LDS (in tiles of BS
// rows when it does not fit) and walks over "rounds" of CPR = block/K
// chromosomes: it inverts their rows into LDS, each lane (c, p) loads its L
// row offsets into registers, accumulates the per-pilot SE over all BS rows,
// and one lane per chromosome reduces over pilots.  See fitness_core.h for
// the canonical arithmetic order.
//
// Variants: for L in {7, 19, 37} (the 1-, 2- and 3-ring hexagonal layouts)
// the BS and cell loops are fully unrolled so every gather is a single
// ds_read_b32 with an immediate offset and the own-cell term is peeled at
// compile time; other L use a runtime loop bounded by LMAX.
#include "fitness_core.h"
#include "pa_internal.h"

namespace pa {

struct FitArgs {
  const float *T2;
  const float *T1;
  const float *T2z;
  const float *Town;
  const float *lconst;
  const uint8_t *pop;
  float *fit;
  int n, L, K, TP;
  float prelog;
  int objective;  // 0: sum of the SE terms, 1: their minimum, 2: minus the Eq. 8 ratios
  int tile_rows;  // generic variant: BS rows per LDS tile
  int inv_off;    // LDS byte offset of the inverse rows
  int e_off;      // LDS byte offset of the per-(c, p) sums
  int stage_off;  // LDS byte offset of the round's chromosome bytes
};

// LDS plan of the population-fitness kernels: the table tile, then the
// inverse rows (<= block*L bytes), then the per-(c, p) sums (block*4 bytes),
// the own-cell squares, the round's chromosome bytes and, for tiled tables,
// the partial sums of a group of kGroup rounds (kGroup*block floats).  An
// asymptotic-SE table that fits whole in its quad layout (fitness_core.h) is
// staged that way (kQuad).
template <int LT, int TPT, int MODE, int BLOCK>
struct ExactPlan {
  // inverse rows at a stride of whole words (inv_stride)
  static constexpr int kInvBytes = ((BLOCK * inv_stride<LT>()) + 15) / 16 * 16;
  static constexpr int kEBytes = BLOCK * 4;
  static constexpr int kOwnBytes = LT * TPT * 4;  // own-cell squares (tiled tables)
  // the round's chromosome bytes, stored as whole words from 4 bytes past
  // each wave's part (wave w's part at w * 64 * LT + 4 (w + 1))
  static constexpr int kStageBytes = ((BLOCK * LT + 4 * (BLOCK / 64 + 1) + 4) + 15) / 16 * 16;
  static constexpr int kBase = kInvBytes + kEBytes + kOwnBytes + kStageBytes;
  static constexpr int kGroup = 8;
  static constexpr int kAccBytes = TilePlan<LT, TPT, MODE, kBase>::kTiles > 1 ? kGroup * BLOCK * 4 : 0;
  using T = TilePlan<LT, TPT, MODE, kBase + kAccBytes>;
  static constexpr int kTiles = T::kTiles;
  static constexpr int kTileRows = T::kTileRows;
  static constexpr int kQuadBytes = LT * TPT * quad_rows<LT>() * 4;
  static constexpr bool kQuad = MODE == 0 && kTiles == 1 && kQuadBytes + kBase + 256 <= kLdsBytes;
  static constexpr int kInvOff = kQuad ? kQuadBytes : T::kTableBytes;
  static constexpr int kEOff = kInvOff + kInvBytes;
  static constexpr int kOwnOff = kEOff + kEBytes;
  static constexpr int kStageOff = kOwnOff + kOwnBytes;
  static constexpr int kAccOff = kStageOff + kStageBytes;
  static constexpr int kTotal = kAccOff + kAccBytes;
  static_assert(kTotal <= kLdsBytes, "LDS plan too large");
};

// Words of a round's chromosome bytes one thread prefetches (a round is at
// most block * L bytes, i.e. at most L / 4 + 1 words per thread).
template <int LT>
constexpr int stage_words() {
  return LT / 4 + 2;
}

template <int LT, int TPT, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fitness_exact(FitArgs a) {
  constexpr int kStagePF = stage_words<LT>();
  using P = ExactPlan<LT, TPT, MODE, BLOCK>;
  constexpr int NT = P::kTiles;
  constexpr int TR = P::kTileRows;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sInv = smem + P::kInvOff;
  float *sE = reinterpret_cast<float *>(smem + P::kEOff);
  float *sOwn = reinterpret_cast<float *>(smem + P::kOwnOff);
  uint8_t *sStage = smem + P::kStageOff;
  const int K = a.K;
  const int LK = LT * K;
  const int CPR = BLOCK / K;
  const int q = threadIdx.x;
  constexpr int ST = inv_stride<LT>();  // inverse row stride (whole words)
  const int rounds = (a.n + CPR - 1) / CPR;
  const int mn = a.objective;
  // a chromosome's lanes in one wave: inverse rows by lane permutes; with a
  // tiled table (K a power of two up to 32, so a pilot reduction in
  // registers) every round is also staged, inverted, summed and reduced by
  // each wave on its own chromosomes, with no barrier between rounds (not for
  // finite-M tables of at most 16 pilots: that kernel's registers would spill
  // more and it runs slower)
  const bool perm = (64 % K) == 0 && K <= 32;
  const bool wave_private = perm && NT > 1 && (MODE == 0 || TPT >= 32);
  const int lane = q & (kWave - 1);
  // the wave's chromosomes of a round: 64 / K of them, from the wave's
  // first; their bytes are contiguous in the round's and staged at the same
  // place (wstage = the wave's first chromosome x LK)
  const int wave = __builtin_amdgcn_readfirstlane(q / kWave);  // wave-uniform
  const int cw0 = wave * (kWave / K);
  const int wstage = cw0 * LK;
  // the wave's staged words start 4 (wave + 1) bytes past its part (room
  // for the bytes before and after its range in its first and last words)
  uint8_t *const wdst = sStage + wstage + 4 * (wave + 1);
  auto wave_range = [&](const ByteRange &rr) {
    const int nb = min(max(rr.n - wstage, 0), (kWave / K) * LK);
    return ByteRange{rr.src + wstage, nb};
  };

  if constexpr (NT > 1) {
    // Tiled table: tiles outermost.  The workgroup's rounds are taken in
    // groups of kGroup; each tile is loaded once per group and every round of
    // the group is restaged, inverted and summed over the tile's rows, the
    // partial sums kept in LDS between tiles (the same per-lane order of
    // additions as lane_sum_tiled, so the same bits).
    float *sAcc = reinterpret_cast<float *>(smem + P::kAccOff);
    load_own(a.Town, LT, TPT, sOwn);  // ordered by the first barrier below
    const int mine = rounds > (int)blockIdx.x ? (rounds - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    for (int i0 = 0; i0 < mine; i0 += P::kGroup) {
      const int ng = min(P::kGroup, mine - i0);
      for (int t = 0; t < NT; ++t) {
        __syncthreads();  // every lane is done with the previous tile
        const int rows = (t + 1) * TR <= LT ? TR : LT - t * TR;
        load_tile<MODE>(a.T2z, a.T1, LT, TPT, t * TR, rows, TR, sT);
        // the next round's chromosome bytes are loaded during this round
        uint32_t pf[kStagePF];
        auto range = [&](int g) {
          const int c0 = ((int)blockIdx.x + (i0 + g) * (int)gridDim.x) * CPR;
          return ByteRange{a.pop + (size_t)c0 * LK, min(CPR, a.n - c0) * LK};
        };
        if (wave_private) {
          prefetch_issue(wave_range(range(0)), pf, lane, kWave);
          __syncthreads();  // the tile
        } else {
          prefetch_issue(range(0), pf);
        }
        for (int g = 0; g < ng; ++g) {
          const int r = (int)blockIdx.x + (i0 + g) * (int)gridDim.x;
          const int c0 = r * CPR;
          const int nc = min(CPR, a.n - c0);
          if (wave_private) {
            // the two waves of a SIMD (w, w + 4) take turns at the higher
            // issue priority, round by round, so that neither falls behind
            // before the next tile's barrier
            if (((g + (wave >> 2)) & 1) != 0)
              __builtin_amdgcn_s_setprio(1);
            else
              __builtin_amdgcn_s_setprio(0);
            // each wave stages and inverts its own chromosomes: no barrier
            // until the next tile (wave_sync keeps the previous round's
            // permute reads of the wave's stage before these writes)
            wave_sync();
            const ByteRange wr = wave_range(range(g));
            prefetch_store(wr, pf, wdst, lane, kWave);
            if (g + 1 < ng) prefetch_issue(wave_range(range(g + 1)), pf, lane, kWave);
            wave_sync();
            // (chromosome c of the round at base + c * LK)
            inverse_rows_permute<LT, ST>(sStage + 4 * (wave + 1) + wr.lead(), K, sInv);
          } else {
            // (with the permute form, a round of a tile before the last ends
            // without a barrier: every lane's reads of sStage come before
            // this round's staging)
            if (perm && g > 0 && t + 1 < NT) __syncthreads();
            const ByteRange rr = range(g);
            prefetch_store(rr, pf, sStage + 4);
            if (g + 1 < ng) prefetch_issue(range(g + 1), pf);
            __syncthreads();
            if (perm) {
              inverse_rows_permute<LT, ST>(sStage + 4 + rr.lead(), K, sInv);
            } else {
              build_inverse(sStage + 4 + rr.lead(), nc * LT, LT, K, sInv, ST);
              __syncthreads();
            }
          }
          const bool active = q / K < nc;
          const uint8_t *ip = sInv + q * ST;
          uint32_t A[LT];
          tiled_offsets<LT, TPT, MODE, TR, ST>(ip, active, A);
          float acc = t == 0 ? obj_init(mn) : sAcc[g * BLOCK + q];
          acc = tiled_rows<LT, TPT, MODE, TR>(A, ip, active, sT, sOwn, a.lconst, t, acc, mn);
          if (t + 1 < NT) {
            // (the barrier after the next round's staging orders this
            // round's sInv reads before that round's inverse rows)
            sAcc[g * BLOCK + q] = acc;
          } else {
            // (ends with a barrier, except in the wave-private form)
            reduce_round(sE, acc, active, nc, K, a.prelog, a.fit + c0, mn, !wave_private);
          }
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    return;
  } else if constexpr (P::kQuad) {
    load_quad(a.T2, LT, TPT, 0, LT, quad_rows<LT>(), sT);
    __syncthreads();
  } else {
    load_tile<MODE>(a.T2, a.T1, LT, TPT, 0, LT, TR, sT);
    __syncthreads();
  }
  // the next round's chromosome bytes are loaded during this round
  uint32_t pf[kStagePF];
  auto range = [&](int r) {
    const int c0 = r * CPR;
    return ByteRange{a.pop + (size_t)c0 * LK, r < rounds ? min(CPR, a.n - c0) * LK : 0};
  };
  prefetch_issue(range(blockIdx.x), pf);
  for (int r = blockIdx.x; r < rounds; r += gridDim.x) {
    const int c0 = r * CPR;
    const int nc = min(CPR, a.n - c0);
    const ByteRange rr = range(r);
    prefetch_store(rr, pf, sStage + 4);
    prefetch_issue(range(r + gridDim.x), pf);
    __syncthreads();
    // (reduce_round's closing barrier keeps the next round's staging after
    // every lane's reads of sStage)
    if (perm) {
      inverse_rows_permute<LT, ST>(sStage + 4 + rr.lead(), K, sInv);
    } else {
      build_inverse(sStage + 4 + rr.lead(), nc * LT, LT, K, sInv, ST);
      __syncthreads();
    }
    const bool active = q / K < nc;
    float acc;
    if constexpr (P::kQuad)
      acc = lane_sum_quad<LT, TPT, ST>(sInv + q * ST, active, sT, mn);
    else
      acc = lane_sum_exact<LT, TPT, MODE, TR, 1, ST>(sInv + q * ST, active, sT, a.T2, a.T1,
                                                     a.lconst, mn);
    reduce_round(sE, acc, active, nc, K, a.prelog, a.fit + c0, mn);
  }
}

template <int LMAX, int MODE>
__global__ __launch_bounds__(1024) void k_fitness_generic(FitArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int L = a.L, K = a.K, TP = a.TP;
  const int TR = a.tile_rows;
  const int NT = (L + TR - 1) / TR;
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sInv = smem + a.inv_off;
  float *sE = reinterpret_cast<float *>(smem + a.e_off);
  uint8_t *sStage = smem + a.stage_off;
  const int LK = L * K;
  const int CPR = (int)blockDim.x / K;
  const int q = threadIdx.x;
  const int rounds = (a.n + CPR - 1) / CPR;

  if (NT == 1) {
    load_tile<MODE>(a.T2, a.T1, L, TP, 0, L, TR, sT);
    __syncthreads();
  }
  for (int r = blockIdx.x; r < rounds; r += gridDim.x) {
    const int c0 = r * CPR;
    const int nc = min(CPR, a.n - c0);
    copy_bytes(a.pop + (size_t)c0 * LK, nc * LK, sStage);
    __syncthreads();
    build_inverse(sStage, nc * L, L, K, sInv);
    __syncthreads();
    const bool active = q / K < nc;
    const int mn = a.objective;
    const float acc = lane_sum_generic<LMAX, MODE>(sInv + q * L, active, L, TP, TR, sT, a.T2,
                                                   a.T1, a.lconst, mn);
    reduce_round(sE, acc, active, nc, K, a.prelog, a.fit + c0, mn);
  }
}

// ---------------------------------------------------------------- dispatch

namespace {

template <int LT, int TPT, int MODE>
constexpr int exact_block() {
  // Small tables: 256 threads so several workgroups share a CU; large ones:
  // 512 threads (8 waves, up to 256 VGPRs each: the unrolled L = 37 row loop
  // spills under the 128-register cap of 1024-thread groups).
  return (LT * LT * TPT * 4 * (MODE == 1 ? 2 : 1) <= 40 * 1024) ? 256 : 512;
}

template <int LT, int TPT, int MODE>
hipError_t run_exact(const FitArgs &a0, const DeviceInfo &dev, int grid_cap, hipStream_t s) {
  constexpr int B = exact_block<LT, TPT, MODE>();
  using P = ExactPlan<LT, TPT, MODE, B>;
  FitArgs a = a0;
  a.inv_off = P::kInvOff;
  a.e_off = P::kEOff;
  a.tile_rows = P::kTileRows;
  const int cpr = B / a.K;
  const int rounds = (a.n + cpr - 1) / cpr;
  const int per_cu = P::kTotal > 0 ? (int)(kLdsBytes / P::kTotal) : 1;
  int grid = dev.cus * (per_cu < 1 ? 1 : per_cu);
  if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
  if (grid > rounds) grid = rounds;
  auto kern = k_fitness_exact<LT, TPT, MODE, B>;
  static LdsAttr attr;
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(kern), P::kTotal);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(B), P::kTotal, s, a);
  return launch_status(ae);
}

template <int LT, int MODE>
hipError_t run_exact_tp(const FitArgs &a, const DeviceInfo &dev, int grid_cap, hipStream_t s,
                        bool *handled) {
  *handled = true;
  switch (a.TP) {
    case 4: return run_exact<LT, 4, MODE>(a, dev, grid_cap, s);
    case 8: return run_exact<LT, 8, MODE>(a, dev, grid_cap, s);
    case 16: return run_exact<LT, 16, MODE>(a, dev, grid_cap, s);
    case 32: return run_exact<LT, 32, MODE>(a, dev, grid_cap, s);
    default: *handled = false; return hipSuccess;
  }
}

template <int MODE>
hipError_t run_exact_any(const FitArgs &a, const DeviceInfo &dev, int grid_cap, hipStream_t s,
                         bool *handled) {
  *handled = false;
  switch (a.L) {
    case 7: return run_exact_tp<7, MODE>(a, dev, grid_cap, s, handled);
    case 19: return run_exact_tp<19, MODE>(a, dev, grid_cap, s, handled);
    case 37: return run_exact_tp<37, MODE>(a, dev, grid_cap, s, handled);
    default: return hipSuccess;
  }
}

template <int LMAX, int MODE>
hipError_t run_generic(const FitArgs &a0, int block, const DeviceInfo &dev, int grid_cap,
                       hipStream_t s) {
  FitArgs a = a0;
  const int inv = (block * a.L + 15) / 16 * 16;
  const int eb = block * 4;
  const int row_bytes = a.L * a.TP * 4 * (MODE == 1 ? 2 : 1);
  const int budget = kLdsBytes - 2 * inv - eb - 256;
  int max_rows = budget / row_bytes;
  if (max_rows < 1) return hipErrorInvalidValue;
  const int tiles = (a.L + max_rows - 1) / max_rows;
  const int tr = (a.L + tiles - 1) / tiles;
  a.tile_rows = tr;
  a.inv_off = tr * row_bytes;
  a.e_off = a.inv_off + inv;
  a.stage_off = a.e_off + eb;
  const int total = a.stage_off + inv;
  const int cpr = block / a.K;
  const int rounds = (a.n + cpr - 1) / cpr;
  int grid = dev.cus * (kLdsBytes / total < 1 ? 1 : kLdsBytes / total);
  if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
  if (grid > rounds) grid = rounds;
  auto kern = k_fitness_generic<LMAX, MODE>;
  static LdsAttr attr;
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(kern), kLdsBytes);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), total, s, a);
  return launch_status(ae);
}

template <int MODE>
hipError_t run_generic_any(const FitArgs &a, int block, const DeviceInfo &dev, int grid_cap,
                           hipStream_t s) {
  if (a.L <= 8) return run_generic<8, MODE>(a, block, dev, grid_cap, s);
  if (a.L <= 16) return run_generic<16, MODE>(a, block, dev, grid_cap, s);
  if (a.L <= 32) return run_generic<32, MODE>(a, block, dev, grid_cap, s);
  return run_generic<64, MODE>(a, block, dev, grid_cap, s);
}

}  // namespace

// shape.block > 0 with shape.grid < 0 forces the generic variant (used by the
// tests to check that every variant gives the same bits).
hipError_t launch_fitness(const DevProblem &p, const uint8_t *pop, int n, float *fit,
                          const FitShape &shape, const DeviceInfo &dev, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  FitArgs a{};
  a.T2 = p.T2;
  a.T1 = p.T1;
  a.T2z = p.T2z;
  a.Town = p.Town;
  a.lconst = p.lconst;
  a.pop = pop;
  a.fit = fit;
  a.n = n;
  a.L = p.L;
  a.K = p.K;
  a.TP = p.TP;
  a.prelog = p.prelog;
  a.objective = p.objective;
  const bool force_generic = shape.grid < 0;
  const int grid_cap = shape.grid > 0 ? shape.grid : 0;
  if (!force_generic) {
    bool handled = false;
    hipError_t e = p.se_mode == 1 ? run_exact_any<1>(a, dev, grid_cap, s, &handled)
                                  : run_exact_any<0>(a, dev, grid_cap, s, &handled);
    if (handled) return e;
  }
  int block = shape.block > 0 ? shape.block : 256;
  if (block < p.K) block = p.K;
  block = (block + 63) / 64 * 64;
  if (block > 1024) block = 1024;
  return p.se_mode == 1 ? run_generic_any<1>(a, block, dev, grid_cap, s)
                        : run_generic_any<0>(a, block, dev, grid_cap, s);
}

}  // namespace pa
