// k_gen_wg.hip -- the one-workgroup solve of a small instance (Alg. 1 with
// the whole population, its fitness and the table resident in LDS).
//
// For instances whose table and population fit one CU, a generation of the
// persistent form is a chain of global round trips (tournament candidates'
// fitness, parents' rows, children, fitness) and a grid barrier.  Here one
// workgroup per instance runs generations [g0, g1) with workgroup barriers
// only: ranking and elites, tournaments, mutation codes, the children's rows
// (crossover, swaps, inverse rows) and their fitness all read and write LDS.
// Global memory is touched at entry (the initial population, or the
// population and fitness of generation g0 for a stepwise call), at every
// generation's trace entry, and at exit (the population and fitness of
// generation g1, and with `best` the result).  Same random words, same
// ranking, same canonical fitness order as the other forms: the same bits.
#include <algorithm>

#include "gen_core.h"
#include "pa_host.h"

namespace pa {
namespace {

constexpr int kWgMaxE = 63;  // elites ranked by one wave (top_e over LDS keys)

// LDS layout of one instance: table | populations x2 | fitness x2 | inverse
// rows | mutation codes x2 | tournaments | reduction scratch | elite indices.
template <int LT, int TPT, int MODE>
struct WgLayout {
  static constexpr bool kQuad = MODE == 0 && LT <= 19;
  static constexpr int kTableBytes =
      kQuad ? LT * TPT * quad_rows<LT>() * 4 : LT * LT * TPT * 4 * (MODE == 1 ? 2 : 1);
  int pop, fit, inv, code, sel, e, idx, total;
  __host__ __device__ WgLayout(int N, int K, int block) {
    auto up = [](int b) { return (b + 15) / 16 * 16; };
    const int popb = up(N * LT * K);
    pop = kTableBytes;
    fit = pop + 2 * popb;
    inv = fit + up(2 * N * 4);
    code = inv + up(N * K * LT);
    sel = code + 2 * popb;
    e = sel + up((N / 2 + 1) * 3 * 4);
    idx = e + block * 4;
    total = idx + 64 * 4;
  }
};

// The E best of the N fitness values in LDS, in rank order, into idx (one
// wave; repeated arg-max over keys below the previous maximum).
__device__ __forceinline__ void top_e_lds(const float *fin, int N, int E, int32_t *idx, int lane) {
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

// Inverse rows of chromosomes [c0, c0 + n) of pop (LDS) into inv: inv[c][s][j]
// = the user of cell j on pilot s (one thread per row).
__device__ __forceinline__ void wg_inverse(const uint8_t *pop, int c0, int n, int LT, int K,
                                           uint8_t *inv, int block) {
  for (int q = threadIdx.x; q < n * LT; q += block) {
    const int c = q / LT, j = q - c * LT;
    const uint8_t *row = pop + ((size_t)(c0 + c) * LT + j) * K;
    uint8_t *dst = inv + (size_t)c * K * LT + j;
    for (int k = 0; k < K; ++k) dst[(int)row[k] * LT] = (uint8_t)k;
  }
}

// One child row with K % 4 == 0, K <= 32, copied as 32-bit words.  With
// K = 4 the row is one register: its swaps (in increasing gene order, for the
// row's hits only) are byte shifts and its inverse entries are stored from
// the register.  Otherwise the swaps run in LDS (apply_swaps) only when the
// row has a hit, and the inverse entries come from word reads of the row.
__device__ __forceinline__ uint32_t swap_bytes(uint32_t w, int k, int kp) {
  const uint32_t a = (w >> (8 * k)) & 0xFFu, b = (w >> (8 * kp)) & 0xFFu;
  w &= ~((0xFFu << (8 * k)) | (0xFFu << (8 * kp)));
  return w | (b << (8 * k)) | (a << (8 * kp));
}
__device__ __forceinline__ void wg_row_words(const uint8_t *from, const uint8_t *code, int off,
                                             bool mutate, int K, uint8_t *row, uint8_t *dst,
                                             int LT) {
  const uint32_t *fw = reinterpret_cast<const uint32_t *>(from);
  const uint32_t *cw = reinterpret_cast<const uint32_t *>(code);
  uint32_t *rw = reinterpret_cast<uint32_t *>(row);
  if (K == 4) {
    uint32_t w = fw[0];
    if (mutate) {
      const uint32_t c = cw[0];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int cd = (int)((c >> (8 * k)) & 0xFFu);
        if (cd != 0) w = swap_bytes(w, k, cd - 1);
      }
    }
    rw[0] = w;
#pragma unroll
    for (int b = 0; b < 4; ++b) dst[(int)((w >> (8 * b)) & 0xFFu) * LT] = (uint8_t)b;
    return;
  }
  const int nw = K >> 2;
  bool hit_any = false;
  for (int i = 0; i < nw; ++i) {
    rw[i] = fw[i];
    if (mutate && cw[i] != 0u) hit_any = true;
  }
  if (hit_any) apply_swaps(row, code, off, K);
  for (int i = 0; i < nw; ++i) {
    const uint32_t x = rw[i];
#pragma unroll
    for (int b = 0; b < 4; ++b) dst[(int)((x >> (8 * b)) & 0xFFu) * LT] = (uint8_t)(4 * i + b);
  }
}

// Any other K: byte copies and apply_swaps.
__device__ __forceinline__ void wg_row_bytes(const uint8_t *from, const uint8_t *code, int off,
                                             bool mutate, int K, uint8_t *row, uint8_t *dst,
                                             int LT) {
  for (int k = 0; k < K; ++k) row[k] = from[k];
  if (mutate) apply_swaps(row, code, off, K);
  for (int k = 0; k < K; ++k) dst[(int)row[k] * LT] = (uint8_t)k;
}

// Fitness of chromosomes [0, n) whose inverse rows are in inv, into fit_out
// (LDS), block / K chromosomes per round.
template <int LT, int TPT, int MODE, int BLOCK>
__device__ __forceinline__ void wg_fitness(const GenInst &I, const uint8_t *inv, int n,
                                           const float *sT, float *sE, float *fit_out) {
  const int K = I.K, cpr = BLOCK / K;
  const int q = threadIdx.x;
  for (int r0 = 0; r0 < n; r0 += cpr) {
    const int nc = min(cpr, n - r0);
    const bool active = q < cpr * K && q / K < nc;
    const uint8_t *ip = inv + (size_t)(active ? r0 * K + q : 0) * LT;
    float acc = 0.0f;
    // a wave without a chromosome lane skips the gathers (it still joins the
    // reduction's barriers)
    if ((q & ~(kWave - 1)) < nc * K) {
      if constexpr (WgLayout<LT, TPT, MODE>::kQuad)
        acc = lane_sum_quad<LT, TPT>(ip, active, sT, I.objective);
      else
        acc = lane_sum_exact<LT, TPT, MODE, LT, 1>(ip, active, const_cast<float *>(sT), I.T2,
                                                   I.T1, I.lconst, I.objective);
    }
    float *dst = fit_out + r0;
    reduce_round_to(sE, acc, active, nc, K, I.prelog, [dst](int c, float v) { dst[c] = v; },
                    I.objective);
  }
}

template <int LT, int TPT, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_gen_wg(const GenInst *insts, int g0, int g1, int best) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const GenInst I = load_inst(insts, blockIdx.x);
  const int K = I.K, LK = LT * K, N = I.N, E = I.E, tid = threadIdx.x;
  const WgLayout<LT, TPT, MODE> W(N, K, BLOCK);
  float *sT = reinterpret_cast<float *>(smem);
  uint8_t *sPop[2] = {smem + W.pop, smem + W.pop + (W.fit - W.pop) / 2};
  float *sFit[2] = {reinterpret_cast<float *>(smem + W.fit),
                    reinterpret_cast<float *>(smem + W.fit) + N};
  uint8_t *sInv = smem + W.inv;
  uint8_t *sCodes[2] = {smem + W.code, smem + W.code + (W.sel - W.code) / 2};
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + W.sel);
  float *sE = reinterpret_cast<float *>(smem + W.e);
  int32_t *sIdx = reinterpret_cast<int32_t *>(smem + W.idx);
  // the table
  if constexpr (WgLayout<LT, TPT, MODE>::kQuad)
    load_quad(I.T2, LT, TPT, 0, LT, quad_rows<LT>(), sT);
  else
    load_tile<MODE>(I.T2, I.T1, LT, TPT, 0, LT, LT, sT);
  // the starting population (and its fitness, unless this is the start)
  const int gs = g0 < 0 ? 0 : g0;
  {
    const uint8_t *src = pop_buf(I, gs & 1);
    for (int i = tid; i < N * LK; i += BLOCK) sPop[gs & 1][i] = gp(src)[i];
    if (g0 >= 0)
      for (int i = tid; i < N; i += BLOCK) sFit[gs & 1][i] = gp(fit_buf(I, gs & 1))[i];
  }
  __syncthreads();
  if (g0 < 0) {
    wg_inverse(sPop[0], 0, N, LT, K, sInv, BLOCK);
    __syncthreads();
    wg_fitness<LT, TPT, MODE, BLOCK>(I, sInv, N, sT, sE, sFit[0]);
  }
  const int gend = min(g1, I.G);
  const bool mutate = K >= 2 && I.ga.thr_mut != 0;
  const int nch = N - E, npairs = (nch + 1) / 2;
  // the waves of the tournaments and of the codes (see the generation loop)
  const int sel_base = BLOCK > kWave ? kWave : 0;
  const int sel_waves = (npairs + kWave - 1) / kWave;
  const int code_base = sel_base + sel_waves * kWave < BLOCK ? sel_base + sel_waves * kWave : 0;
  // the waves the children's fitness leaves idle (a population smaller than
  // one round of lanes) draw the next generation's codes meanwhile
  const int fit_lanes = min(nch, BLOCK / K) * K;
  const int pre_base = (fit_lanes + kWave - 1) / kWave * kWave;
  // (only when one pass of eight lanes per group of 32 genes fits them: more
  // passes take longer than the gathers they would hide behind)
  const bool prefetch =
      mutate && nch > 0 && pre_base < BLOCK && 8 * nch * ((LK + 31) >> 5) <= BLOCK - pre_base;
  for (int g = gs; g < gend; ++g) {
    const uint8_t *pin = sPop[g & 1];
    uint8_t *pout = sPop[(g + 1) & 1];
    const float *fin = sFit[g & 1];
    float *fout = sFit[(g + 1) & 1];
    // three independent jobs on separate waves: wave 0 ranks (the elites, at
    // least the best for the trace), the next waves draw the tournaments and
    // the rest the mutation codes (each job falls back to every thread from
    // its first wave on when the workgroup is too small for the split)
    if (tid < kWave) top_e_lds(fin, N, E > 1 ? E : 1, sIdx, tid);
    // tournaments, crossover decisions and cuts, one thread per pair (the
    // words of the pair's first slot)
    for (int q = tid - sel_base; tid >= sel_base && q < npairs; q += BLOCK - sel_base) {
      const uint32_t a = (uint32_t)(E + 2 * q);
      const Stream st{I.ga.seed_lo, I.ga.seed_hi, a, (uint32_t)g, I.ga.instance_id, kTagSelect};
      const Words4 b0 = st.block(0u), b1 = st.block(1u);
      const uint32_t Nu = (uint32_t)N;
      const uint32_t u0 = bounded(b0.x, Nu), v0 = bounded(b0.y, Nu);
      const uint32_t u1 = bounded(b0.z, Nu), v1 = bounded(b0.w, Nu);
      const uint32_t p1 = beats(rank_key(fin[v0]), v0, rank_key(fin[u0]), u0) ? v0 : u0;
      const uint32_t p2 = beats(rank_key(fin[v1]), v1, rank_key(fin[u1]), u1) ? v1 : u1;
      const bool cross = LT >= 2 && hit(b1.x, I.ga.thr_cross);
      sSel[3 * q] = (int32_t)p1;
      sSel[3 * q + 1] = (int32_t)p2;
      sSel[3 * q + 2] = cross ? 1 + (int)bounded(b1.y, (uint32_t)(LT - 1)) : LT;
    }
    uint8_t *sCode = sCodes[g & 1];
    if (mutate && !(prefetch && g > gs))
      mutation_codes_block(sCode, nch, LK, K, I.ga, (uint32_t)g, E, BLOCK, code_base);
    __syncthreads();
    // the children's rows: crossover, swaps, inverse rows (one thread per row)
    for (int r = tid; r < nch * LT; r += BLOCK) {
      const int ci = r / LT, j = r - ci * LT;
      const int q = ci >> 1;
      const bool second = (ci & 1) != 0;
      const int p1 = sSel[3 * q], p2 = sSel[3 * q + 1], cut = sSel[3 * q + 2];
      const int src = j < cut ? (second ? p2 : p1) : (second ? p1 : p2);
      uint8_t *row = pout + (size_t)(E + ci) * LK + j * K;
      const uint8_t *from = pin + (size_t)src * LK + j * K;
      const uint8_t *code = sCode + (size_t)ci * LK + j * K;
      uint8_t *dst = sInv + (size_t)ci * K * LT + j;
      if ((K & 3) == 0 && K <= 32)
        wg_row_words(from, code, ci * LK + j * K, mutate, K, row, dst, LT);
      else
        wg_row_bytes(from, code, ci * LK + j * K, mutate, K, row, dst, LT);
    }
    // elites into the first E slots, with their fitness (by the threads past
    // the rows', else by all of them after their rows)
    {
      const int ebase = nch * LT < BLOCK ? nch * LT : 0;
      if (tid >= ebase) {
        for (int i = tid - ebase; i < E * LK; i += BLOCK - ebase) {
          const int e = i / LK;
          pout[i] = pin[sIdx[e] * LK + (i - e * LK)];
        }
        for (int e = tid - ebase; e < E; e += BLOCK - ebase) fout[e] = fin[sIdx[e]];
      }
    }
    if (tid == 0) gp(I.trace)[g] = fin[sIdx[0]];
    __syncthreads();
    if (prefetch && g + 1 < gend)
      mutation_codes_block(sCodes[(g + 1) & 1], nch, LK, K, I.ga, (uint32_t)(g + 1), E, BLOCK,
                           pre_base);
    wg_fitness<LT, TPT, MODE, BLOCK>(I, sInv, nch, sT, sE, fout + E);
  }
  // the population and fitness of generation gend, and the result
  const int gb = gend & 1;
  {
    uint8_t *dst = pop_buf(I, gb);
    for (int i = tid; i < N * LK; i += BLOCK) gp(dst)[i] = sPop[gb][i];
    for (int i = tid; i < N; i += BLOCK) gp(fit_buf(I, gb))[i] = sFit[gb][i];
  }
  if (best && gend == I.G) {
    if (tid < kWave) top_e_lds(sFit[gb], N, 1, sIdx, tid);
    __syncthreads();
    const int b = sIdx[0];
    if (tid == 0) {
      *gp(I.best_idx) = b;
      *gp(I.best_fit) = sFit[gb][b];
      gp(I.trace)[I.G] = sFit[gb][b];
    }
    for (int i = tid; i < LK; i += BLOCK) gp(I.best_out)[i] = sPop[gb][b * LK + i];
  }
}

template <int LT, int TPT, int MODE, int BLOCK>
hipError_t wg_launch(const GenInst *d_insts, int ninst, int g0, int g1, bool best, int maxN,
                     int maxK, int *lds_out, hipStream_t s) {
  const int lds = WgLayout<LT, TPT, MODE>(maxN, maxK, BLOCK).total;
  if (lds_out) {
    *lds_out = lds;
    return hipSuccess;
  }
  static LdsAttr attr;
  const hipError_t ae =
      allow_lds_once(attr, reinterpret_cast<const void *>(k_gen_wg<LT, TPT, MODE, BLOCK>), kLdsBytes);
  hipLaunchKernelGGL((k_gen_wg<LT, TPT, MODE, BLOCK>), dim3(ninst), dim3(BLOCK), lds, s, d_insts,
                     g0, g1, best ? 1 : 0);
  return launch_status(ae);
}

template <int LT, int TPT, int MODE>
hipError_t wg_dispatch_block(int block, const GenInst *d, int n, int g0, int g1, bool best,
                             int maxN, int maxK, int *lds, hipStream_t s) {
  if (block == 256) return wg_launch<LT, TPT, MODE, 256>(d, n, g0, g1, best, maxN, maxK, lds, s);
  if (block == 512) return wg_launch<LT, TPT, MODE, 512>(d, n, g0, g1, best, maxN, maxK, lds, s);
  return hipErrorInvalidValue;
}

template <int LT, int MODE>
hipError_t wg_dispatch_tp(int TP, int block, const GenInst *d, int n, int g0, int g1, bool best,
                          int maxN, int maxK, int *lds, hipStream_t s) {
  switch (TP) {
    case 4: return wg_dispatch_block<LT, 4, MODE>(block, d, n, g0, g1, best, maxN, maxK, lds, s);
    case 8: return wg_dispatch_block<LT, 8, MODE>(block, d, n, g0, g1, best, maxN, maxK, lds, s);
    case 16: return wg_dispatch_block<LT, 16, MODE>(block, d, n, g0, g1, best, maxN, maxK, lds, s);
    case 32:
      if constexpr (LT <= 19)
        return wg_dispatch_block<LT, 32, MODE>(block, d, n, g0, g1, best, maxN, maxK, lds, s);
      return hipErrorInvalidValue;  // an L=37, TP=32 table does not fit beside a population
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// The one-workgroup form for (L, TP, mode) with `block` threads: with lds_out
// set, only the LDS bytes of the largest instance (maxN, maxK) into *lds_out
// (hipErrorInvalidValue when no such variant exists); else the launch of
// generations [g0, g1) of ninst instances, one workgroup each.
hipError_t launch_gen_wg(const GenInst *d_insts, int ninst, int L, int TP, int mode, int block,
                         int g0, int g1, bool best, int maxN, int maxK, int *lds_out,
                         hipStream_t s) {
  if (maxN < 2 || maxK < 1 || maxK > TP) return hipErrorInvalidValue;
  if (mode == 0) {
    if (L == 7) return wg_dispatch_tp<7, 0>(TP, block, d_insts, ninst, g0, g1, best, maxN, maxK, lds_out, s);
    if (L == 19) return wg_dispatch_tp<19, 0>(TP, block, d_insts, ninst, g0, g1, best, maxN, maxK, lds_out, s);
    if (L == 37) return wg_dispatch_tp<37, 0>(TP, block, d_insts, ninst, g0, g1, best, maxN, maxK, lds_out, s);
  } else if (mode == 1) {
    if (L == 7) return wg_dispatch_tp<7, 1>(TP, block, d_insts, ninst, g0, g1, best, maxN, maxK, lds_out, s);
    if (L == 19) return wg_dispatch_tp<19, 1>(TP, block, d_insts, ninst, g0, g1, best, maxN, maxK, lds_out, s);
  }
  return hipErrorInvalidValue;
}

int wg_max_elites() { return kWgMaxE; }

}  // namespace pa
