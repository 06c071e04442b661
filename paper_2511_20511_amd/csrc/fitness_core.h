// fitness_core.h -- device code of the fitness evaluation (Sec. 3.2, Eq. 5-6):
// the uplink sum spectral efficiency of chromosomes whose inverse rows are in
// LDS, against the normalised fading table staged in LDS.
//
// Work mapping: one lane per (chromosome c, pilot p).  For every BS row l
// (uniform across the wave) the lane gathers the L table entries
// T[l][j][u_j(p)], u_j(p) the user of cell j on pilot p, out of one row
// segment of at most 32 consecutive words per j: lanes of all chromosomes in
// the wave read from the same segment, so every bank serves one word (or a
// broadcast) and the gather is free of bank conflicts.
//
// Canonical FP32 order (identical in every variant, so a chromosome's fitness
// has the same bits whatever the batch, tile or launch shape):
//   per (c, p):   for l = 0 .. L-1 in order:
//                   I = sum_{j != l} T2[l][j][u_j(p)] in increasing j (from 0),
//                   b2 = T2[l][l][u_l(p)],
//                   asymptotic: se = log2(fma(b2, rcp(I), 1))
//                   finite-M:   S = sum_j T1[l][j][u_j(p)] in increasing j,
//                               se = log2(fma(b2, rcp(fma(c2_l, fma(a_l, S, 1), I)), 1))
//                   acc += se
//   per c:        pairwise tree over p (stride halving from the next power
//                 of two, missing partners skipped), then * prelog.
// rcp and log2 are the hardware v_rcp_f32 / v_log_f32 (about 1 ulp).
#pragma once
#include "pa_dev.h"

namespace pa {

// Objective `mn`: 0 the sum of the SE terms (Eq. 7); 1 the minimum of the
// users' SINR (max-min SIR; the SINR is b2 * rcp(den), about 1e-7 relative,
// where log2(1 + x) in FP32 would lose the small terms); 2 the sum of minus
// the users' interference-to-signal ratios of Eq. 8 (tables of first-power
// gains: b2 is the own gain, I the sum of the interferers').  The reductions
// are taken in the canonical order; only objective 0 is scaled by the pre-log.
__device__ __forceinline__ float obj_init(int mn) { return mn == 1 ? __builtin_inff() : 0.0f; }
__device__ __forceinline__ float obj_add(float acc, float se, int mn) {
  return mn == 1 ? __builtin_fminf(acc, se) : acc + se;
}

// Branch-free in the objective: marked unpredictable, the final choice stays a
// select; as a uniform branch around the log it would split each BS row into
// blocks of its own and keep adjacent rows' LDS reads from pairing (ds_read2).
__device__ __forceinline__ float se_asym(float b2, float I, int mn = 0) {
  const float r = __builtin_amdgcn_rcpf(mn == 2 ? b2 : I);
  const float se = __builtin_amdgcn_logf(__builtin_fmaf(b2, r, 1.0f));
  const float q = (mn == 2 ? -I : b2) * r;
  return __builtin_unpredictable(mn == 0) ? se : q;
}

// (objective 2 takes no finite-M form: the host rejects that combination)
__device__ __forceinline__ float se_finite(float b2, float I, float S, float a, float c2,
                                           int mn = 0) {
  const float t = __builtin_fmaf(a, S, 1.0f);
  const float den = __builtin_fmaf(c2, t, I);
  const float r = __builtin_amdgcn_rcpf(den);
  return mn == 1 ? b2 * r : __builtin_amdgcn_logf(__builtin_fmaf(b2, r, 1.0f));
}

// Inverse rows of the chromosomes of a round, stored pilot-major:
// inv[c][s][j] = the user of cell j that sends pilot s in chromosome c, so a
// lane (c, s) finds its L entries contiguous.  One thread per row (c, j) of
// the round's bytes `src` (LDS, 4-byte aligned, nrows*K bytes), read as
// aligned 32-bit words; pilots >= K (invalid input) are skipped so the write
// stays inside the chromosome.
__device__ __forceinline__ void build_inverse(const uint8_t *src, int nrows, int L, int K,
                                              uint8_t *sInv, int stride = 0) {
  const int ST = stride > 0 ? stride : L;  // inverse row stride (bytes)
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
    const int c = r / L, j = r - c * L;
    const uint8_t *rp = src + r * K;
    const int mis = (int)((uintptr_t)rp & 3u);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(rp - mis);
    const int nw = (mis + K + 3) >> 2;
    uint8_t *dst = sInv + c * K * ST + j;
#pragma unroll 4
    for (int i = 0; i < nw; ++i) {
      const uint32_t v = w[i];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 4 * i + b - mis;
        const int s = (int)((v >> (8 * b)) & 0xFFu);
        if (k >= 0 && k < K && s < K) dst[s * ST] = (uint8_t)k;
      }
    }
  }
}

// The inverse row of lane q = (c, p) of a round (chromosome c = q / K, pilot
// p = q % K; inv[j] = the user of cell j on pilot p) into sInv + q * LT,
// straight from the round's chromosome bytes in LDS (row-major [c][j][k]):
// lane (c, x) reads the pilot s of user x of cell j and sends x to lane
// (c, s) with ds_permute, so each lane writes only its own row and no
// workgroup pass or barrier is needed.  K must divide 64 (a chromosome's
// lanes lie in one wave) and every lane of the wave calls it.  Rows must be
// permutations: lanes past the round's last chromosome read stale bytes and
// send inside their own group.  The same inverse rows as build_inverse.
template <int LT, int ST = LT>
__device__ __forceinline__ void inverse_rows_permute(const uint8_t *stage, int K, uint8_t *sInv) {
  const int q = (int)threadIdx.x;
  const int x = q & (K - 1);
  const int base = (q & 63) - x;
  const uint8_t *row = stage + (q - x) * LT + x;  // user x of cell 0 of chromosome q / K
  uint8_t *dst = sInv + q * ST;
  // all reads, then all permutes, then all writes (interleaved, each write
  // could alias a later read and the three would wait on each other per cell)
  int v[LT];
#pragma unroll
  for (int j = 0; j < LT; ++j) v[j] = row[j * K];
#pragma unroll
  for (int j = 0; j < LT; ++j) v[j] = __builtin_amdgcn_ds_permute((base + (v[j] & (K - 1))) << 2, x);
  if constexpr (ST % 4 == 0) {
    // a row stride of whole words: the row as 32-bit stores
#pragma unroll
    for (int i = 0; i < ST / 4; ++i) {
      uint32_t w = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (4 * i + b < LT) w |= ((uint32_t)v[4 * i + b] & 0xFFu) << (8 * b);
      reinterpret_cast<uint32_t *>(dst)[i] = w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < LT; ++j) dst[j] = (uint8_t)v[j];
  }
}

// Row stride of the population-fitness kernels' inverse rows: L rounded up to
// whole 32-bit words, so that a lane writes and reads its row by words.
template <int LT>
constexpr int inv_stride() {
  return (LT + 3) & ~3;
}

// The LT bytes of a lane's inverse row into A: 32-bit reads when the rows'
// stride ST is a whole number of words (ip then 4-byte aligned), else bytes.
template <int LT, int ST>
__device__ __forceinline__ void read_inv_row(const uint8_t *ip, uint32_t (&A)[LT]) {
  if constexpr (ST % 4 == 0) {
#pragma unroll
    for (int i = 0; i < (LT + 3) / 4; ++i) {
      const uint32_t w = reinterpret_cast<const uint32_t *>(ip)[i];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (4 * i + b < LT) A[4 * i + b] = (w >> (8 * b)) & 0xFFu;
    }
  } else {
#pragma unroll
    for (int j = 0; j < LT; ++j) A[j] = ip[j];
  }
}

// LDS tile layout: cell-major, T[j][lr][p] (asymptotic) or T[j][lr][2][p]
// (finite-M: the T2 row then the T1 row), lr the BS row inside the tile.  A
// lane's base register A[j] = byte address of T[j][0][u_j(p)]; the BS row is a
// compile-time immediate offset lr * row_bytes (at most a few KiB), so each
// gather is one ds_read_b32 with an immediate offset.

// One BS row for a lane, L known at compile time: returns the SE term.
template <int LT, int MODE>
__device__ __forceinline__ float row_term_exact(const char *lds, const uint32_t (&A)[LT],
                                                uint32_t off, uint32_t t1_bytes, int l,
                                                float a_l, float c2_l, int mn = 0) {
  float I = 0.0f, b2 = 0.0f;
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const float g = *reinterpret_cast<const float *>(lds + A[j] + off);
    if (j == l)
      b2 = g;
    else
      I = I + g;
  }
  if constexpr (MODE == 1) {
    float S = 0.0f;
#pragma unroll
    for (int j = 0; j < LT; ++j)
      S = S + *reinterpret_cast<const float *>(lds + A[j] + off + t1_bytes);
    return se_finite(b2, I, S, a_l, c2_l, mn);
  } else {
    return se_asym(b2, I, mn);
  }
}

// Same for a runtime L <= LMAX.
template <int LMAX, int MODE>
__device__ __forceinline__ float row_term_generic(const char *lds, const uint32_t (&A)[LMAX],
                                                  uint32_t off, uint32_t t1_bytes, int L, int l,
                                                  float a_l, float c2_l, int mn = 0) {
  float I = 0.0f, b2 = 0.0f, S = 0.0f;
#pragma unroll
  for (int j = 0; j < LMAX; ++j) {
    if (j < L) {
      const float g = *reinterpret_cast<const float *>(lds + A[j] + off);
      if (j == l)
        b2 = g;
      else
        I = I + g;
      if constexpr (MODE == 1) S = S + *reinterpret_cast<const float *>(lds + A[j] + off + t1_bytes);
    }
  }
  if constexpr (MODE == 1) return se_finite(b2, I, S, a_l, c2_l, mn);
  return se_asym(b2, I, mn);
}

// Copies BS rows [r0, r0 + rows) of the cell-major tables T2[j][l][TP]
// (and T1) into the LDS tile T[j][lr][..] with rows_alloc rows per cell.
// Each thread issues up to 8 independent 16-byte loads before storing, so a
// small workgroup is not bound by one global-memory round trip per element.
template <int MODE>
__device__ __forceinline__ void load_tile(const float *__restrict__ T2, const float *__restrict__ T1,
                                          int L, int TP, int r0, int rows, int rows_alloc,
                                          float *dst) {
  constexpr int kBatch = 8;
  const int q = TP >> 2;  // float4 per table row
  const int per_cell = rows * q;
  const int total = L * per_cell;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gptr<const f4> s2 = gp(reinterpret_cast<const f4 *>(T2));
  const gptr<const f4> s1 = gp(reinterpret_cast<const f4 *>(T1));
  f4 *d = reinterpret_cast<f4 *>(dst);
  const int step = (int)blockDim.x;
  for (int base = threadIdx.x; base < total; base += kBatch * step) {
    f4 v2[kBatch], v1[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = min(base + u * step, total - 1);  // clamped: every load is in bounds
      const int j = i / per_cell, rem = i - j * per_cell;
      const int lr = rem / q, c = rem - lr * q;
      const size_t src = ((size_t)j * L + r0 + lr) * q + c;
      v2[u] = s2[src];
      if constexpr (MODE == 1) v1[u] = s1[src];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * step;
      if (i < total) {
        const int j = i / per_cell, rem = i - j * per_cell;
        const int lr = rem / q, c = rem - lr * q;
        if constexpr (MODE == 0) {
          d[(j * rows_alloc + lr) * q + c] = v2[u];
        } else {
          d[((j * rows_alloc + lr) * 2) * q + c] = v2[u];
          d[((j * rows_alloc + lr) * 2 + 1) * q + c] = v1[u];
        }
      }
    }
  }
}

constexpr int kLdsBytes = 163840;  // LDS per workgroup on gfx950

// LDS plan: the table tile next to `EXTRA` bytes of other buffers.
template <int LT, int TPT, int MODE, int EXTRA>
struct TilePlan {
  static constexpr int kRowBytes = LT * TPT * 4 * (MODE == 1 ? 2 : 1);  // one BS row, all cells
  static constexpr int kBudget = kLdsBytes - EXTRA - 256;
  static constexpr int kMaxRows = kBudget / kRowBytes;
  static constexpr int kTiles = (LT + kMaxRows - 1) / kMaxRows;
  static constexpr int kTileRows = (LT + kTiles - 1) / kTiles;
  static constexpr int kTableBytes = kTileRows * kRowBytes;
  static_assert(kMaxRows >= 1, "one BS row must fit in LDS");
};

// Sum over all BS rows of the SE terms of lane (c, p) in the canonical order;
// `ip` = inv[c][p][0..L).  With more than one tile the tiles are (re)loaded
// here, so every thread of the workgroup must call this (inactive lanes too).
template <int LT, int TPT, int MODE, int TR, int NT, int ST = LT>
__device__ __forceinline__ float lane_sum_exact(const uint8_t *ip, bool active, float *sT,
                                                const float *__restrict__ T2,
                                                const float *__restrict__ T1,
                                                const float *__restrict__ lconst, int mn = 0) {
  constexpr int ROWB = TPT * 4 * (MODE == 1 ? 2 : 1);  // bytes per (cell, BS row)
  constexpr int CELLB = TR * ROWB;                      // bytes per cell in the tile
  const char *lds = reinterpret_cast<const char *>(sT);
  // ip lies inside the inverse-row region for inactive lanes too: every lane
  // loads (no per-element branch, all loads in flight at once), then masks
  uint32_t A[LT];
  read_inv_row<LT, ST>(ip, A);
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const uint32_t v = active ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (TPT - 1)) * 4u;
  }
  float acc = obj_init(mn);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if constexpr (NT > 1) {
      __syncthreads();
      const int rows = (t + 1) * TR <= LT ? TR : LT - t * TR;
      load_tile<MODE>(T2, T1, LT, TPT, t * TR, rows, TR, sT);
      __syncthreads();
    }
#pragma unroll
    for (int lr = 0; lr < TR; ++lr) {
      const int l = t * TR + lr;
      if (l < LT) {
        float a_l = 0.0f, c2_l = 0.0f;
        if constexpr (MODE == 1) {
          a_l = gp(lconst)[2 * l];
          c2_l = gp(lconst)[2 * l + 1];
        }
        acc = obj_add(acc,
                      row_term_exact<LT, MODE>(lds, A, (uint32_t)(lr * ROWB), TPT * 4u, l, a_l,
                                               c2_l, mn),
                      mn);
      }
    }
  }
  return acc;
}

// Quad layout of a whole table in LDS: Q[j][u][l], the BS rows l of one
// (cell j, pilot u) contiguous and padded to LP rows, LP a multiple of 4 with
// LP / 4 odd so that the 16-byte row groups of different pilots start in
// different bank groups.  A lane then reads four BS rows of one cell with a
// single ds_read_b128 (the padding rows are never used).
template <int LT>
constexpr int quad_rows() {
  return ((LT + 3) / 4) % 2 == 1 ? (LT + 3) / 4 * 4 : (LT + 3) / 4 * 4 + 4;
}

// Copies BS rows [r0, r0 + rows) of the cell-major table T2[j][l][TP] into
// the quad layout Q[j][u][lr] with LP rows per (cell, pilot) (r0 and LP
// multiples of 4, rows <= LP).  A thread takes 4 rows x 4 pilots of one cell:
// four 16-byte global loads (a row past the table's last is clamped: its
// values land in padding rows that are never read), a 4x4 transpose in
// registers and four 16-byte LDS stores.
__device__ __forceinline__ void load_quad(const float *__restrict__ T2, int L, int TP, int r0,
                                          int rows, int LP, float *dst) {
  constexpr int kBatch = 4;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int q = TP >> 2;             // float4 per table row
  const int ng = (rows + 3) >> 2;    // row groups
  const int per_cell = ng * q;
  const int total = L * per_cell;
  const gptr<const f4> s2 = gp(reinterpret_cast<const f4 *>(T2));
  f4 *d = reinterpret_cast<f4 *>(dst);
  const int step = (int)blockDim.x;
  for (int base = threadIdx.x; base < total; base += kBatch * step) {
    f4 v[kBatch][4];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = min(base + u * step, total - 1);  // clamped: every load is in bounds
      const int j = i / per_cell, rem = i - j * per_cell;
      const int g = rem / q, c = rem - g * q;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = min(r0 + 4 * g + r, L - 1);
        v[u][r] = s2[((size_t)j * L + l) * q + c];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = base + u * step;
      if (i < total) {
        const int j = i / per_cell, rem = i - j * per_cell;
        const int g = rem / q, c = rem - g * q;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const f4 o = {v[u][0][k], v[u][1][k], v[u][2][k], v[u][3][k]};
          d[(((size_t)j * TP + 4 * c + k) * LP + 4 * g) >> 2] = o;
        }
      }
    }
  }
}

// lane_sum_exact (asymptotic SE) on the quad layout: for each group of four
// BS rows, one 16-byte gather per cell feeds the four rows' interference
// sums, each over j != l in increasing j; the SE terms are added in
// increasing l.  Same arithmetic, same order, same bits as lane_sum_exact.
template <int LT, int TPT, int ST = LT>
__device__ __forceinline__ float lane_sum_quad(const uint8_t *ip, bool active, const float *sQ,
                                               int mn = 0) {
  constexpr int LP = quad_rows<LT>();
  constexpr int CELLB = TPT * LP * 4;  // bytes per cell
  typedef float f4 __attribute__((ext_vector_type(4)));
  const char *lds = reinterpret_cast<const char *>(sQ);
  uint32_t A[LT];
  read_inv_row<LT, ST>(ip, A);  // in bounds for inactive lanes too
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const uint32_t v = active ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (TPT - 1)) * (uint32_t)(LP * 4);
  }
  float acc = obj_init(mn);
#pragma unroll
  for (int g = 0; g < LP / 4; ++g) {
    if (4 * g < LT) {
      float I[4] = {0.0f, 0.0f, 0.0f, 0.0f}, b2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < LT; ++j) {
        const f4 v = *reinterpret_cast<const f4 *>(lds + A[j] + 16 * g);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 4 * g + r;
          if (l < LT) {
            if (j == l)
              b2[r] = v[r];
            else
              I[r] = I[r] + v[r];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * g + r < LT) acc = obj_add(acc, se_asym(b2[r], I[r], mn), mn);
      // the next group's gathers wait for this group's sum: without this the
      // compiler hoists every group's loads to the top and spills
#pragma unroll
      for (int j = 0; j < LT; ++j) asm volatile("" : "+v"(A[j]) : "v"(acc));
    }
  }
  return acc;
}

// Latency form of lane_sum_exact for a whole-table tile: the BS rows are
// split over RS groups of GS lanes (GS >= 64, so the group index is uniform
// per wave).  Lane ql of group rg computes the SE terms of rows l = rg,
// rg + RS, ... and stores them in sSe[ql][l]; after a barrier lane ql of group
// 0 adds its L terms in increasing l, the canonical order (same bits as
// lane_sum_exact).  Returns that sum in group 0 (0 elsewhere).  Every thread
// of the workgroup must call it.
template <int LT, int TPT, int MODE>
__device__ __forceinline__ float lane_sum_split(const uint8_t *sInv, int ql, bool active, int rg,
                                                int RS, const float *sT, float *sSe,
                                                const float *__restrict__ lconst,
                                                int mn = 0) {
  constexpr int ROWB = TPT * 4 * (MODE == 1 ? 2 : 1);
  constexpr int CELLB = LT * ROWB;
  const char *lds = reinterpret_cast<const char *>(sT);
  const uint8_t *ip = sInv + ql * LT;  // inside the inverse region for every lane
  uint32_t A[LT];
#pragma unroll
  for (int j = 0; j < LT; ++j) A[j] = ip[j];
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const uint32_t v = active ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (TPT - 1)) * 4u;
  }
  for (int l = rg; l < LT; l += RS) {
    const uint32_t off = (uint32_t)(l * ROWB);
    float I = 0.0f, b2 = 0.0f;
#pragma unroll
    for (int j = 0; j < LT; ++j) {
      const float g = *reinterpret_cast<const float *>(lds + A[j] + off);
      const bool own = j == l;
      b2 = own ? g : b2;
      I = own ? I : I + g;
    }
    float se;
    if constexpr (MODE == 1) {
      float S = 0.0f;
#pragma unroll
      for (int j = 0; j < LT; ++j)
        S = S + *reinterpret_cast<const float *>(lds + A[j] + off + TPT * 4);
      se = se_finite(b2, I, S, gp(lconst)[2 * l], gp(lconst)[2 * l + 1], mn);
    } else {
      se = se_asym(b2, I, mn);
    }
    sSe[ql * LT + l] = se;
  }
  __syncthreads();
  float acc = obj_init(mn);
  if (rg == 0) {
#pragma unroll
    for (int l = 0; l < LT; ++l) acc = obj_add(acc, sSe[ql * LT + l], mn);
  }
  return acc;
}

// lane_sum_split on the quad layout (asymptotic SE): group rg takes the
// four-row groups rg, rg + RS, ...; per group one 16-byte gather per cell
// feeds four interference sums (over j != l in increasing j), the SE terms go
// to sSe[ql][l] and after a barrier lane ql of group 0 adds its L terms in
// increasing l.  Same bits as lane_sum_split.  Every thread of the workgroup
// must call it.
template <int LT, int TPT>
__device__ __forceinline__ float lane_sum_split_quad(const uint8_t *sInv, int ql, bool active,
                                                     int rg, int RS, const float *sQ, float *sSe,
                                                     int mn = 0) {
  constexpr int LP = quad_rows<LT>();
  constexpr int CELLB = TPT * LP * 4;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const char *lds = reinterpret_cast<const char *>(sQ);
  const uint8_t *ip = sInv + ql * LT;  // inside the inverse region for every lane
  uint32_t A[LT];
#pragma unroll
  for (int j = 0; j < LT; ++j) A[j] = ip[j];
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const uint32_t v = active ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (TPT - 1)) * (uint32_t)(LP * 4);
  }
  for (int g = rg; 4 * g < LT; g += RS) {
    float I[4] = {0.0f, 0.0f, 0.0f, 0.0f}, b2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < LT; ++j) {
      const f4 v = *reinterpret_cast<const f4 *>(lds + A[j] + 16 * g);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool own = j == 4 * g + r;
        b2[r] = own ? v[r] : b2[r];
        I[r] = own ? I[r] : I[r] + v[r];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int l = 4 * g + r;
      if (l < LT) sSe[ql * LT + l] = se_asym(b2[r], I[r], mn);
    }
  }
  __syncthreads();
  float acc = obj_init(mn);
  if (rg == 0) {
#pragma unroll
    for (int l = 0; l < LT; ++l) acc = obj_add(acc, sSe[ql * LT + l], mn);
  }
  return acc;
}

// Tiled tables (more BS rows than LDS holds).  The tiles hold the table with
// its own-cell entries zeroed (T2z[j][l][.] = 0 for j == l) and the own-cell
// squares come from a small LDS table sOwn[l][p], so the tile loop need not
// be unrolled: I sums every j in increasing order, and adding the exact +0.0
// at j == l gives the same bits as skipping it.

// A lane's base offsets into a tile of TR BS rows (cell-major).
template <int LT, int TPT, int MODE, int TR, int ST = LT>
__device__ __forceinline__ void tiled_offsets(const uint8_t *ip, bool active, uint32_t (&A)[LT]) {
  constexpr int ROWB = TPT * 4 * (MODE == 1 ? 2 : 1);
  constexpr int CELLB = TR * ROWB;
  // ip lies inside the inverse-row region for inactive lanes too
  read_inv_row<LT, ST>(ip, A);
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    const uint32_t v = active ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (TPT - 1)) * 4u;
  }
}

// SE term of BS row l (row lr of the tile in LDS) for a lane.
template <int LT, int TPT, int MODE>
__device__ __forceinline__ float tiled_row_se(const uint32_t (&A)[LT], const uint8_t *ip,
                                              bool active, const char *lds, const float *sOwn,
                                              const float *__restrict__ lconst, int l, int lr,
                                              int mn) {
  constexpr int ROWB = TPT * 4 * (MODE == 1 ? 2 : 1);
  const uint32_t ownr = ip[l];  // in bounds for inactive lanes too
  const uint32_t own = active ? ownr : 0u;
  const float b2 = sOwn[l * TPT + (int)(own & (TPT - 1))];
  const uint32_t off = (uint32_t)(lr * ROWB);
  float I = 0.0f;
#pragma unroll
  for (int j = 0; j < LT; ++j) I = I + *reinterpret_cast<const float *>(lds + A[j] + off);
  if constexpr (MODE == 1) {
    float S = 0.0f;
#pragma unroll
    for (int j = 0; j < LT; ++j)
      S = S + *reinterpret_cast<const float *>(lds + A[j] + off + TPT * 4);
    return se_finite(b2, I, S, gp(lconst)[2 * l], gp(lconst)[2 * l + 1], mn);
  } else {
    return se_asym(b2, I, mn);
  }
}

// Adds the SE terms of the BS rows of tile t (already in LDS) to acc, in
// increasing l.
template <int LT, int TPT, int MODE, int TR>
__device__ __forceinline__ float tiled_rows(uint32_t (&A)[LT], const uint8_t *ip, bool active,
                                            const float *sT, const float *sOwn,
                                            const float *__restrict__ lconst, int t, float acc,
                                            int mn = 0) {
  const char *lds = reinterpret_cast<const char *>(sT);
  const int rows = (t + 1) * TR <= LT ? TR : LT - t * TR;
  // Branch-free over the tile's rows (a row past the last BS row of a short
  // final tile reads stale but in-bounds LDS and is not added), so the rows
  // stay in order instead of being hoisted past per-row branches.
#pragma unroll
  for (int lr = 0; lr < TR; ++lr) {
    const int l = min(t * TR + lr, LT - 1);
    const float se = tiled_row_se<LT, TPT, MODE>(A, ip, active, lds, sOwn, lconst, l, lr, mn);
    const float next = obj_add(acc, se, mn);
    acc = lr < rows ? next : acc;
    // the gathers of rows lr + 1 .. lr + 4 wait for the sum up to this row
    // (four rows in flight; one, two, three, six and eight measured slower):
    // without this the compiler hoists every row's loads to the top of the
    // tile and spills
    if (lr % 4 == 3) {
#pragma unroll
      for (int j = 0; j < LT; ++j) asm volatile("" : "+v"(A[j]) : "v"(acc));
    }
  }
  return acc;
}

// The SE terms of the BS rows of tile T >= 1 (already in LDS) into
// hold[l - TR], to be added after tile 0's.
template <int LT, int TPT, int MODE, int TR, int T>
__device__ __forceinline__ void tiled_terms(uint32_t (&A)[LT], const uint8_t *ip, bool active,
                                            const float *sT, const float *sOwn,
                                            const float *__restrict__ lconst,
                                            float (&hold)[LT - TR], int mn) {
  static_assert(T >= 1 && T * TR < LT, "tile T holds BS rows past tile 0");
  constexpr int rows = (T + 1) * TR <= LT ? TR : LT - T * TR;
  const char *lds = reinterpret_cast<const char *>(sT);
#pragma unroll
  for (int lr = 0; lr < rows; ++lr) {
    const int l = T * TR + lr;
    const float se = tiled_row_se<LT, TPT, MODE>(A, ip, active, lds, sOwn, lconst, l, lr, mn);
    hold[l - TR] = se;
    if (lr % 4 == 3) {  // four rows in flight, as in tiled_rows
#pragma unroll
      for (int j = 0; j < LT; ++j) asm volatile("" : "+v"(A[j]) : "v"(se));
    }
  }
}

// Tile t of a round: tile 0 adds to acc, the others fill hold (t is
// dispatched to a compile-time tile index, so hold is indexed statically).
template <int LT, int TPT, int MODE, int TR, int T>
__device__ __forceinline__ void tiled_visit(int t, uint32_t (&A)[LT], const uint8_t *ip,
                                            bool active, const float *sT, const float *sOwn,
                                            const float *__restrict__ lconst, float &acc,
                                            float (&hold)[LT - TR], int mn) {
  constexpr int NT = (LT + TR - 1) / TR;
  if (t == T) {
    if constexpr (T == 0)
      acc = tiled_rows<LT, TPT, MODE, TR>(A, ip, active, sT, sOwn, lconst, 0, acc, mn);
    else
      tiled_terms<LT, TPT, MODE, TR, T>(A, ip, active, sT, sOwn, lconst, hold, mn);
  }
  if constexpr (T + 1 < NT)
    tiled_visit<LT, TPT, MODE, TR, T + 1>(t, A, ip, active, sT, sOwn, lconst, acc, hold, mn);
}

// The whole sum for one round.  `held` is the tile a previous round left in
// LDS (-1: none).  When it is the last tile the tiles are visited in
// decreasing order, otherwise in increasing order, so that a run of rounds
// loads NT - 1 tiles per round instead of NT; in either order tile 0's terms
// are summed into acc and the others' held in registers and added after, in
// increasing l: the canonical order, whatever the visiting order.  Updates
// `held`.  Every thread of the workgroup must call it (inactive lanes too).
template <int LT, int TPT, int MODE, int TR>
__device__ __forceinline__ float lane_sum_tiled(const uint8_t *ip, bool active, float *sT,
                                                const float *sOwn, const float *__restrict__ T2z,
                                                const float *__restrict__ T1,
                                                const float *__restrict__ lconst, int &held,
                                                int mn = 0) {
  constexpr int NT = (LT + TR - 1) / TR;
  static_assert(NT >= 2, "tiled sums hold more than one tile");
  uint32_t A[LT];
  tiled_offsets<LT, TPT, MODE, TR>(ip, active, A);
  float acc = obj_init(mn);
  float hold[LT - TR];
  const bool down = held == NT - 1;
#pragma unroll 1
  for (int v = 0; v < NT; ++v) {
    const int t = down ? NT - 1 - v : v;
    if (v != 0 || held != t) {
      __syncthreads();
      const int rows = (t + 1) * TR <= LT ? TR : LT - t * TR;
      load_tile<MODE>(T2z, T1, LT, TPT, t * TR, rows, TR, sT);
      __syncthreads();
    }
    tiled_visit<LT, TPT, MODE, TR, 0>(t, A, ip, active, sT, sOwn, lconst, acc, hold, mn);
  }
#pragma unroll
  for (int l = TR; l < LT; ++l) acc = obj_add(acc, hold[l - TR], mn);
  held = down ? 0 : NT - 1;
  return acc;
}

// Global-to-LDS copy without registers (global_load_lds): one wave
// instruction moves 64 x SIZE bytes from per-lane global addresses into LDS at
// a wave-uniform base + lane x SIZE (lanes switched off write nothing).  The
// data is in LDS once the wave's vector-memory counter has drained.
template <int SIZE>
__device__ __forceinline__ void lds_dma(const void *gsrc, void *lds_base) {
  static_assert(SIZE == 4 || SIZE == 16, "4 or 16 bytes per lane");
  const auto g = (const __attribute__((address_space(1))) void *)gsrc;
  const auto l = (__attribute__((address_space(3))) void *)lds_base;
  if constexpr (SIZE == 16)
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
}
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// BS rows [r0, r0 + TR) of the zero-diagonal table (and T1) into the tile
// layout T[j][lr][..] of load_tile, by global_load_lds, 16 bytes per lane
// (a row past the table's last is read clamped and lands in tile rows that are
// never used).  Issues only: wait_vmem() and a barrier publish the tile.
template <int LT, int TPT, int MODE, int TR>
__device__ __forceinline__ void dma_tile(const float *__restrict__ T2z,
                                         const float *__restrict__ T1, int r0, float *sT) {
  constexpr int HALF = TPT * 4;                      // one table row (bytes)
  constexpr int ROWB = HALF * (MODE == 1 ? 2 : 1);   // one tile row
  constexpr int CELLB = TR * ROWB;
  constexpr int TOTAL = LT * CELLB;
  constexpr int CHUNKS = (TOTAL + 1023) / 1024;
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int nw = (int)(blockDim.x >> 6);
  char *base = reinterpret_cast<char *>(sT);
  for (int k = wave; k < CHUNKS; k += nw) {
    const int o = k * 1024 + lane * 16;
    if (o < TOTAL) {
      const int j = o / CELLB, rem = o - j * CELLB;
      const int lr = rem / ROWB, pb = rem - lr * ROWB;
      const int l = min(r0 + lr, LT - 1);
      const float *tab = (MODE == 1 && pb >= HALF) ? T1 : T2z;
      const int off = (MODE == 1 && pb >= HALF) ? pb - HALF : pb;
      const char *src = reinterpret_cast<const char *>(tab) + ((size_t)(j * LT + l) * TPT) * 4 + off;
      lds_dma<16>(src, base + __builtin_amdgcn_readfirstlane(k) * 1024);
    }
  }
}

// lane_sum_tiled whose last visit's tile comes in by dma_tile, with hooks:
// hook.before_load() runs before the barrier that precedes that load (all
// threads), hook.issue() after it and before the tile's loads are issued (its
// own global_load_lds traffic is then in flight with the tile's); the barrier
// after the tile waits for both.  Same sum, same bits as lane_sum_tiled.
template <int LT, int TPT, int MODE, int TR, class Hook>
__device__ __forceinline__ float lane_sum_tiled_hook(const uint8_t *ip, bool active, float *sT,
                                                     const float *sOwn,
                                                     const float *__restrict__ T2z,
                                                     const float *__restrict__ T1,
                                                     const float *__restrict__ lconst, int &held,
                                                     int mn, Hook &hook) {
  constexpr int NT = (LT + TR - 1) / TR;
  static_assert(NT >= 2, "tiled sums hold more than one tile");
  uint32_t A[LT];
  tiled_offsets<LT, TPT, MODE, TR>(ip, active, A);
  float acc = obj_init(mn);
  float hold[LT - TR];
  const bool down = held == NT - 1;
#pragma unroll 1
  for (int v = 0; v < NT; ++v) {
    const int t = down ? NT - 1 - v : v;
    if (v != 0 || held != t) {
      const bool last = v == NT - 1;
      if (last) hook.before_load();
      __syncthreads();
      if (last) hook.issue();
      dma_tile<LT, TPT, MODE, TR>(T2z, T1, t * TR, sT);
      wait_vmem();
      __syncthreads();
    }
    tiled_visit<LT, TPT, MODE, TR, 0>(t, A, ip, active, sT, sOwn, lconst, acc, hold, mn);
  }
#pragma unroll
  for (int l = TR; l < LT; ++l) acc = obj_add(acc, hold[l - TR], mn);
  held = down ? 0 : NT - 1;
  return acc;
}

// No work around the tile loads.
struct NoTileHook {
  __device__ __forceinline__ void before_load() {}
  __device__ __forceinline__ void issue() {}
};

// Copies the own-cell squares T2[l][l][.] of every BS row into LDS as
// sOwn[l][p] (L x TP floats).
__device__ __forceinline__ void load_own(const float *__restrict__ Town, int L, int TP, float *sOwn) {
  for (int i = threadIdx.x; i < L * TP; i += blockDim.x) sOwn[i] = gp(Town)[i];
}

template <int LMAX, int MODE>
__device__ __forceinline__ float lane_sum_generic(const uint8_t *ip, bool active, int L, int TP,
                                                  int TR, float *sT,
                                                  const float *__restrict__ T2,
                                                  const float *__restrict__ T1,
                                                  const float *__restrict__ lconst,
                                                  int mn = 0) {
  const int NT = (L + TR - 1) / TR;
  const int ROWB = TP * 4 * (MODE == 1 ? 2 : 1);
  const int CELLB = TR * ROWB;
  const char *lds = reinterpret_cast<const char *>(sT);
  uint32_t A[LMAX];
#pragma unroll
  for (int j = 0; j < LMAX; ++j) A[j] = ip[j < L ? j : 0];
#pragma unroll
  for (int j = 0; j < LMAX; ++j) {
    const uint32_t v = (active && j < L) ? A[j] : 0u;
    A[j] = (uint32_t)(j * CELLB) + (v & (uint32_t)(TP - 1)) * 4u;
  }
  float acc = obj_init(mn);
  for (int t = 0; t < NT; ++t) {
    const int l0 = t * TR;
    const int rows = min(TR, L - l0);
    if (NT > 1) {
      __syncthreads();
      load_tile<MODE>(T2, T1, L, TP, l0, rows, TR, sT);
      __syncthreads();
    }
    for (int lr = 0; lr < rows; ++lr) {
      const int l = l0 + lr;
      float a_l = 0.0f, c2_l = 0.0f;
      if (MODE == 1) {
        a_l = gp(lconst)[2 * l];
        c2_l = gp(lconst)[2 * l + 1];
      }
      acc = obj_add(acc,
                    row_term_generic<LMAX, MODE>(lds, A, (uint32_t)(lr * ROWB),
                                                 (uint32_t)TP * 4u, L, l, a_l, c2_l, mn),
                    mn);
    }
  }
  return acc;
}

// Per-chromosome pairwise tree over pilots of the lanes' sums, then * prelog:
// fit_out[c] for c < nc.  Called by every thread; ends with a barrier.
template <int S>
__device__ __forceinline__ float add_from_lane_plus(float v, int mn) {
  // v (+ or min) the value of lane + S in the same row of 16 lanes; DPP row_shl:S
  const int o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + S, 0xF, 0xF, false);
  return obj_add(v, __int_as_float(o), mn);
}

// reduce_round writing each chromosome's value through out(c, v) (LDS or
// global); same tree, same bits.
template <class Out>
__device__ __forceinline__ void reduce_round_to(float *sE, float acc, bool active, int nc, int K,
                                                float prelog, Out &&out, int mn = 0,
                                                bool sync = true) {
  // pairwise tree over the K pilot sums of a chromosome, one lane per pilot:
  // for s = P/2, P/4, .., 1 (P = K rounded up to a power of two) lane p < s
  // adds lane p + s when p + s < K; the result is in lane 0.
  const int q = threadIdx.x;
  const int c = q / K, p = q - c * K;
  float v = acc;
  if (K <= 32 && (K & (K - 1)) == 0) {
    // a chromosome's lanes lie inside one DPP row (K <= 16) or one aligned
    // group of 32 lanes (K = 32): the tree in registers; the stride-16 step
    // reads lane p ^ 16 (= p + 16 for the lanes p < 16 that keep their sum)
    // with a bit-mask swizzle inside the 32-lane group
    if (K >= 32) {
      const int o = __builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (0x10 << 10));
      v = obj_add(v, __int_as_float(o), mn);
    }
    if (K >= 16) v = add_from_lane_plus<8>(v, mn);
    if (K >= 8) v = add_from_lane_plus<4>(v, mn);
    if (K >= 4) v = add_from_lane_plus<2>(v, mn);
    if (K >= 2) v = add_from_lane_plus<1>(v, mn);
    if (active && p == 0 && c < nc) out(c, mn ? v : prelog * v);  // pre-log: objective 0
    // the caller's next LDS writes follow every lane's reads (sync = false: a
    // caller whose waves share no LDS between rounds)
    if (sync) __syncthreads();
    return;
  }
  // otherwise through LDS, one barrier per stride
  if (active) sE[q] = v;
  int p2 = 1;
  while (p2 < K) p2 <<= 1;
  for (int s = p2 >> 1; s >= 1; s >>= 1) {
    __syncthreads();
    if (active && p < s && p + s < K) {
      v = obj_add(v, sE[q + s], mn);
      sE[q] = v;
    }
  }
  if (active && p == 0 && c < nc) out(c, mn ? v : prelog * v);
  __syncthreads();
}

__device__ __forceinline__ void reduce_round(float *sE, float acc, bool active, int nc, int K,
                                             float prelog, float *fit_out, int mn = 0,
                                             bool sync = true) {
  reduce_round_to(sE, acc, active, nc, K, prelog, [fit_out](int c, float v) { gp(fit_out)[c] = v; },
                  mn, sync);
}

}  // namespace pa
