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

__device__ __forceinline__ float se_asym(float b2, float I) {
  const float r = __builtin_amdgcn_rcpf(I);
  return __builtin_amdgcn_logf(__builtin_fmaf(b2, r, 1.0f));
}

__device__ __forceinline__ float se_finite(float b2, float I, float S, float a, float c2) {
  const float t = __builtin_fmaf(a, S, 1.0f);
  const float den = __builtin_fmaf(c2, t, I);
  const float r = __builtin_amdgcn_rcpf(den);
  return __builtin_amdgcn_logf(__builtin_fmaf(b2, r, 1.0f));
}

// In-place pairwise tree of seg[0..K) (result in seg[0]).
__device__ __forceinline__ void tree_sum(float *seg, int K) {
  int p2 = 1;
  while (p2 < K) p2 <<= 1;
  for (int s = p2 >> 1; s >= 1; s >>= 1)
    for (int p = 0; p < s; ++p)
      if (p + s < K) seg[p] = seg[p] + seg[p + s];
}

// Inverse rows of the chromosomes of a round, stored pilot-major:
// inv[c][s][j] = the user of cell j that sends pilot s in chromosome c, so a
// lane (c, s) finds its L entries contiguous.  Gene g of the round is
// (c, j, k) with g = (c*L + j)*K + k.  Pilots >= K (invalid input) are skipped
// so the LDS write stays inside the chromosome.
__device__ __forceinline__ void build_inverse(const uint8_t *__restrict__ src, int ngenes, int L,
                                              int K, uint8_t *sInv) {
  for (int g = threadIdx.x; g < ngenes; g += blockDim.x) {
    const int cj = g / K, k = g - cj * K;
    const int c = cj / L, j = cj - c * L;
    const int s = src[g];
    if (s < K) sInv[(c * K + s) * L + j] = (uint8_t)k;
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
                                                float a_l, float c2_l) {
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
    return se_finite(b2, I, S, a_l, c2_l);
  } else {
    return se_asym(b2, I);
  }
}

// Same for a runtime L <= LMAX.
template <int LMAX, int MODE>
__device__ __forceinline__ float row_term_generic(const char *lds, const uint32_t (&A)[LMAX],
                                                  uint32_t off, uint32_t t1_bytes, int L, int l,
                                                  float a_l, float c2_l) {
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
  if constexpr (MODE == 1) return se_finite(b2, I, S, a_l, c2_l);
  return se_asym(b2, I);
}

// Copies BS rows [r0, r0 + rows) of the cell-major tables T2[j][l][TP]
// (and T1) into the LDS tile T[j][lr][..] with rows_alloc rows per cell.
template <int MODE>
__device__ __forceinline__ void load_tile(const float *__restrict__ T2, const float *__restrict__ T1,
                                          int L, int TP, int r0, int rows, int rows_alloc,
                                          float *dst) {
  const int q = TP >> 2;                 // float4 per table row
  const int per_cell = rows * q;
  const float4 *s2 = reinterpret_cast<const float4 *>(T2);
  const float4 *s1 = reinterpret_cast<const float4 *>(T1);
  float4 *d = reinterpret_cast<float4 *>(dst);
  for (int i = threadIdx.x; i < L * per_cell; i += blockDim.x) {
    const int j = i / per_cell, rem = i - j * per_cell;
    const int lr = rem / q, c = rem - lr * q;
    const size_t src = ((size_t)j * L + r0 + lr) * q + c;
    if constexpr (MODE == 0) {
      d[(j * rows_alloc + lr) * q + c] = s2[src];
    } else {
      d[((j * rows_alloc + lr) * 2) * q + c] = s2[src];
      d[((j * rows_alloc + lr) * 2 + 1) * q + c] = s1[src];
    }
  }
}

}  // namespace pa
