// k_kmeans.hip -- K-means seed chromosome (Sec. 4.1: users are partitioned
// into spatial clusters; Sec. 1 contribution 2: clustering initialises the
// GA population).
//
// Features: each user's offset from its own BS in integer millimetres
// (llround of 1000 x metres).  k = K clusters.  Start: farthest-point
// (first the user farthest from its BS, then repeatedly the user farthest
// from the chosen centroids; ties to the lowest user).  Then integer Lloyd
// iterations (at most 100): assign to the nearest centroid (ties to the
// lowest cluster), stop when no label changes, else move each non-empty
// centroid to floor((2*sum + n) / (2n)).  Finally, per cell, (user, cluster)
// pairs are taken by increasing (distance, user, cluster) and each free user
// gets a free cluster index as its pilot.  All arithmetic is integer, so the
// order of the (parallel) reductions cannot change the result.
#include "pa_dev.h"
#include "pa_internal.h"

namespace pa {

constexpr int kKmBlock = 1024;
constexpr int kKmWaves = kKmBlock / kWave;

__device__ __forceinline__ int64_t d2(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int64_t dx = ax - bx, dy = ay - by;
  return dx * dx + dy * dy;
}

__device__ __forceinline__ int64_t rdiv_floor(int64_t s, int64_t n) {
  const int64_t num = 2 * s + n, den = 2 * n;
  int64_t q = num / den;
  if ((num % den != 0) && (num < 0)) q -= 1;
  return q;
}

struct KmArgs {
  const double *user_xy;
  const double *bs_xy;
  int L, K;
  uint8_t *seed;
  int32_t *cent_out;
  int32_t *labels_out;
  int32_t *iters_out;
};

__device__ __forceinline__ void kmeans_body(const KmArgs &a) {
  __shared__ int32_t qx[kMaxGenes], qy[kMaxGenes];
  __shared__ int64_t mind[kMaxGenes];
  __shared__ uint8_t lab[kMaxGenes];
  __shared__ int64_t cx[kMaxK], cy[kMaxK];
  __shared__ unsigned long long sx[kMaxK], sy[kMaxK];
  __shared__ int cnt[kMaxK];
  __shared__ uint64_t red[kKmWaves];
  __shared__ int changed;

  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int L = a.L, K = a.K, n = L * K;

  // 1. features
  for (int u = tid; u < n; u += kKmBlock) {
    const int j = u / K;
    const double ox = 1000.0 * (a.user_xy[2 * u] - a.bs_xy[2 * j]);
    const double oy = 1000.0 * (a.user_xy[2 * u + 1] - a.bs_xy[2 * j + 1]);
    qx[u] = (int32_t)llround(ox);
    qy[u] = (int32_t)llround(oy);
    mind[u] = d2(qx[u], qy[u], 0, 0);
    lab[u] = 0xFF;
  }
  __syncthreads();

  // 2. farthest-point start; key = distance << 12 | (4095 - user)
  for (int c = 0; c < K; ++c) {
    uint64_t best = 0;
    for (int u = tid; u < n; u += kKmBlock) {
      const uint64_t key = ((uint64_t)mind[u] << 12) | (uint64_t)(4095 - u);
      best = key > best ? key : best;
    }
    best = wave_max_u64(best);
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (tid == 0) {
      uint64_t b = red[0];
      for (int w = 1; w < kKmWaves; ++w) b = red[w] > b ? red[w] : b;
      const int u = 4095 - (int)(b & 4095u);
      cx[c] = qx[u];
      cy[c] = qy[u];
    }
    __syncthreads();
    for (int u = tid; u < n; u += kKmBlock) {
      const int64_t d = d2(qx[u], qy[u], cx[c], cy[c]);
      mind[u] = (c == 0 || d < mind[u]) ? d : mind[u];
    }
    __syncthreads();
  }

  // 3. Lloyd iterations
  int it = 0;
  for (it = 0; it < 100; ++it) {
    if (tid == 0) changed = 0;
    if (tid < K) {
      sx[tid] = 0;
      sy[tid] = 0;
      cnt[tid] = 0;
    }
    __syncthreads();
    for (int u = tid; u < n; u += kKmBlock) {
      int bc = 0;
      int64_t bd = d2(qx[u], qy[u], cx[0], cy[0]);
      for (int c = 1; c < K; ++c) {
        const int64_t d = d2(qx[u], qy[u], cx[c], cy[c]);
        if (d < bd) {
          bd = d;
          bc = c;
        }
      }
      if ((int)lab[u] != bc) changed = 1;
      lab[u] = (uint8_t)bc;
      atomicAdd(&sx[bc], (unsigned long long)(long long)qx[u]);
      atomicAdd(&sy[bc], (unsigned long long)(long long)qy[u]);
      atomicAdd(&cnt[bc], 1);
    }
    __syncthreads();
    if (!changed) break;
    if (tid < K && cnt[tid] > 0) {
      cx[tid] = rdiv_floor((int64_t)sx[tid], cnt[tid]);
      cy[tid] = rdiv_floor((int64_t)sy[tid], cnt[tid]);
    }
    __syncthreads();
  }

  // 4. per-cell greedy matching, one wave per cell; key = d << 12 | k << 6 | p
  for (int j = wave; j < L; j += kKmWaves) {
    uint64_t user_free = (K == 64) ? ~0ull : ((1ull << K) - 1ull);
    uint64_t pilot_free = user_free;
    for (int step = 0; step < K; ++step) {
      uint64_t best = ~0ull;
      for (int pr = lane; pr < K * K; pr += kWave) {
        const int k = pr / K, p = pr - (pr / K) * K;
        if (((user_free >> k) & 1ull) && ((pilot_free >> p) & 1ull)) {
          const int u = j * K + k;
          const uint64_t key = ((uint64_t)d2(qx[u], qy[u], cx[p], cy[p]) << 12) |
                               ((uint64_t)k << 6) | (uint64_t)p;
          best = key < best ? key : best;
        }
      }
      best = wave_min_u64(best);
      const int k = (int)((best >> 6) & 63u), p = (int)(best & 63u);
      user_free &= ~(1ull << k);
      pilot_free &= ~(1ull << p);
      if (lane == 0) a.seed[j * K + k] = (uint8_t)p;
    }
  }
  if (tid < K) {
    a.cent_out[2 * tid] = (int32_t)cx[tid];
    a.cent_out[2 * tid + 1] = (int32_t)cy[tid];
  }
  for (int u = tid; u < n; u += kKmBlock) a.labels_out[u] = lab[u];
  if (tid == 0) *a.iters_out = it;
}

__global__ __launch_bounds__(kKmBlock) void k_kmeans_seed(KmArgs a) { kmeans_body(a); }

// One workgroup per instance listed in `which`.
__global__ __launch_bounds__(kKmBlock) void k_kmeans_batch(const GenInst *insts,
                                                            const int32_t *which) {
  const GenInst &I = insts[which[blockIdx.x]];
  KmArgs a{I.user_xy, I.bs_xy, I.L, I.K, I.seed, I.km_cent, I.km_labels, I.km_iters};
  kmeans_body(a);
}

hipError_t launch_kmeans_batch(const GenInst *insts, const int32_t *which, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kmeans_batch, dim3(n), dim3(kKmBlock), 0, s, insts, which);
  return hipGetLastError();
}

hipError_t launch_kmeans_seed(const DevProblem &p, hipStream_t s) {
  KmArgs a{p.user_xy, p.bs_xy, p.L, p.K, p.seed, p.km_cent, p.km_labels, p.km_iters};
  hipLaunchKernelGGL(k_kmeans_seed, dim3(1), dim3(kKmBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace pa
