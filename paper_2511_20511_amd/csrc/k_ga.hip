// k_ga.hip -- one GA generation (elitism + selection + crossover + mutation),
// the initial population, and the best chromosome of a population.
//
// Work mapping: one wavefront per task.  Task 0 of a generation copies the
// elites (Sec. 1, contribution 1: the best candidates are preserved); task t
// >= 1 builds the child in slot E + t - 1 in the wave's LDS buffer and writes
// it out.  A workgroup holds kGaWaves waves; all waves meet the same barriers.
#include "ga_core.h"

namespace pa {

constexpr int kGaWaves = 4;
constexpr int kGaBlock = kGaWaves * kWave;

struct GaArgs {
  const uint8_t *pin;
  const float *fin;
  uint8_t *pout;
  float *fout;   // may be null: receives elites' fitness in slots 0..E-1
  float *trace;  // may be null: trace[gen] = best fitness of the input
  int L, K, N;
  uint32_t gen;
  DevGa ga;
};

__global__ __launch_bounds__(kGaBlock) void k_ga_step(GaArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t sbuf[kGaWaves][kMaxGenes];
  __shared__ int32_t sidx[kGaWaves][kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int task = blockIdx.x * kGaWaves + wave;
  const int L = a.L, K = a.K, N = a.N, E = a.ga.E;
  const int LK = L * K;
  const int ntasks = 1 + (N - E);
  uint8_t *buf = sbuf[wave];

  if (task == 0) {
    // elites in rank order, plus the best fitness for the trace
    const int Ek = E < 64 ? (E > 1 ? E : 1) : 0;
    if (Ek > 0) {
      top_e_wave(a.fin, N, Ek, sidx[wave], lane);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (a.trace && lane == 0) a.trace[a.gen] = a.fin[sidx[wave][0]];
      for (int e = 0; e < E; ++e) {
        const int src = sidx[wave][e];
        for (int i = lane; i < LK; i += kWave) a.pout[(size_t)e * LK + i] = a.pin[(size_t)src * LK + i];
        if (a.fout && lane == 0) a.fout[e] = a.fin[src];
      }
    } else {
      // E >= 64: every lane ranks its chromosomes by counting who beats them
      for (int i = lane; i < N; i += kWave) {
        const int r = rank_of(a.fin, N, i);
        if (r == 0 && a.trace) a.trace[a.gen] = a.fin[i];
        if (r < E) {
          for (int g = 0; g < LK; ++g) a.pout[(size_t)r * LK + g] = a.pin[(size_t)i * LK + g];
          if (a.fout) a.fout[r] = a.fin[i];
        }
      }
    }
  }
  const bool child = task >= 1 && task < ntasks;
  const int s = E + task - 1;
  if (child) {
    const int pair_a = E + ((s - E) & ~1);
    const bool second = ((s - E) & 1) != 0;
    const Pairing pr = select_parents(a.fin, N, L, a.ga, a.gen, pair_a, lane);
    const uint8_t *first = a.pin + (size_t)(second ? pr.p2 : pr.p1) * LK;
    const uint8_t *rest = a.pin + (size_t)(second ? pr.p1 : pr.p2) * LK;
    const int cutg = pr.cut * K;
    for (int i = lane; i < LK; i += kWave) buf[i] = i < cutg ? first[i] : rest[i];
  }
  __syncthreads();
  if (child) {
    const Stream dec{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)s, a.gen, a.ga.instance_id, kTagMutDecide};
    const Stream par{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)s, a.gen, a.ga.instance_id, kTagMutPartner};
    mutate_rows(buf, L, K, dec, par, a.ga.thr_mut, lane);
  }
  __syncthreads();
  if (child)
    for (int i = lane; i < LK; i += kWave) a.pout[(size_t)s * LK + i] = buf[i];
}

struct InitArgs {
  const uint8_t *seed;  // may be null when n_km == 0
  uint8_t *pop;
  int L, K, N;
  DevGa ga;
};

__global__ __launch_bounds__(kGaBlock) void k_init_pop(InitArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t sbuf[kGaWaves][kMaxGenes];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int n = blockIdx.x * kGaWaves + wave;
  const int L = a.L, K = a.K, LK = L * K;
  uint8_t *buf = sbuf[wave];
  const bool active = n < a.N;
  const bool from_seed = active && n < a.ga.n_km;
  if (from_seed)
    for (int i = lane; i < LK; i += kWave) buf[i] = a.seed[i];
  __syncthreads();
  if (active) {
    if (from_seed) {
      if (n >= 1) {
        const Stream dec{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration,
                         a.ga.instance_id, kTagInitDecide};
        const Stream par{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration,
                         a.ga.instance_id, kTagInitPartner};
        mutate_rows(buf, L, K, dec, par, a.ga.thr_init, lane);
      }
    } else {
      const Stream shf{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration,
                       a.ga.instance_id, kTagInitShuffle};
      shuffle_rows(buf, L, K, shf, lane);
    }
  }
  __syncthreads();
  if (active)
    for (int i = lane; i < LK; i += kWave) a.pop[(size_t)n * LK + i] = buf[i];
}

__global__ __launch_bounds__(kWave) void k_best(const float *__restrict__ fit, int N,
                                                int32_t *best_idx, float *best_fit) {
  __shared__ int32_t idx[1];
  top_e_wave(fit, N, 1, idx, threadIdx.x);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (threadIdx.x == 0) {
    *best_idx = idx[0];
    *best_fit = fit[idx[0]];
  }
}

hipError_t launch_ga_step(const DevProblem &p, const DevGa &ga, uint32_t gen, const uint8_t *pin,
                          const float *fin, uint8_t *pout, float *fit_out, float *trace,
                          hipStream_t s) {
  GaArgs a{pin, fin, pout, fit_out, trace, p.L, p.K, ga.N, gen, ga};
  const int ntasks = 1 + (ga.N - ga.E);
  const int grid = (ntasks + kGaWaves - 1) / kGaWaves;
  hipLaunchKernelGGL(k_ga_step, dim3(grid), dim3(kGaBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_pop(const DevProblem &p, const DevGa &ga, uint8_t *pop, hipStream_t s) {
  InitArgs a{p.seed, pop, p.L, p.K, ga.N, ga};
  const int grid = (ga.N + kGaWaves - 1) / kGaWaves;
  hipLaunchKernelGGL(k_init_pop, dim3(grid), dim3(kGaBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_best(const float *fit, int N, int32_t *best_idx, float *best_fit,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_best, dim3(1), dim3(kWave), 0, s, fit, N, best_idx, best_fit);
  return hipGetLastError();
}

}  // namespace pa
