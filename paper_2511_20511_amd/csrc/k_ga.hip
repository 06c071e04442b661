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
  int cpw;       // children per workgroup
  DevGa ga;
};

// Workgroup 0 copies the elites; workgroup b >= 1 builds the children of
// slots E + (b-1)*cpw ... with the whole workgroup (ga_core.h) and writes them.
// Dynamic LDS: children (cpw*L*K) | mutation codes (cpw*L*K) | 2 ints per child
// | 64 elite indices.
__global__ __launch_bounds__(kGaBlock) void k_ga_step(GaArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int L = a.L, K = a.K, N = a.N, E = a.ga.E;
  const int LK = L * K;
  const int cb = (a.cpw * LK + 15) / 16 * 16;
  uint8_t *sChild = smem;
  uint8_t *sHits = smem + cb;
  int32_t *sSel = reinterpret_cast<int32_t *>(smem + 2 * cb);
  int32_t *sIdx = sSel + 2 * a.cpw;
  if (blockIdx.x == 0) {
    copy_elites_block(a.pin, a.fin, N, E, LK, a.pout, a.fout, a.trace, (int)a.gen, sIdx);
    return;
  }
  const int s0 = E + ((int)blockIdx.x - 1) * a.cpw;
  const int nc = min(a.cpw, N - s0);
  build_children_block(a.pin, a.fin, N, E, L, K, a.ga, a.gen, s0, nc, sChild, sHits, sSel,
                       (int)blockDim.x);
  store_bytes(a.pout + (size_t)s0 * LK, sChild, nc * LK);
}

struct InitArgs {
  const uint8_t *seed;  // may be null when n_km == 0
  uint8_t *pop;
  int L, K, N;
  DevGa ga;
};

// Individual n of the initial population, built by one wave in `buf`.
__device__ __forceinline__ void init_individual(const InitArgs &a, int n, uint8_t *buf, int lane) {
  const int L = a.L, K = a.K, LK = L * K;
  if (n < a.ga.n_km) {
    for (int i = lane; i < LK; i += kWave) buf[i] = a.seed[i];
    wave_sync();
    if (n >= 1) {
      const Stream dec{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration,
                       a.ga.instance_id, kTagInitDecide};
      const Stream par{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration,
                       a.ga.instance_id, kTagInitPartner};
      mutate_rows(buf, L, K, dec, par, a.ga.thr_init, lane);
    }
  } else {
    const Stream shf{a.ga.seed_lo, a.ga.seed_hi, (uint32_t)n, kInitGeneration, a.ga.instance_id,
                     kTagInitShuffle};
    shuffle_rows(buf, L, K, shf, lane);
  }
  wave_sync();
  for (int i = lane; i < LK; i += kWave) a.pop[(size_t)n * LK + i] = buf[i];
}

__global__ __launch_bounds__(kGaBlock) void k_init_pop(InitArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t sbuf[kGaWaves][kMaxGenes];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int n = blockIdx.x * kGaWaves + wave;
  if (n < a.N) init_individual(a, n, sbuf[wave], lane);
}

// blockIdx.y = instance; individuals beyond an instance's N do nothing.
__global__ __launch_bounds__(kGaBlock) void k_init_batch(const GenInst *insts,
                                                          const int32_t *which) {
  __shared__ __attribute__((aligned(16))) uint8_t sbuf[kGaWaves][kMaxGenes];
  const GenInst &I = insts[which ? which[blockIdx.y] : (int)blockIdx.y];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int n = blockIdx.x * kGaWaves + wave;
  if (n < I.N) {
    InitArgs a{I.seed, pop_buf(I, 0), I.L, I.K, I.N, I.ga};
    init_individual(a, n, sbuf[wave], lane);
  }
}

// One wave per instance: best of its final population, which also closes
// its trace.
__global__ __launch_bounds__(kWave) void k_best_batch(const GenInst *insts, int gen,
                                                       const int32_t *which) {
  __shared__ int32_t idx[1];
  const GenInst &I = insts[which ? which[blockIdx.x] : (int)blockIdx.x];
  const int G = gen < 0 ? I.G : (gen < I.G ? gen : I.G);
  const float *fit = fit_buf(I, G & 1);
  top_e_wave(fit, I.N, 1, idx, threadIdx.x);
  wave_sync();
  if (threadIdx.x == 0) {
    *I.best_idx = idx[0];
    *I.best_fit = fit[idx[0]];
    I.trace[G] = fit[idx[0]];
  }
  const int LK = I.L * I.K;
  const uint8_t *src = pop_buf(I, G & 1) + (size_t)idx[0] * LK;
  for (int i = threadIdx.x; i < LK; i += kWave) I.best_out[i] = src[i];
}

hipError_t launch_init_batch(const GenInst *insts, int ninst, int maxN, hipStream_t s,
                             const int32_t *which) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_batch, dim3((maxN + kGaWaves - 1) / kGaWaves, ninst), dim3(kGaBlock),
                     0, s, insts, which);
  return hipGetLastError();
}

hipError_t launch_best_batch(const GenInst *insts, int ninst, int gen, hipStream_t s,
                             const int32_t *which) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best_batch, dim3(ninst), dim3(kWave), 0, s, insts, gen, which);
  return hipGetLastError();
}

__global__ __launch_bounds__(kWave) void k_best(const float *__restrict__ fit, int N,
                                                int32_t *best_idx, float *best_fit) {
  __shared__ int32_t idx[1];
  top_e_wave(fit, N, 1, idx, threadIdx.x);
  wave_sync();
  if (threadIdx.x == 0) {
    *best_idx = idx[0];
    *best_fit = fit[idx[0]];
  }
}

hipError_t launch_ga_step(const DevProblem &p, const DevGa &ga, uint32_t gen, const uint8_t *pin,
                          const float *fin, uint8_t *pout, float *fit_out, float *trace,
                          hipStream_t s) {
  const int LK = p.L * p.K;
  const int nchild = ga.N - ga.E;
  // enough workgroups to spread the children (and their Philox work) over the
  // GPU, at most 24 KiB of children per workgroup
  int cpw = (nchild + 255) / 256;
  const int cap = 24576 / LK;
  cpw = cpw > cap ? cap : cpw;
  cpw = cpw < 1 ? 1 : (cpw > 64 ? 64 : cpw);
  GaArgs a{pin, fin, pout, fit_out, trace, p.L, p.K, ga.N, gen, cpw, ga};
  const int grid = 1 + (nchild + cpw - 1) / cpw;
  const int cb = (cpw * LK + 15) / 16 * 16;
  const size_t lds = 2 * (size_t)cb + 8 * (size_t)cpw + 256;
  hipLaunchKernelGGL(k_ga_step, dim3(grid), dim3(kGaBlock), lds, s, a);
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
