// pa_internal.h -- structures shared by the host runtime (api.cpp) and the
// kernel launchers (k_*.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "pa_dev.h"

namespace pa {

// A kernel's dynamic-LDS limit is raised once per kernel, by whichever
// thread launches it first (std::call_once: the server's worker and caller
// threads may race to the first launch); later launches reuse the outcome.
struct LdsAttr {
  std::once_flag once;
  hipError_t err = hipSuccess;
};
inline hipError_t allow_lds_once(LdsAttr &a, const void *kern, int bytes) {
  std::call_once(a.once, [&] {
    a.err = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (a.err != hipSuccess) (void)hipGetLastError();  // not sticky: reported with the launch
  });
  return a.err;
}
// Status of a launch made after allow_lds_once returned attr_err: the launch's
// own error, or, when the launch failed and raising the limit had failed
// too, that earlier failure (the likely cause).
inline hipError_t launch_status(hipError_t attr_err) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess && attr_err != hipSuccess) return attr_err;
  return e;
}

constexpr int kMaxL = 64;
constexpr int kMaxK = 64;
constexpr int kMaxGenes = kMaxL * kMaxK;  // 4096 genes per chromosome

// Table row padding: the pilot axis of the FP32 tables is padded to 4, 8, 16,
// 32 or 64 entries so a BS row has a compile-time stride in the kernels.
inline int pad_pilots(int K) {
  int p = 4;
  while (p < K) p <<= 1;
  return p;
}

// Device copy of one problem.  All pointers are device memory owned by the
// instance.
struct DevProblem {
  int L = 0, K = 0, TP = 0;  // cells, users (= pilots), padded pilot stride
  int se_mode = 0;
  int objective = 0;         // 0: sum of the SE terms, 1: their minimum, 2: Eq. 8
  float prelog = 1.0f;       // 1 - tau/T, or 1
  double *beta = nullptr;    // [L][L][K] FP64 as given
  float *T2 = nullptr;       // [L(cell j)][L(BS l)][TP] normalised beta squared (FP32)
  float *T1 = nullptr;       // same layout, normalised beta (finite-M only)
  float *T2z = nullptr;      // T2 with the own-cell entries (j == l) zeroed
  float *Town = nullptr;     // [L(BS l)][TP] own-cell squares T2[l][l][.]
  float *lconst = nullptr;   // [L][2]: tau*rho_l and (1 + rho_l*B_l)/(M tau rho_l^2)
  double *user_xy = nullptr; // [L][K][2] or null
  double *bs_xy = nullptr;   // [L][2] or null
  uint8_t *seed = nullptr;   // [L][K] K-means seed chromosome
  int32_t *km_cent = nullptr;   // [K][2]
  int32_t *km_labels = nullptr; // [L*K]
  int32_t *km_iters = nullptr;  // [1]
};

// GA parameters as the kernels need them (thresholds already computed).
struct DevGa {
  int N = 0, E = 0, n_km = 0;
  uint64_t thr_cross = 0, thr_mut = 0, thr_init = 0;
  uint32_t seed_lo = 0, seed_hi = 0, instance_id = 0;
};

// Launch-shape knobs of the fitness kernel (never change result bits).
struct FitShape {
  int block = 256;  // threads per workgroup
  int grid = 0;     // 0 = one workgroup per round of chromosomes (capped)
};

struct DeviceInfo {
  int cus = 256;
  size_t lds_per_block = 163840;
};

// One instance as the batched kernels see it (an array of these lives in
// device memory).  Populations and fitness are double-buffered: generation g
// reads buffer g & 1 and writes buffer 1 - (g & 1); the initial population
// and its fitness live in buffer 0.
struct GenInst {
  const float *T2, *T1, *lconst, *T2z, *Town;
  uint8_t *pop[2];
  float *fit[2];
  float *trace;        // [G + 1]
  int32_t *best_idx;   // [1]
  float *best_fit;     // [1]
  uint8_t *best_out;   // [L*K]: copy of the best chromosome of the final population
  const double *user_xy, *bs_xy;
  uint8_t *seed;
  int32_t *km_cent, *km_labels, *km_iters;
  int L, K, TP, N, E, G;
  float prelog;
  int se_mode;
  int objective;
  DevGa ga;
};


// A descriptor read with scalar loads (the constant address space: nothing
// writes descriptors while a kernel that reads them runs), so that its fields
// live in scalar registers; i must be wave-uniform.
__device__ __forceinline__ GenInst load_inst(const GenInst *insts, int i) {
  static_assert(sizeof(GenInst) % 4 == 0, "descriptor of whole words");
  typedef __attribute__((address_space(4))) const uint32_t *cwords;
  const cwords src = (cwords)reinterpret_cast<const uint32_t *>(insts + __builtin_amdgcn_readfirstlane(i));
  GenInst I;
  uint32_t *dst = reinterpret_cast<uint32_t *>(&I);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(GenInst) / 4); ++w) dst[w] = src[w];
  return I;
}

// Buffer b of an instance, by selection (no dynamic index, so a descriptor
// copied into registers stays in registers).
__device__ __forceinline__ uint8_t *pop_buf(const GenInst &I, int b) {
  return b ? I.pop[1] : I.pop[0];
}
__device__ __forceinline__ float *fit_buf(const GenInst &I, int b) {
  return b ? I.fit[1] : I.fit[0];
}

enum : int32_t { kTaskElite = 0, kTaskChild = 1, kTaskEval = 2 };

// A unit of work of one generation launch: the elites of an instance, or the
// children (or, before the first generation, the fitness) of slots [s0, s1).
struct GenTask {
  int32_t inst, kind, s0, s1;
};

// A group of instances sharing (L, TP, SE mode) that one kernel variant runs.
struct GenClass {
  int L = 0, TP = 0, mode = 0;
  int block = 0;                  // threads per workgroup of the generation kernel
  int grid = 0;                   // workgroups
  const GenTask *tasks = nullptr; // device
  int ntasks = 0;
  const GenTask *eval_tasks = nullptr;  // device: initial-population fitness
  int neval = 0;
  // non-null: the launch runs `tasks` with each instance at its own
  // generation gens[inst] (device; -1 = the initial fitness, eval tasks)
  const int32_t *gens = nullptr;
  // non-null (device, grid + 1 entries): the generation launches' runs of
  // `tasks` are [bounds[r], bounds[r + 1]) (cut by task cost) instead of
  // runs of equal task counts; the initial-fitness launch ignores it
  const int32_t *bounds = nullptr;
  // non-null: launch nothing, store how many workgroups of the class's
  // kernel (at `block`) one CU holds at once
  int *query_per_cu = nullptr;
};

// ---- launchers (return hipSuccess or the first HIP error) ----------------
hipError_t launch_prep(const DevProblem &p, int M, double rho, hipStream_t s);
hipError_t launch_fitness(const DevProblem &p, const uint8_t *pop, int n, float *fit,
                          const FitShape &shape, const DeviceInfo &dev, hipStream_t s);
hipError_t launch_kmeans_seed(const DevProblem &p, hipStream_t s);
hipError_t launch_init_pop(const DevProblem &p, const DevGa &ga, uint8_t *pop, hipStream_t s);
// One generation of operators.  fit_out (may be null) receives the elites'
// fitness in slots 0..E-1; trace (may be null) receives the best fitness of
// the input population at index `gen`.
hipError_t launch_ga_step(const DevProblem &p, const DevGa &ga, uint32_t gen, const uint8_t *pin,
                          const float *fin, uint8_t *pout, float *fit_out, float *trace,
                          hipStream_t s);
// Best chromosome of a population: writes best index (int32) and fitness.
hipError_t launch_best(const float *fit, int N, int32_t *best_idx, float *best_fit,
                       hipStream_t s);

// ---- batched, descriptor-driven launchers ------------------------------
// Children per task (= chromosomes per LDS round) of the generation kernel
// for a class, and its workgroup size.
int gen_children_per_task(int L, int K, int TP, int mode, int block);
int gen_default_block(int L, int TP, int mode);
hipError_t launch_kmeans_batch(const GenInst *insts, const int32_t *which, int n, hipStream_t s);
// which (device, may be null = 0..ninst-1): the instances to initialise.
hipError_t launch_init_batch(const GenInst *insts, int ninst, int maxN, hipStream_t s,
                             const int32_t *which = nullptr);
// gen = -1: fitness of the initial populations (the class's eval tasks).
hipError_t launch_gen(const GenInst *insts, const GenClass &c, int gen, const DeviceInfo &dev,
                      hipStream_t s);
// Persistent form: generations [g0, g1) of a class in one launch of `grid`
// co-resident workgroups separated by grid barriers on the counter `bar`
// (zeroed before the launch); a barrier wait that times out sets *err.  With
// best != 0 it ends with the best of each of the first `ninst` instances.
struct PersistLaunch {
  int g0, g1, best, ninst, grid;
  uint32_t *bar;
  int32_t *err;
};
// capacity != null: only stores the largest co-resident grid of the class's
// persistent kernel (0 when the class has none) and launches nothing.
hipError_t launch_gen_persist(const GenInst *insts, const GenClass &c, const PersistLaunch &pl,
                              const DeviceInfo &dev, int *capacity, hipStream_t s);
// One-workgroup form: generations [g0, g1) of ninst instances of one class
// (L, TP, mode), one workgroup of `block` threads each, with the population,
// its fitness and the table in LDS (g0 = -1: from the initial population; with
// best, the result at each instance's last generation).  lds_out != null: only
// the LDS bytes for the largest instance (maxN, maxK) into *lds_out, or
// hipErrorInvalidValue when no such kernel variant exists.
hipError_t launch_gen_wg(const GenInst *d_insts, int ninst, int L, int TP, int mode, int block,
                         int g0, int g1, bool best, int maxN, int maxK, int *lds_out,
                         hipStream_t s);
// Most elites the one-workgroup form ranks (one wave).
int wg_max_elites();
// Best of each instance's population after generation `gen` (or after its
// last generation when gen < 0); closes the trace at that generation.
hipError_t launch_best_batch(const GenInst *insts, int ninst, int gen, hipStream_t s,
                             const int32_t *which = nullptr);

}  // namespace pa
