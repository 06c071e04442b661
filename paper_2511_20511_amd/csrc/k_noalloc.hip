// k_noalloc.hip -- pa_solve_noalloc: the solve of pa_solve without any device
// allocation, for callers that cannot allocate (code under graph capture,
// tight serving loops).  Everything the solve needs beyond the instance's
// tables and the caller's outputs -- its descriptor, task lists and the
// double-buffered populations and fitness -- lives in one fixed device array
// per GPU, `scratch`.  A setup kernel writes the descriptor and task lists
// into it from kernel arguments (no host-to-device copy), then the solve runs
// the same kernels as the per-generation form of pa_solve: K-means seeding,
// initial population, initial fitness, one fused generation launch per
// generation, best of the last population.  Same random words, same ranking,
// same bits as pa_solve.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken with hipGetSymbolAddress once per device (from
// pa_context_create, with that device current) and only that address is
// ever passed to kernels.  Every call on a device shares that device's array
// and overwrites it; nothing in it has to start at zero (every byte a solve
// reads was written earlier in the same solve).  Calls that overlap on one
// device race.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "pa_host.h"

namespace pa {

constexpr size_t kNoAllocBytes = size_t(8) << 20;  // 8 MiB per device
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::once_flag g_once[kNoAllocDevices];
void *g_ptr[kNoAllocDevices];
hipError_t g_err[kNoAllocDevices];

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Descriptor and task lists of one instance, written by one workgroup: the
// elite task then child tasks of cpr children (generation launches), and
// tasks of cpr chromosomes covering the population (initial fitness).
__global__ __launch_bounds__(256) void k_noalloc_setup(GenInst I, int cpr, GenInst *desc,
                                                       GenTask *tasks, int ntasks,
                                                       GenTask *evals, int nevals,
                                                       int32_t *which) {
  if (threadIdx.x == 0) {
    *desc = I;
    *which = 0;
  }
  for (int t = threadIdx.x; t < ntasks; t += blockDim.x) {
    GenTask k;
    k.inst = 0;
    if (t == 0) {
      k.kind = kTaskElite;
      k.s0 = 0;
      k.s1 = I.E;
    } else {
      k.kind = kTaskChild;
      k.s0 = I.E + (t - 1) * cpr;
      k.s1 = min(I.N, k.s0 + cpr);
    }
    tasks[t] = k;
  }
  for (int t = threadIdx.x; t < nevals; t += blockDim.x) {
    GenTask k;
    k.inst = 0;
    k.kind = kTaskEval;
    k.s0 = t * cpr;
    k.s1 = min(I.N, k.s0 + cpr);
    evals[t] = k;
  }
}

}  // namespace

// Device address of this device's scratch array (hipGetSymbolAddress, once
// per device, with the device current); its error otherwise.
hipError_t noalloc_scratch(int device, void **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
  std::call_once(g_once[device], [device] {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_err[device] = e;
  });
  *ptr = g_ptr[device];
  return g_err[device];
}

}  // namespace pa

using namespace pa;

extern "C" pa_status pa_solve_noalloc(pa_instance *in, const pa_ga_params *g, uint8_t *d_best,
                                      float *d_best_fit, float *d_trace, void *stream) {
  if (!in || !d_best || !d_best_fit) return set_error(PA_EINVAL, "instance or output is NULL");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  if (!in->ctx->scratch)
    return set_error(PA_EDEVICE, "the no-allocation scratch of device %d is unavailable",
                     in->ctx->device);
  const DevProblem &p = in->p;
  const int L = p.L, K = p.K, TP = p.TP, N = g->pop, E = g->elite, G = g->gens;
  GenClass c;
  c.L = L;
  c.TP = TP;
  c.mode = p.se_mode;
  c.block = gen_class_block(L, TP, p.se_mode, K);
  const int cpr = std::max(1, c.block / K);
  const int ntasks = 1 + (N - E + cpr - 1) / cpr;
  const int nevals = (N + cpr - 1) / cpr;
  const size_t LK = (size_t)L * K;
  // scratch layout (256-byte aligned pieces)
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t at = off;
    off += up256(bytes);
    return at;
  };
  const size_t o_desc = take(sizeof(GenInst));
  const size_t o_tasks = take(sizeof(GenTask) * ntasks);
  const size_t o_evals = take(sizeof(GenTask) * nevals);
  const size_t o_which = take(sizeof(int32_t));
  const size_t o_idx = take(sizeof(int32_t));
  const size_t o_trace = d_trace ? 0 : take(sizeof(float) * ((size_t)G + 1));
  const size_t o_fit0 = take(sizeof(float) * N), o_fit1 = take(sizeof(float) * N);
  const size_t o_pop0 = take(LK * N), o_pop1 = take(LK * N);
  if (off > kNoAllocBytes)
    return set_error(PA_EINVAL,
                     "solve needs %zu bytes of scratch (2 N L K + 8 N + tasks), more than the "
                     "%zu of pa_solve_noalloc", off, kNoAllocBytes);
  unsigned char *base = static_cast<unsigned char *>(in->ctx->scratch);
  GenInst I;
  std::memset(&I, 0, sizeof I);
  I.T2 = p.T2;
  I.T1 = p.T1;
  I.T2z = p.T2z;
  I.Town = p.Town;
  I.lconst = p.lconst;
  I.pop[0] = base + o_pop0;
  I.pop[1] = base + o_pop1;
  I.fit[0] = reinterpret_cast<float *>(base + o_fit0);
  I.fit[1] = reinterpret_cast<float *>(base + o_fit1);
  I.trace = d_trace ? d_trace : reinterpret_cast<float *>(base + o_trace);
  I.best_idx = reinterpret_cast<int32_t *>(base + o_idx);
  I.best_fit = d_best_fit;
  I.best_out = d_best;
  I.user_xy = p.user_xy;
  I.bs_xy = p.bs_xy;
  I.seed = p.seed;
  I.km_cent = p.km_cent;
  I.km_labels = p.km_labels;
  I.km_iters = p.km_iters;
  I.L = L;
  I.K = K;
  I.TP = TP;
  I.N = N;
  I.E = E;
  I.G = G;
  I.prelog = p.prelog;
  I.se_mode = p.se_mode;
  I.objective = p.objective;
  I.ga = ga_from_params(g);
  GenInst *d_desc = reinterpret_cast<GenInst *>(base + o_desc);
  GenTask *d_tasks = reinterpret_cast<GenTask *>(base + o_tasks);
  GenTask *d_evals = reinterpret_cast<GenTask *>(base + o_evals);
  int32_t *d_which = reinterpret_cast<int32_t *>(base + o_which);
  c.tasks = d_tasks;
  c.ntasks = ntasks;
  c.eval_tasks = d_evals;
  c.neval = nevals;
  c.grid = gen_class_grid(L, TP, p.se_mode, c.block, ntasks, in->ctx->info.cus);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, s, I, cpr, d_desc, d_tasks, ntasks,
                     d_evals, nevals, d_which);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_kmeans_batch(d_desc, d_which, I.ga.n_km > 0 ? 1 : 0, s);
  if (e == hipSuccess) e = launch_init_batch(d_desc, 1, N, s);
  if (e == hipSuccess) e = launch_gen(d_desc, c, -1, in->ctx->info, s);
  for (int gen = 0; gen < G && e == hipSuccess; ++gen)
    e = launch_gen(d_desc, c, gen, in->ctx->info, s);
  if (e == hipSuccess) e = launch_best_batch(d_desc, 1, -1, s);
  if (e != hipSuccess) return hip_error(e, "pa_solve_noalloc");
  return PA_OK;
}
