// api.cpp -- host runtime behind include/pa.h: argument validation, device
// buffers of contexts and instances, and the solve loops.  Every step of the
// method runs in the kernels of k_*.hip; this file only checks, allocates,
// copies and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_host.h"

using namespace pa;

namespace {

thread_local std::string g_err;

pa_status fail(pa_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

pa_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? PA_ENOMEM : PA_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

#define HIP_TRY(call, what)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

uint64_t threshold(double p) {
  if (p >= 1.0) return 1ull << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

bool prob_ok(double p) { return p >= 0.0 && p <= 1.0; }

pa_status validate_problem(const pa_problem *pr) {
  if (!pr) return fail(PA_EINVAL, "problem is NULL");
  if (pr->L < 1 || pr->L > kMaxL) return fail(PA_EINVAL, "L=%d outside [1, %d]", pr->L, kMaxL);
  if (pr->K < 1 || pr->K > kMaxK) return fail(PA_EINVAL, "K=%d outside [1, %d]", pr->K, kMaxK);
  if (pr->tau != pr->K) return fail(PA_EINVAL, "tau=%d must equal K=%d", pr->tau, pr->K);
  if (pr->T != 0 && pr->T <= pr->tau)
    return fail(PA_EINVAL, "coherence length T=%d must be 0 or > tau=%d", pr->T, pr->tau);
  if (pr->T < 0) return fail(PA_EINVAL, "T=%d is negative", pr->T);
  if (pr->se_mode != PA_SE_ASYMPTOTIC && pr->se_mode != PA_SE_FINITE_M)
    return fail(PA_EINVAL, "unknown se_mode %d", pr->se_mode);
  if (pr->objective != PA_OBJ_SUM_SE && pr->objective != PA_OBJ_MIN_SINR &&
      pr->objective != PA_OBJ_INTERCLUSTER)
    return fail(PA_EINVAL, "unknown objective %d", pr->objective);
  if (pr->objective == PA_OBJ_INTERCLUSTER && pr->se_mode != PA_SE_ASYMPTOTIC)
    return fail(PA_EINVAL, "the Eq. 8 objective has no finite-M form (se_mode must be asymptotic)");
  const bool asym = pr->se_mode == PA_SE_ASYMPTOTIC;
  if (asym && pr->L < 2)
    return fail(PA_EINVAL, "asymptotic SE needs L >= 2 (one cell has no interference)");
  if (!asym) {
    if (pr->M < 1) return fail(PA_EINVAL, "M=%d must be >= 1", pr->M);
    if (!(pr->rho > 0.0) || !std::isfinite(pr->rho))
      return fail(PA_EINVAL, "rho must be finite and > 0");
  }
  if (!pr->beta) return fail(PA_EINVAL, "beta is NULL");
  const int L = pr->L, K = pr->K;
  for (int l = 0; l < L; ++l) {
    double mx = 0.0, mn = INFINITY;
    for (int i = 0; i < L * K; ++i) {
      const double b = pr->beta[(size_t)l * L * K + i];
      if (!std::isfinite(b)) return fail(PA_EINVAL, "beta[%d][..] has a non-finite entry", l);
      if (asym ? !(b > 0.0) : !(b >= 0.0))
        return fail(PA_EINVAL, "beta[%d][..] has an entry %s 0", l, asym ? "<=" : "<");
      if (b > mx) mx = b;
      if (b > 0.0 && b < mn) mn = b;
    }
    if (mx > 0.0 && mx / mn > 0x1p60)
      return fail(PA_EINVAL, "beta at BS %d spans more than 2^60 (max/min %g)", l, mx / mn);
  }
  if ((pr->user_xy == nullptr) != (pr->bs_xy == nullptr))
    return fail(PA_EINVAL, "user_xy and bs_xy must both be given or both be NULL");
  if (pr->user_xy) {
    for (int j = 0; j < L; ++j) {
      const double bx = pr->bs_xy[2 * j], by = pr->bs_xy[2 * j + 1];
      if (!std::isfinite(bx) || !std::isfinite(by)) return fail(PA_EINVAL, "bs_xy not finite");
      for (int k = 0; k < K; ++k) {
        const double ux = pr->user_xy[2 * (j * K + k)], uy = pr->user_xy[2 * (j * K + k) + 1];
        const double ox = 1000.0 * (ux - bx), oy = 1000.0 * (uy - by);
        if (!(std::fabs(ox) <= 8388608.0) || !(std::fabs(oy) <= 8388608.0))
          return fail(PA_EINVAL, "user (%d,%d) is not within 8388 m of its BS", j, k);
      }
    }
  }
  return PA_OK;
}

pa_status validate_params_pos(bool has_pos, const pa_ga_params *g) {
  if (!g) return fail(PA_EINVAL, "params is NULL");
  if (g->pop < 2 || g->pop > 65536) return fail(PA_EINVAL, "pop=%d outside [2, 65536]", g->pop);
  if (g->gens < 0) return fail(PA_EINVAL, "gens=%d is negative", g->gens);
  if (g->elite < 0 || g->elite > g->pop)
    return fail(PA_EINVAL, "elite=%d outside [0, pop=%d]", g->elite, g->pop);
  if (!prob_ok(g->p_cross) || !prob_ok(g->p_mut) || !prob_ok(g->p_init) ||
      !prob_ok(g->kmeans_frac))
    return fail(PA_EINVAL, "probabilities must lie in [0, 1]");
  if (g->kmeans_frac > 0.0 && !has_pos)
    return fail(PA_EINVAL, "kmeans_frac > 0 needs user and BS positions");
  return PA_OK;
}

pa_status validate_params(const pa_instance *inst, const pa_ga_params *g) {
  return validate_params_pos(inst->has_pos, g);
}

DevGa make_ga(const pa_ga_params *g) {
  DevGa d;
  d.N = g->pop;
  d.E = g->elite;
  d.n_km = 0;
  if (g->kmeans_frac > 0.0) {
    int n = (int)std::floor(g->kmeans_frac * (double)g->pop + 0.5);
    if (n < 1) n = 1;
    if (n > g->pop) n = g->pop;
    d.n_km = n;
  }
  d.thr_cross = threshold(g->p_cross);
  d.thr_mut = threshold(g->p_mut);
  d.thr_init = threshold(g->p_init);
  d.seed_lo = (uint32_t)(g->seed & 0xffffffffu);
  d.seed_hi = (uint32_t)(g->seed >> 32);
  d.instance_id = g->instance_id;
  return d;
}

template <class T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count ? count : 1));
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

pa_status ensure_work_impl(pa_instance *in, int N, int G) {
  const size_t LK = (size_t)in->p.L * in->p.K;
  if (in->work_N < N) {
    dfree(in->popA);
    dfree(in->popB);
    dfree(in->fitA);
    dfree(in->fitB);
    in->popA = in->popB = nullptr;
    in->fitA = in->fitB = nullptr;
    in->work_N = 0;
    HIP_TRY(dalloc(&in->popA, LK * N), "hipMalloc(population)");
    HIP_TRY(dalloc(&in->popB, LK * N), "hipMalloc(population)");
    HIP_TRY(dalloc(&in->fitA, (size_t)N), "hipMalloc(fitness)");
    HIP_TRY(dalloc(&in->fitB, (size_t)N), "hipMalloc(fitness)");
    in->work_N = N;
  }
  if (in->work_G < G) {
    dfree(in->trace);
    in->trace = nullptr;
    in->work_G = -1;
    HIP_TRY(dalloc(&in->trace, (size_t)G + 1), "hipMalloc(trace)");
    in->work_G = G;
  }
  if (!in->best_idx) HIP_TRY(dalloc(&in->best_idx, 1), "hipMalloc(best)");
  if (!in->best_fit) HIP_TRY(dalloc(&in->best_fit, 1), "hipMalloc(best)");
  if (!in->ev0) HIP_TRY(hipEventCreate(&in->ev0), "hipEventCreate");
  if (!in->ev1) HIP_TRY(hipEventCreate(&in->ev1), "hipEventCreate");
  return PA_OK;
}

// Copies the result of a finished solve (population in popA, fitness fitA,
// trace filled up to G-1) to the host.
pa_status finish_solve(pa_instance *in, int N, int G, pa_result *out, hipStream_t s) {
  HIP_TRY(launch_best(in->fitA, N, in->best_idx, in->best_fit, s), "launch best");
  HIP_TRY(hipMemcpyAsync(in->trace + G, in->best_fit, sizeof(float), hipMemcpyDeviceToDevice, s),
          "copy trace");
  HIP_TRY(hipEventRecord(in->ev1, s), "hipEventRecord");
  int32_t bi = 0;
  float bf = 0.0f;
  HIP_TRY(hipMemcpyAsync(&bi, in->best_idx, sizeof bi, hipMemcpyDeviceToHost, s), "copy best");
  HIP_TRY(hipMemcpyAsync(&bf, in->best_fit, sizeof bf, hipMemcpyDeviceToHost, s), "copy best");
  if (out->trace)
    HIP_TRY(hipMemcpyAsync(out->trace, in->trace, sizeof(float) * (G + 1), hipMemcpyDeviceToHost,
                           s),
            "copy trace");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (bi < 0 || bi >= N) return fail(PA_EINTERNAL, "best index %d out of range", bi);
  const size_t LK = (size_t)in->p.L * in->p.K;
  if (out->best)
    HIP_TRY(hipMemcpy(out->best, in->popA + (size_t)bi * LK, LK, hipMemcpyDeviceToHost),
            "copy best chromosome");
  out->best_fit = bf;
  out->best_index = bi;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, in->ev0, in->ev1), "hipEventElapsedTime");
  out->device_ms = ms;
  return PA_OK;
}

pa_status set_device(pa_context *ctx) {
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  return PA_OK;
}

}  // namespace

namespace pa {
pa_status set_error(pa_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
pa_status hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
pa_status validate_ga(const pa_instance *inst, const pa_ga_params *g) {
  return validate_params(inst, g);
}
DevGa ga_from_params(const pa_ga_params *g) { return make_ga(g); }
pa_status ensure_work(pa_instance *in, int N, int G) { return ensure_work_impl(in, N, G); }
pa_status use_device(pa_context *ctx) { return set_device(ctx); }
}  // namespace pa

extern "C" {

const char *pa_version(void) { return "pa-mi355x 0.1 (gfx950)"; }

const char *pa_last_error(void) { return g_err.c_str(); }

const char *pa_status_string(pa_status s) {
  switch (s) {
    case PA_OK: return "ok";
    case PA_EINVAL: return "invalid argument";
    case PA_ENOMEM: return "out of memory";
    case PA_EDEVICE: return "device error";
    case PA_EAGAIN: return "try again";
    case PA_ECANCELED: return "cancelled";
    case PA_EINTERNAL: return "internal error";
    case PA_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

pa_status pa_problem_check(const pa_problem *prob) { return validate_problem(prob); }

pa_status pa_params_check(const pa_problem *prob, const pa_ga_params *params) {
  pa_status st = validate_problem(prob);
  if (st != PA_OK) return st;
  return validate_params_pos(prob->user_xy != nullptr, params);
}

pa_status pa_context_create(int32_t device, pa_context **out) {
  if (!out) return fail(PA_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev)
    return fail(PA_EINVAL, "device %d outside [0, %d)", device, ndev);
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PA_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  pa_context *c = new (std::nothrow) pa_context;
  if (!c) return fail(PA_ENOMEM, "host allocation failed");
  c->device = device;
  c->info.cus = prop.multiProcessorCount;
  c->info.lds_per_block = prop.sharedMemPerBlock;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipStreamCreate");
  }
  // the no-allocation entry point's scratch: a failed lookup only disables
  // that entry point (it then reports PA_EDEVICE)
  if (noalloc_scratch(device, &c->scratch) != hipSuccess) c->scratch = nullptr;
  *out = c;
  return PA_OK;
}

void pa_context_destroy(pa_context *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  free_plan(ctx->batch_plan);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

void pa_instance_destroy(pa_instance *in) {
  if (!in) return;
  (void)hipSetDevice(in->ctx->device);
  free_plan(in->plan);
  if (in->ctx->batch_plan) {  // a batch plan may point at this instance's buffers
    free_plan(in->ctx->batch_plan);
    in->ctx->batch_plan = nullptr;
  }
  DevProblem &p = in->p;
  for (void *ptr : {(void *)p.beta, (void *)p.T2, (void *)p.T1, (void *)p.T2z, (void *)p.Town,
                    (void *)p.lconst,
                    (void *)p.user_xy, (void *)p.bs_xy, (void *)p.seed, (void *)p.km_cent,
                    (void *)p.km_labels, (void *)p.km_iters, (void *)in->popA, (void *)in->popB,
                    (void *)in->fitA, (void *)in->fitB, (void *)in->trace, (void *)in->best_idx,
                    (void *)in->best_fit})
    dfree(ptr);
  if (in->ev0) (void)hipEventDestroy(in->ev0);
  if (in->ev1) (void)hipEventDestroy(in->ev1);
  delete in;
}

pa_status pa_instance_create(pa_context *ctx, const pa_problem *prob, pa_instance **out) {
  if (!ctx || !out) return fail(PA_EINVAL, "context or out is NULL");
  *out = nullptr;
  pa_status st = validate_problem(prob);
  if (st != PA_OK) return st;
  if ((st = set_device(ctx)) != PA_OK) return st;
  pa_instance *in = new (std::nothrow) pa_instance;
  if (!in) return fail(PA_ENOMEM, "host allocation failed");
  in->ctx = ctx;
  in->M = prob->M;
  in->rho = prob->rho;
  in->T = prob->T;
  in->has_pos = prob->user_xy != nullptr;
  DevProblem &p = in->p;
  p.L = prob->L;
  p.K = prob->K;
  p.TP = pad_pilots(prob->K);
  p.se_mode = prob->se_mode;
  p.objective = prob->objective;
  p.prelog = prob->T > 0 ? (float)(1.0 - (double)prob->K / (double)prob->T) : 1.0f;
  const size_t L = p.L, K = p.K, TP = p.TP;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  chk(dalloc(&p.beta, L * L * K));
  chk(dalloc(&p.T2, L * L * TP));
  chk(dalloc(&p.T2z, L * L * TP));
  chk(dalloc(&p.Town, L * TP));
  if (p.se_mode == PA_SE_FINITE_M) chk(dalloc(&p.T1, L * L * TP));
  chk(dalloc(&p.lconst, 2 * L));
  chk(dalloc(&p.seed, L * K));
  chk(dalloc(&p.km_cent, 2 * K));
  chk(dalloc(&p.km_labels, L * K));
  chk(dalloc(&p.km_iters, 1));
  if (in->has_pos) {
    chk(dalloc(&p.user_xy, L * K * 2));
    chk(dalloc(&p.bs_xy, L * 2));
  }
  if (e != hipSuccess) {
    pa_instance_destroy(in);
    return hip_fail(e, "hipMalloc(instance)");
  }
  hipStream_t s = ctx->stream;
  chk(hipMemcpyAsync(p.beta, prob->beta, sizeof(double) * L * L * K, hipMemcpyHostToDevice, s));
  chk(hipMemsetAsync(p.lconst, 0, sizeof(float) * 2 * L, s));
  chk(hipMemsetAsync(p.km_iters, 0, sizeof(int32_t), s));
  if (in->has_pos) {
    chk(hipMemcpyAsync(p.user_xy, prob->user_xy, sizeof(double) * L * K * 2,
                       hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(p.bs_xy, prob->bs_xy, sizeof(double) * L * 2, hipMemcpyHostToDevice, s));
  }
  if (e == hipSuccess) e = launch_prep(p, prob->M, prob->rho, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    pa_instance_destroy(in);
    return hip_fail(e, "instance upload");
  }
  *out = in;
  return PA_OK;
}

pa_status pa_kmeans_init(pa_instance *in, const pa_ga_params *g, uint8_t *d_pop, void *stream) {
  if (!in || !d_pop) return fail(PA_EINVAL, "instance or d_pop is NULL");
  pa_status st = validate_params(in, g);
  if (st != PA_OK) return st;
  if ((st = set_device(in->ctx)) != PA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const DevGa ga = make_ga(g);
  if (ga.n_km > 0) HIP_TRY(launch_kmeans_seed(in->p, s), "launch kmeans");
  HIP_TRY(launch_init_pop(in->p, ga, d_pop, s), "launch init");
  return PA_OK;
}

pa_status pa_fitness(pa_instance *in, const uint8_t *d_pop, int32_t n, float *d_fit,
                     void *stream) {
  if (!in) return fail(PA_EINVAL, "instance is NULL");
  if (n < 0) return fail(PA_EINVAL, "n=%d is negative", n);
  if (n == 0) return PA_OK;
  if (!d_pop || !d_fit) return fail(PA_EINVAL, "d_pop or d_fit is NULL");
  pa_status st = set_device(in->ctx);
  if (st != PA_OK) return st;
  FitShape shape;
  HIP_TRY(launch_fitness(in->p, d_pop, n, d_fit, shape, in->ctx->info, (hipStream_t)stream),
          "launch fitness");
  return PA_OK;
}

pa_status pa_fitness_shaped(pa_instance *in, const uint8_t *d_pop, int32_t n, float *d_fit,
                            int32_t block, int32_t grid_cap, int32_t generic, void *stream) {
  if (!in) return fail(PA_EINVAL, "instance is NULL");
  if (n < 0) return fail(PA_EINVAL, "n=%d is negative", n);
  if (block != 0 && (block < 64 || block > 1024 || block % 64 != 0 || block < in->p.K))
    return fail(PA_EINVAL, "block=%d must be 0 or a multiple of 64 in [max(64,K), 1024]", block);
  if (grid_cap < 0) return fail(PA_EINVAL, "grid_cap=%d is negative", grid_cap);
  if (n == 0) return PA_OK;
  if (!d_pop || !d_fit) return fail(PA_EINVAL, "d_pop or d_fit is NULL");
  pa_status st = set_device(in->ctx);
  if (st != PA_OK) return st;
  FitShape shape;
  shape.block = block;
  shape.grid = generic ? -1 : grid_cap;
  HIP_TRY(launch_fitness(in->p, d_pop, n, d_fit, shape, in->ctx->info, (hipStream_t)stream),
          "launch fitness");
  return PA_OK;
}

pa_status pa_ga_step(pa_instance *in, const pa_ga_params *g, int32_t gen, const uint8_t *d_pop_in,
                     const float *d_fit_in, uint8_t *d_pop_out, void *stream) {
  if (!in || !d_pop_in || !d_fit_in || !d_pop_out)
    return fail(PA_EINVAL, "instance or a buffer is NULL");
  pa_status st = validate_params(in, g);
  if (st != PA_OK) return st;
  if (gen < 0) return fail(PA_EINVAL, "gen=%d is negative", gen);
  const size_t bytes = (size_t)g->pop * in->p.L * in->p.K;
  const uintptr_t a0 = (uintptr_t)d_pop_in, b0 = (uintptr_t)d_pop_out;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(PA_EINVAL, "d_pop_in and d_pop_out overlap");
  if ((st = set_device(in->ctx)) != PA_OK) return st;
  HIP_TRY(launch_ga_step(in->p, make_ga(g), (uint32_t)gen, d_pop_in, d_fit_in, d_pop_out, nullptr,
                         nullptr, (hipStream_t)stream),
          "launch ga_step");
  return PA_OK;
}

pa_status pa_solve_plain(pa_instance *in, const pa_ga_params *g, pa_result *out, void *stream) {
  if (!in || !out) return fail(PA_EINVAL, "instance or result is NULL");
  pa_status st = validate_params(in, g);
  if (st != PA_OK) return st;
  if ((st = set_device(in->ctx)) != PA_OK) return st;
  const int N = g->pop, G = g->gens;
  if ((st = ensure_work_impl(in, N, G)) != PA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const DevGa ga = make_ga(g);
  FitShape shape;
  HIP_TRY(hipEventRecord(in->ev0, s), "hipEventRecord");
  if (ga.n_km > 0) HIP_TRY(launch_kmeans_seed(in->p, s), "launch kmeans");
  HIP_TRY(launch_init_pop(in->p, ga, in->popA, s), "launch init");
  HIP_TRY(launch_fitness(in->p, in->popA, N, in->fitA, shape, in->ctx->info, s), "launch fitness");
  for (int gen = 0; gen < G; ++gen) {
    HIP_TRY(launch_ga_step(in->p, ga, (uint32_t)gen, in->popA, in->fitA, in->popB, nullptr,
                           in->trace, s),
            "launch ga_step");
    HIP_TRY(launch_fitness(in->p, in->popB, N, in->fitB, shape, in->ctx->info, s),
            "launch fitness");
    std::swap(in->popA, in->popB);
    std::swap(in->fitA, in->fitB);
  }
  return finish_solve(in, N, G, out, s);
}

pa_status pa_instance_kmeans_state(pa_instance *in, uint8_t *seed, int32_t *centroids,
                                   int32_t *labels, int32_t *iters) {
  if (!in) return fail(PA_EINVAL, "instance is NULL");
  pa_status st = set_device(in->ctx);
  if (st != PA_OK) return st;
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  const size_t L = in->p.L, K = in->p.K;
  if (seed) HIP_TRY(hipMemcpy(seed, in->p.seed, L * K, hipMemcpyDeviceToHost), "copy seed");
  if (centroids)
    HIP_TRY(hipMemcpy(centroids, in->p.km_cent, sizeof(int32_t) * 2 * K, hipMemcpyDeviceToHost),
            "copy centroids");
  if (labels)
    HIP_TRY(hipMemcpy(labels, in->p.km_labels, sizeof(int32_t) * L * K, hipMemcpyDeviceToHost),
            "copy labels");
  if (iters) HIP_TRY(hipMemcpy(iters, in->p.km_iters, sizeof(int32_t), hipMemcpyDeviceToHost), "copy iters");
  return PA_OK;
}

}  // extern "C"
