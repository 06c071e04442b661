// k_exhaustive.hip -- exhaustive search over pilot assignments (the EX-PA
// reference of Sec. 3.3 / Sec. 6): the fitness is invariant under a global
// relabelling of the pilots, so cell 0 is fixed to the identity and the
// K!^(L-1) assignments of cells 1..L-1 are enumerated, in chunks: a kernel
// unranks each chromosome of the chunk, the fitness kernel scores it and a
// wave takes the chunk's best.  Ranking is on the FP32 fitness, ties to the
// lowest enumeration rank.
#include <algorithm>

#include "pa_host.h"

namespace pa {
namespace {

constexpr int kUnrankBlock = 256;
constexpr int kExMaxK = 12;  // K! < 2^32

// Chromosome of enumeration rank base + c, one thread per (c, cell j): cell 0
// is the identity; cell j >= 1 is the permutation of lexicographic rank d_j,
// d_j the base-K! digit of the rank at position L-1-j (cell L-1 varies
// fastest, the order of an odometer over the cells).  The permutation of
// rank d is read from its factorial-base digits: position k takes the
// (d / (K-1-k)!)-th smallest user not yet placed.
__global__ __launch_bounds__(kUnrankBlock) void k_unrank(uint64_t base, int n, int L, int K,
                                                          uint32_t kfact, uint8_t *pop) {
  const int r = blockIdx.x * kUnrankBlock + threadIdx.x;
  if (r >= n * L) return;
  const int c = r / L, j = r - c * L;
  gptr<uint8_t> row = gp(pop + (size_t)r * K);
  if (j == 0) {
    for (int k = 0; k < K; ++k) row[k] = (uint8_t)k;
    return;
  }
  uint64_t idx = base + (uint64_t)c;
  for (int t = L - 1; t > j; --t) idx /= kfact;
  uint32_t d = (uint32_t)(idx % kfact);
  uint32_t f = kfact / (uint32_t)K;  // (K-1)!
  uint32_t used = 0;
  for (int k = 0; k < K; ++k) {
    uint32_t q = d / f;
    d -= q * f;
    int e = 0;
    for (; e < K; ++e) {
      if ((used >> e) & 1u) continue;
      if (q == 0) break;
      --q;
    }
    row[k] = (uint8_t)e;
    used |= 1u << e;
    if (k < K - 1) f /= (uint32_t)(K - 1 - k);
  }
}

hipError_t launch_unrank(uint64_t base, int n, int L, int K, uint32_t kfact, uint8_t *pop,
                         hipStream_t s) {
  const int rows = n * L;
  hipLaunchKernelGGL(k_unrank, dim3((rows + kUnrankBlock - 1) / kUnrankBlock), dim3(kUnrankBlock),
                     0, s, base, n, L, K, kfact, pop);
  return hipGetLastError();
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" pa_status pa_exhaustive(pa_instance *in, int64_t max_count, pa_result *out,
                                   int64_t *best_rank, int64_t *count, void *stream) {
  if (!in || !out) return set_error(PA_EINVAL, "instance or result is NULL");
  const int L = in->p.L, K = in->p.K;
  if (K > kExMaxK)
    return set_error(PA_EINVAL, "K=%d > %d: too many permutations per cell", K, kExMaxK);
  const int64_t limit = max_count > 0 ? max_count : (int64_t)1 << 32;
  uint64_t kfact = 1;
  for (int k = 2; k <= K; ++k) kfact *= (uint64_t)k;
  uint64_t total = 1;
  for (int j = 1; j < L; ++j) {
    if (total > (uint64_t)limit / kfact) {
      return set_error(PA_EINVAL, "K!^(L-1) = %llu^%d exceeds max_count=%lld",
                       (unsigned long long)kfact, L - 1, (long long)limit);
    }
    total *= kfact;
  }
  pa_status st = use_device(in->ctx);
  if (st != PA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const size_t LK = (size_t)L * K;
  const int chunk = (int)std::min<uint64_t>(total, (uint64_t)1 << 20);
  const int nchunks = (int)((total + chunk - 1) / chunk);
  uint8_t *pop = nullptr;
  float *fit = nullptr, *cfit = nullptr;
  int32_t *cidx = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&pop, LK * chunk);
  if (e == hipSuccess) e = hipMalloc(&fit, sizeof(float) * chunk);
  if (e == hipSuccess) e = hipMalloc(&cfit, sizeof(float) * nchunks);
  if (e == hipSuccess) e = hipMalloc(&cidx, sizeof(int32_t) * nchunks);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int ch = 0; ch < nchunks && e == hipSuccess; ++ch) {
    const uint64_t base = (uint64_t)ch * chunk;
    const int n = (int)std::min<uint64_t>(chunk, total - base);
    e = launch_unrank(base, n, L, K, (uint32_t)kfact, pop, s);
    if (e == hipSuccess) e = launch_fitness(in->p, pop, n, fit, FitShape{}, in->ctx->info, s);
    if (e == hipSuccess) e = launch_best(fit, n, cidx + ch, cfit + ch, s);
  }
  std::vector<float> hf(nchunks);
  std::vector<int32_t> hi(nchunks);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hf.data(), cfit, sizeof(float) * nchunks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hi.data(), cidx, sizeof(int32_t) * nchunks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  uint64_t best = 0;
  float bf = 0.0f;
  if (e == hipSuccess) {
    // chunks in increasing rank: a later chunk wins only with a larger fitness
    // (NaN never wins; the first chunk's best stands in for an all-NaN run)
    bf = hf[0];
    best = (uint64_t)hi[0];
    for (int ch = 1; ch < nchunks; ++ch) {
      if (hf[ch] > bf || (bf != bf && hf[ch] == hf[ch])) {
        bf = hf[ch];
        best = (uint64_t)ch * chunk + (uint64_t)hi[ch];
      }
    }
    e = launch_unrank(best, 1, L, K, (uint32_t)kfact, pop, s);
    if (e == hipSuccess && out->best)
      e = hipMemcpyAsync(out->best, pop, LK, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (pop) (void)hipFree(pop);
  if (fit) (void)hipFree(fit);
  if (cfit) (void)hipFree(cfit);
  if (cidx) (void)hipFree(cidx);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_error(e, "pa_exhaustive");
  out->best_fit = bf;
  out->best_index = -1;
  out->device_ms = ms;
  if (best_rank) *best_rank = (int64_t)best;
  if (count) *count = (int64_t)total;
  return PA_OK;
}
