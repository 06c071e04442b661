// k_peak.hip -- peak-rate probes of the device: the denominators of the
// rooflines the benchmark reports for the LDS-gather kernels.  Measured:
//   - conflict-free LDS gathers with ds_read_b32 (each half-wave reads 32
//     words in 32 distinct banks, a permutation like a pilot row's),
//   - LDS reads with ds_read_b128 (consecutive 16-byte words per lane),
//   - FP32 VALU issue (independent v_add_f32 chains).
// One workgroup of 1024 threads per CU (its LDS allocation keeps a second one
// off the CU); each workgroup times its own loop with the shader-clock
// counter, so the rates come out per clock and per CU whatever clock the
// device runs at, and the event time of the launch gives that clock.
#include <vector>

#include "pa_host.h"

namespace pa {
namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeLds = 96 * 1024;   // more than half the CU's LDS: one workgroup per CU
constexpr int kProbeRows = 64;         // 256-byte rows read per pass and wave (b32)
constexpr int kProbePasses = 2048;

// the loop of one wave: kProbePasses x kProbeRows ds_read_b32, a 3-input xor
// per pair of reads keeps the loads alive at half a VALU op per read
__global__ __launch_bounds__(kProbeThreads) void k_peak_lds_b32(uint64_t *cycles, uint32_t *sink) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  for (int i = threadIdx.x; i < kProbeLds / 4; i += blockDim.x) lds[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // half-wave h reads words (7 * lane mod 32) of its own 128-byte half-row:
  // 32 distinct banks per half-wave
  const uint32_t base = (uint32_t)((((lane * 7) & 31) + (lane >> 5) * 32) * 4);
  const char *p = reinterpret_cast<const char *>(lds) + base;
  uint32_t a0 = 0, a1 = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memtime();
  for (int pass = 0; pass < kProbePasses; ++pass) {
    const char *q = p + ((pass & 3) * kProbeRows * 256);
#pragma unroll
    for (int r = 0; r < kProbeRows; r += 2) {
      const uint32_t x = *reinterpret_cast<const uint32_t *>(q + r * 256);
      const uint32_t y = *reinterpret_cast<const uint32_t *>(q + (r + 1) * 256);
      a0 = a0 ^ x ^ y;
    }
    asm volatile("" : "+v"(a0), "+v"(a1));
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
  if (a0 == 0x12345678u) sink[threadIdx.x] = a0 ^ a1;
}

// kProbePasses x 16 ds_read_b128 per wave (1 KiB each), two 3-input xors per read
__global__ __launch_bounds__(kProbeThreads) void k_peak_lds_b128(uint64_t *cycles, uint32_t *sink) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  for (int i = threadIdx.x; i < kProbeLds / 4; i += blockDim.x) lds[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const char *p = reinterpret_cast<const char *>(lds) + lane * 16;
  uint32_t a0 = 0, a1 = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memtime();
  for (int pass = 0; pass < kProbePasses; ++pass) {
    const char *q = p + ((pass & 3) * 16 * 1024);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const u4 v = *reinterpret_cast<const u4 *>(q + r * 1024);
      a0 = a0 ^ v.x ^ v.y;
      a1 = a1 ^ v.z ^ v.w;
    }
    asm volatile("" : "+v"(a0), "+v"(a1));
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
  if (a0 == 0x12345678u) sink[threadIdx.x] = a0 ^ a1;
}

// kProbePasses x 64 v_add_f32 per wave, in 8 independent chains
__global__ __launch_bounds__(kProbeThreads) void k_peak_valu(uint64_t *cycles, float *sink,
                                                             float step) {
  float a[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) a[c] = (float)(threadIdx.x + c);
  __syncthreads();
  const uint64_t t0 = __builtin_amdgcn_s_memtime();
  for (int pass = 0; pass < kProbePasses; ++pass) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int c = 0; c < 8; ++c) a[c] = a[c] + step;
    }
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]),
                 "+v"(a[6]), "+v"(a[7]));
  }
  __syncthreads();
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  if (threadIdx.x == 0) cycles[blockIdx.x] = t1 - t0;
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s = s + a[c];
  if (s == -1.0f) sink[threadIdx.x] = s;
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" pa_status pa_device_peaks(pa_context *ctx, pa_peak_rates *out) {
  if (!ctx || !out) return set_error(PA_EINVAL, "context or out is NULL");
  pa_status st = use_device(ctx);
  if (st != PA_OK) return st;
  const int cus = ctx->info.cus;
  uint64_t *d_cyc = nullptr;
  uint32_t *d_sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&d_cyc, sizeof(uint64_t) * cus);
  if (e == hipSuccess) e = hipMalloc(&d_sink, sizeof(uint32_t) * kProbeThreads);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  static LdsAttr a32, a128;
  const hipError_t ae32 =
      allow_lds_once(a32, reinterpret_cast<const void *>(k_peak_lds_b32), kProbeLds);
  const hipError_t ae128 =
      allow_lds_once(a128, reinterpret_cast<const void *>(k_peak_lds_b128), kProbeLds);
  static LdsAttr av;
  const hipError_t aev = allow_lds_once(av, reinterpret_cast<const void *>(k_peak_valu), kProbeLds);
  hipStream_t s = ctx->stream;
  std::vector<uint64_t> cyc(cus);
  double rate[3] = {0.0, 0.0, 0.0};
  double mhz = 0.0;
  const double wave_ops[3] = {(double)kProbePasses * kProbeRows * 256.0,  // bytes per wave
                              (double)kProbePasses * 16 * 1024.0,
                              (double)kProbePasses * 64};                 // instructions per wave
  const double waves = kProbeThreads / 64;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
      e = hipEventRecord(e0, s);
      if (e != hipSuccess) break;
      if (k == 0)
        hipLaunchKernelGGL(k_peak_lds_b32, dim3(cus), dim3(kProbeThreads), kProbeLds, s, d_cyc, d_sink);
      else if (k == 1)
        hipLaunchKernelGGL(k_peak_lds_b128, dim3(cus), dim3(kProbeThreads), kProbeLds, s, d_cyc,
                           d_sink);
      else
        // the LDS allocation (unused) keeps a second workgroup off the CU
        hipLaunchKernelGGL(k_peak_valu, dim3(cus), dim3(kProbeThreads), kProbeLds, s, d_cyc,
                           reinterpret_cast<float *>(d_sink), 1.0f);
      e = launch_status(k == 0 ? ae32 : k == 1 ? ae128 : aev);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipMemcpyAsync(cyc.data(), d_cyc, sizeof(uint64_t) * cus,
                                              hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) break;
    double sum = 0.0;
    uint64_t mx = 1;
    for (uint64_t c : cyc) {
      sum += waves * wave_ops[k] / (double)(c ? c : 1);
      mx = c > mx ? c : mx;
    }
    rate[k] = sum / cus;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f && k == 2)
      mhz = (double)mx / (ms * 1e3);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_cyc) (void)hipFree(d_cyc);
  if (d_sink) (void)hipFree(d_sink);
  if (e != hipSuccess) return hip_error(e, "peak probes");
  out->lds_b32 = rate[0];
  out->lds_b128 = rate[1];
  out->valu_f32 = rate[2];
  out->clock_mhz = mhz;
  out->cus = cus;
  return PA_OK;
}
