// k_prep.hip -- builds the FP32 device tables of one problem from its FP64
// large-scale fading table (Sec. 3.1, Eq. 2).
//
// Per BS l the row beta[l][.][.] is scaled by 2^-e_l, e_l the binary exponent
// of its largest entry, so the largest scaled value lies in [0.5, 1).  Scaling
// everything one BS hears by the same power of two leaves the asymptotic SINR
// of Eq. 5 unchanged and is exact in FP64; the squares then fit FP32.  For the
// finite-M bound the SNR is rescaled by the inverse power (rho_l = rho 2^e_l)
// so every product rho*beta is unchanged.  For the inter-cluster interference
// of Eq. 8 (objective 2) the tables hold the scaled gains themselves, not their
// squares (its ratios are of first powers, and are unchanged by the scaling).
#include "pa_dev.h"
#include "pa_internal.h"

namespace pa {

constexpr int kPrepBlock = 256;

__global__ __launch_bounds__(kPrepBlock) void k_prep(const double *__restrict__ beta, int L, int K,
                                                      int TP, int finite_m, int first_power,
                                                      double rho, int M,
                                                      float *__restrict__ T2,
                                                      float *__restrict__ T1,
                                                      float *__restrict__ T2z,
                                                      float *__restrict__ Town,
                                                      float *__restrict__ lconst) {
  __shared__ double red[kPrepBlock];
  const int l = blockIdx.x;
  const int LK = L * K;
  const double *row = beta + (size_t)l * LK;
  double mx = 0.0;
  for (int i = threadIdx.x; i < LK; i += blockDim.x) mx = fmax(mx, row[i]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kPrepBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);
  // cell-major device layout: T[j][l][p], p padded to TP with zeros
  for (int i = threadIdx.x; i < L * TP; i += blockDim.x) {
    const int j = i / TP, p = i - j * TP;
    double b = 0.0;
    if (p < K) b = ldexp(row[j * K + p], -e);
    const size_t dst = ((size_t)j * L + l) * TP + p;
    const float sq = first_power ? (float)b : (float)(b * b);
    T2[dst] = sq;
    T2z[dst] = j == l ? 0.0f : sq;
    if (j == l) Town[l * TP + p] = sq;
    if (finite_m) T1[dst] = (float)b;
  }
  if (finite_m && threadIdx.x == 0) {
    double B = 0.0;  // everything BS l hears, scaled, summed in (j, k) order
    for (int i = 0; i < LK; ++i) B += ldexp(row[i], -e);
    const double rho_l = ldexp(rho, e);
    const double tau = (double)K;
    lconst[2 * l + 0] = (float)(tau * rho_l);
    lconst[2 * l + 1] = (float)((1.0 + rho_l * B) / ((double)M * tau * rho_l * rho_l));
  }
}

hipError_t launch_prep(const DevProblem &p, int M, double rho, hipStream_t s) {
  const int finite_m = p.se_mode == 1;
  const int first_power = p.objective == 2;
  hipLaunchKernelGGL(k_prep, dim3(p.L), dim3(kPrepBlock), 0, s, p.beta, p.L, p.K, p.TP, finite_m,
                     first_power, rho, M, p.T2, p.T1, p.T2z, p.Town, p.lconst);
  return hipGetLastError();
}

}  // namespace pa
