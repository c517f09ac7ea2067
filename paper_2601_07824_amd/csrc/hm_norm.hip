// hm_norm.hip -- optional check that an input state is normalised (HM_OPT_CHECK_NORM).
//
// Every result of the library assumes sum_x |psi_x|^2 = 1 (S_q scales as the norm to the power 4q;
// the pure-state mana formula holds for unit vectors).  With the option set, each entry point that
// takes a state first computes the squared norm in FP64 on the device (fixed-order reduction),
// copies it to pinned host memory, synchronises the caller's stream and rejects the call with
// HM_E_NOT_NORMALIZED when it deviates from 1 by more than 1e-5 (complex64) or 1e-12 (complex128).
// The device and host scalars are owned by the library, one pair per device, allocated on first
// use and kept until the process ends.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

static constexpr int NORM_BLOCKS = 256, NORM_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(NORM_THREADS) void k_norm2_part(const vec2<T> *psi, uint64_t D, double *part) {
  __shared__ double red[NORM_THREADS];
  const uint32_t t = threadIdx.x;
  double s = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * NORM_THREADS + t; i < D; i += (uint64_t)gridDim.x * NORM_THREADS) {
    const vec2<T> v = psi[i];
    s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  red[t] = s;
  __syncthreads();
  for (uint32_t w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NORM_THREADS) void k_norm2_final(double *part, int nb) {
  __shared__ double red[NORM_THREADS];
  const uint32_t t = threadIdx.x;
  red[t] = (int)t < nb ? part[t] : 0.0;
  __syncthreads();
  for (uint32_t w = NORM_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) part[NORM_BLOCKS] = red[0];
}

int check_norm(const void *psi, uint64_t D, int dbl, hipStream_t st) {
  static std::mutex mu;
  static double *dev_part[64] = {};
  static double *host_val[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(E_HIP, "norm check: no current device");
  std::lock_guard<std::mutex> g(mu);
  if (!dev_part[dev] && hipMalloc((void **)&dev_part[dev], (NORM_BLOCKS + 1) * sizeof(double)) != hipSuccess)
    return fail(E_HIP, "norm check: device allocation failed");
  if (!host_val[dev] && hipHostMalloc((void **)&host_val[dev], sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(E_HIP, "norm check: pinned allocation failed");
  const uint64_t want = (D + NORM_THREADS - 1) / NORM_THREADS;
  const int nb = (int)(want < (uint64_t)NORM_BLOCKS ? want : (uint64_t)NORM_BLOCKS);
  if (dbl) hipLaunchKernelGGL(k_norm2_part<double>, dim3(nb), dim3(NORM_THREADS), 0, st, (const vec2<double> *)psi, D, dev_part[dev]);
  else hipLaunchKernelGGL(k_norm2_part<float>, dim3(nb), dim3(NORM_THREADS), 0, st, (const vec2<float> *)psi, D, dev_part[dev]);
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(NORM_THREADS), 0, st, dev_part[dev], nb);
  if (hipPeekAtLastError() != hipSuccess) return fail(E_HIP, "norm check launch: %s", hipGetErrorString(hipGetLastError()));
  if (hipMemcpyAsync(host_val[dev], dev_part[dev] + NORM_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(E_HIP, "norm check: %s", hipGetErrorString(hipGetLastError()));
  const double v = *host_val[dev];
  const double tol = dbl ? 1e-12 : 1e-5;
  if (!(fabs(v - 1.0) <= tol))
    return fail(E_NOT_NORMALIZED, "state not normalised: sum |psi|^2 = %.17g (tolerance %g)", v, tol);
  return OK;
}

}  // namespace hm
