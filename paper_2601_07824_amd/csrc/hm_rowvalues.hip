// hm_rowvalues.hip -- signed real Pauli expectations of one X-row (debug / inspection entry point).
//
// <P_{a,b}> = i^{popcount(a & b)} chi_b(a), where chi(a) is the full-length (unfolded) Walsh-Hadamard
// transform of v_x = conj(psi_{x^a}) psi_x (Eq. Z_ovN) and P_{a,b} the Hermitian Pauli string with
// X-part a and Z-part b.  This path is not performance critical: the product, each butterfly stage
// and the phase are separate elementwise kernels over a workspace copy of v.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

template <typename T>
__global__ void k_rv_product(const vec2<T> *psi, uint64_t D, uint64_t a, vec2<T> *v) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= D) return;
  const vec2<T> p = psi[x], y = psi[x ^ a];
  vec2<T> o;
  o.x = y.x * p.x + y.y * p.y;
  o.y = y.x * p.y - y.y * p.x;
  v[x] = o;
}

template <typename T>
__global__ void k_rv_stage(vec2<T> *v, uint64_t D, uint64_t h) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D / 2) return;
  const uint64_t lo = ((i / h) * 2 * h) + (i % h), hi = lo + h;
  const vec2<T> u = v[lo], w = v[hi];
  vec2<T> s, d;
  s.x = u.x + w.x;
  s.y = u.y + w.y;
  d.x = u.x - w.x;
  d.y = u.y - w.y;
  v[lo] = s;
  v[hi] = d;
}

template <typename T>
__global__ void k_rv_phase(const vec2<T> *v, uint64_t D, uint64_t a, double *out) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= D) return;
  const vec2<T> c = v[b];
  // i^k chi: k = 0: re, 1: -im, 2: -re, 3: im
  const int k = __popcll(a & b) & 3;
  double r = (k == 0) ? (double)c.x : (k == 1) ? -(double)c.y : (k == 2) ? -(double)c.x : (double)c.y;
  out[b] = r;
}

size_t sre_row_values_workspace(int N, int dbl) { return align256(((size_t)1 << N) * (dbl ? 16 : 8)); }

template <typename T>
static int rv_t(int N, const void *psi, uint64_t a, double *out, void *ws, hipStream_t st) {
  const uint64_t D = 1ull << N;
  vec2<T> *v = (vec2<T> *)ws;
  const unsigned thr = 256;
  hipLaunchKernelGGL(k_rv_product<T>, dim3((unsigned)((D + thr - 1) / thr)), dim3(thr), 0, st, (const vec2<T> *)psi, D, a, v);
  for (uint64_t h = 1; h < D; h <<= 1)
    hipLaunchKernelGGL(k_rv_stage<T>, dim3((unsigned)((D / 2 + thr - 1) / thr)), dim3(thr), 0, st, v, D, h);
  hipLaunchKernelGGL(k_rv_phase<T>, dim3((unsigned)((D + thr - 1) / thr)), dim3(thr), 0, st, (const vec2<T> *)v, D, a, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "row values launch: %s", hipGetErrorString(hipGetLastError()));
}

int sre_row_values_launch(int N, int dbl, const void *psi, uint64_t a, double *out, void *ws, hipStream_t st) {
  return dbl ? rv_t<double>(N, psi, a, out, ws, st) : rv_t<float>(N, psi, a, out, ws, st);
}

}  // namespace hm
