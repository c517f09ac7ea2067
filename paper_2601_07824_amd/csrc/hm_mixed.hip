// hm_mixed.hip -- mana of a mixed qutrit state (Sec. "Mana of mixed states via a fast tensor-product
// transform" of "Computing quantum magic of state vectors", Eq. MN_factor_mana and its Algorithm) and
// the reduced density matrix of a pure state (Sec. "Mana calculation", subsystem mana).
//
// All 9^N values w_u = Tr(rho A_u) are one tensor power of a 9 x 9 single-qutrit matrix applied to the
// vectorised density matrix.  On the GPU the density matrix (row-major, rho[r 3^N + c] = <r|rho|c>,
// qutrit k = base-3 digit k of r and c) is first reordered so that qutrit k's pair (r_k, c_k) is the
// base-9 digit k of the position (p = sum_k (3 r_k + c_k) 9^k); then one HBM-streaming pass per qutrit
// applies the single-qutrit matrix to every fibre of 9 values along that digit, in place.  The pass
// over the last digit (the fibres are 9 consecutive values) does not write back: it reduces
// sum_u |w_u|, sum_u w_u and sum_u w_u^2 in FP64 (fixed order) instead.
//
// The single-qutrit matrix, from A_ab|x> = omega^{2b(a-x)} |2a - x> (the phase-space point operators of
// Eq. phase-space up to a relabelling of the points): with x_mu = rho_{r,c} at mu = 3 r + c,
//   w_{3a+b} = sum_c omega^{2b(a-c)} x_{3((2a - c) mod 3) + c},
// three non-zero entries per row (the F_3 blocks of the paper's factorisation M = P (F3+F3+F3) P').
// Mana = log2(sum_u |w_u| / 3^N) (Eq. mana with W = Tr(rho A)/3^N).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

// 9^k positions of the reordered vector: contributions of a row index r and a column index c.
__global__ void k_mixed_digits(int n, uint64_t D, uint64_t *pr, uint64_t *pc) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= D) return;
  uint64_t v = x, r = 0, c = 0, w = 1;
  for (int k = 0; k < n; ++k, w *= 9, v /= 3) {
    r += 3 * (v % 3) * w;
    c += (v % 3) * w;
  }
  pr[x] = r;
  pc[x] = c;
}

// v[pr[r] + pc[c]] = rho[r D + c]: one block row of 256 columns per thread block (coalesced reads).
template <typename T>
__global__ __launch_bounds__(256) void k_mixed_vec(const vec2<T> *rho, uint64_t D, const uint64_t *pr,
                                                   const uint64_t *pc, vec2<T> *v) {
  const uint64_t r = blockIdx.y + ((uint64_t)blockIdx.z << 16);
  if (r >= D) return;
  const uint64_t base = pr[r];
  for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < D; c += (uint64_t)gridDim.x * 256)
    v[base + pc[c]] = rho[r * D + c];
}

// The single-qutrit transform of one fibre x[0..8] -> y[0..8].
template <typename T>
__device__ __forceinline__ void mixed_fibre(const vec2<T> (&x)[9], vec2<T> (&y)[9]) {
  const T h = T(-0.5), s = T(0.86602540378443864676372317075294);  // omega = h + i s
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T re = T(0), im = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const vec2<T> z = x[3 * ((2 * a - c + 3) % 3) + c];
        const int m = (2 * b * (a - c + 3)) % 3;  // omega^m
        if (m == 0) {
          re += z.x;
          im += z.y;
        } else {
          const T si = m == 1 ? s : -s;
          re += h * z.x - si * z.y;
          im += h * z.y + si * z.x;
        }
      }
      y[3 * a + b].x = re;
      y[3 * a + b].y = im;
    }
}

// One pass along base-9 digit k (stride 9^k), in place.  Thread f owns fibre f.
template <typename T>
__global__ __launch_bounds__(256) void k_mixed_leg(vec2<T> *v, uint64_t n_fibres, uint64_t stride) {
  for (uint64_t f = (uint64_t)blockIdx.x * 256 + threadIdx.x; f < n_fibres; f += (uint64_t)gridDim.x * 256) {
    const uint64_t base = (f / stride) * stride * 9 + f % stride;
    vec2<T> x[9], y[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = v[base + a * stride];
    mixed_fibre<T>(x, y);
#pragma unroll
    for (int a = 0; a < 9; ++a) v[base + a * stride] = y[a];
  }
}

// The pass along digit 0 (fibres of 9 consecutive values) with the reduction instead of a write:
// per-block FP64 partials {sum |w|, sum w, sum w^2} of the real parts (w is real for a Hermitian rho).
static constexpr int MIXED_RED_BLOCKS = 2048;
template <typename T>
__global__ __launch_bounds__(256) void k_mixed_last(const vec2<T> *v, uint64_t n_fibres, double *part) {
  __shared__ double red[3][256];
  double m = 0.0, s = 0.0, q = 0.0;
  for (uint64_t f = (uint64_t)blockIdx.x * 256 + threadIdx.x; f < n_fibres; f += (uint64_t)gridDim.x * 256) {
    vec2<T> x[9], y[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = v[f * 9 + a];
    mixed_fibre<T>(x, y);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const double w = (double)y[a].x;
      m += fabs(w);
      s += w;
      q = fma(w, w, q);
    }
  }
  red[0][threadIdx.x] = m;
  red[1][threadIdx.x] = s;
  red[2][threadIdx.x] = q;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[blockIdx.x * 3 + k] = red[k][0];
}

__global__ __launch_bounds__(256) void k_mixed_total(const double *part, int nblk, int N, double *out) {
  __shared__ double red[3][256];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[i * 3 + k];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double D = pow(3.0, (double)N);
    out[0] = log2(red[0][0] / D);  // Eq. mana: log2 sum_u |W(u)|, W = Tr(rho A_u) / 3^N
    out[1] = red[1][0] / D;        // sum_u W(u) = Tr rho
    out[2] = red[2][0] / D;        // 3^N sum_u W(u)^2 = Tr rho^2
  }
}

// rho_A[i D_A + j] = sum_b psi[i + D_A b] conj(psi[j + D_A b]) (FP64 sums): the subsystem of the
// qutrits 0..n_a-1 (low digits); one block row of 256 columns j per thread block.
template <typename T>
__global__ __launch_bounds__(256) void k_reduced_density(const vec2<T> *psi, uint64_t DA, uint64_t DB, vec2<T> *rho) {
  const uint64_t i = blockIdx.y + ((uint64_t)blockIdx.z << 16);
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= DA || j >= DA) return;
  double re = 0.0, im = 0.0;
  for (uint64_t b = 0; b < DB; ++b) {
    const vec2<T> p = psi[i + DA * b], q = psi[j + DA * b];
    // p conj(q)
    re = fma((double)p.x, (double)q.x, fma((double)p.y, (double)q.y, re));
    im = fma((double)p.y, (double)q.x, fma(-(double)p.x, (double)q.y, im));
  }
  vec2<T> o;
  o.x = (T)re;
  o.y = (T)im;
  rho[i * DA + j] = o;
}

static uint64_t pow_u(uint64_t b, int e) {
  uint64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// [digit tables pr, pc (2 x 3^N u64)][partials][reordered vector 9^N values]
int mixed_workspace(int N, int dbl, size_t *bytes) {
  if (N < 1 || N > 10) return fail(E_SIZE, "mixed mana: n = %d outside [1, 10]", N);
  const uint64_t D = pow_u(3, N);
  *bytes = 2 * align256(D * 8) + align256(MIXED_RED_BLOCKS * 3 * sizeof(double)) + align256(D * D * (dbl ? 16 : 8));
  return OK;
}

template <typename T>
static int mixed_t(int N, const void *rho, double *out, void *ws, hipStream_t st) {
  const uint64_t D = pow_u(3, N);
  char *w = (char *)ws;
  uint64_t *pr = (uint64_t *)w;
  uint64_t *pc = (uint64_t *)(w + align256(D * 8));
  double *part = (double *)(w + 2 * align256(D * 8));
  vec2<T> *v = (vec2<T> *)(w + 2 * align256(D * 8) + align256(MIXED_RED_BLOCKS * 3 * sizeof(double)));
  hipLaunchKernelGGL(k_mixed_digits, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, st, N, D, pr, pc);
  {
    ProfScope prof("mixed_vec", st);
    const unsigned gx = (unsigned)((D + 255) / 256 < 64 ? (D + 255) / 256 : 64);
    hipLaunchKernelGGL(k_mixed_vec<T>, dim3(gx, (unsigned)(D < 65536 ? D : 65536), (unsigned)((D + 65535) >> 16)),
                       dim3(256), 0, st, (const vec2<T> *)rho, D, (const uint64_t *)pr, (const uint64_t *)pc, v);
  }
  const uint64_t nf = D * D / 9;
  const unsigned grid = (unsigned)((nf + 255) / 256 < 16384 ? (nf + 255) / 256 : 16384);
  uint64_t stride = D * D / 9;  // 9^(N-1): the highest digit first
  for (int k = N - 1; k >= 1; --k, stride /= 9) {
    ProfScope prof("mixed_leg", st);
    hipLaunchKernelGGL(k_mixed_leg<T>, dim3(grid), dim3(256), 0, st, v, nf, stride);
  }
  {
    ProfScope prof("mixed_last", st);
    hipLaunchKernelGGL(k_mixed_last<T>, dim3(MIXED_RED_BLOCKS), dim3(256), 0, st, (const vec2<T> *)v, nf, part);
  }
  hipLaunchKernelGGL(k_mixed_total, dim3(1), dim3(256), 0, st, (const double *)part, MIXED_RED_BLOCKS, N, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "mixed mana launch: %s", hipGetErrorString(hipGetLastError()));
}

int mixed_launch(int N, int dbl, const void *rho, double *out, void *ws, hipStream_t st) {
  return dbl ? mixed_t<double>(N, rho, out, ws, st) : mixed_t<float>(N, rho, out, ws, st);
}

int reduced_density_launch(int N, int NA, int dbl, const void *psi, void *rho, hipStream_t st) {
  const uint64_t DA = pow_u(3, NA), DB = pow_u(3, N - NA);
  const dim3 grid((unsigned)((DA + 255) / 256), (unsigned)(DA < 65536 ? DA : 65536), (unsigned)((DA + 65535) >> 16));
  ProfScope prof("reduced_density", st);
  if (dbl) hipLaunchKernelGGL(k_reduced_density<double>, grid, dim3(256), 0, st, (const double2 *)psi, DA, DB, (double2 *)rho);
  else hipLaunchKernelGGL(k_reduced_density<float>, grid, dim3(256), 0, st, (const float2 *)psi, DA, DB, (float2 *)rho);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "reduced density launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace hm
