// hm_mixed.hip -- mana of a mixed qutrit state (Sec. "Mana of mixed states via a fast tensor-product
// transform" of "Computing quantum magic of state vectors", Eq. MN_factor_mana and its Algorithm) and
// the reduced density matrix of a pure state (Sec. "Mana calculation", subsystem mana).
//
// All 9^N values w_u = Tr(rho A_u) are one tensor power of a 9 x 9 single-qutrit matrix applied to the
// vectorised density matrix.  On the GPU the density matrix (row-major, rho[r 3^N + c] = <r|rho|c>,
// qutrit k = base-3 digit k of r and c) is reordered so that qutrit k's pair (r_k, c_k) is the base-9
// digit k of the position (p = sum_k (3 r_k + c_k) 9^k), and the single-qutrit matrix is applied along
// every digit.  Several digits share one HBM-streaming pass through LDS:
//   * pass A reads a 27 x 27 block of rho (qutrits 0..2 of its rows and columns vary, 27 contiguous
//     columns per row), reorders it in LDS, applies the matrix along digits 0, 1, 2 and writes the
//     729 values contiguously (the reordering costs no pass of its own);
//   * each pass B takes digits k, k + 1 with digit 0 along for contiguous 144-B segments (9 x 81
//     values per tile), in place (a last single digit takes digits 0 and 1 along);
//   * the last pass does not write back: it reduces sum_u |w_u|, sum_u w_u and sum_u w_u^2 in FP64
//     (fixed order) instead.
// N = 8 thus streams the 9^N values 4 times (read + write 3 times, read once) instead of N + 1.
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

static constexpr int MIXED_NT = 256;
static constexpr int MIXED_RED_BLOCKS = 2048;

// Fibres of 9 values at stride `st` inside an LDS tile: fibre f (f < nfib) starts at
// (f / st) * 9 st + f % st; thread t takes fibres t, t + MIXED_NT, ...
template <typename T>
__device__ __forceinline__ void lds_digit(vec2<T> *t, int nfib, int st) {
  for (int f = threadIdx.x; f < nfib; f += MIXED_NT) {
    const int base = (f / st) * st * 9 + f % st;
    vec2<T> x[9], y[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = t[base + a * st];
    mixed_fibre<T>(x, y);
#pragma unroll
    for (int a = 0; a < 9; ++a) t[base + a * st] = y[a];
  }
}

// FP64 sums {sum |w|, sum w, sum w^2} of the real parts of the tile's n values into acc.
template <typename T>
__device__ __forceinline__ void lds_sums(const vec2<T> *t, int n, double (&acc)[3]) {
  for (int e = threadIdx.x; e < n; e += MIXED_NT) {
    const double w = (double)t[e].x;  // real for a Hermitian rho
    acc[0] += fabs(w);
    acc[1] += w;
    acc[2] = fma(w, w, acc[2]);
  }
}

// Fixed-order workgroup sums of acc into part[blockIdx.x].
__device__ __forceinline__ void block_sums_out(double (&acc)[3], double *part) {
  __shared__ double red[3][MIXED_NT];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (unsigned w = MIXED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[blockIdx.x * 3 + k] = red[k][0];
}

// Pass A: tile q (q < 9^(N - M)) is the 3^M x 3^M block of rho whose rows and columns share the
// base-3 digits M.. of q's pairs (mu_k = 3 r_k + c_k = base-9 digit k - M of q); in LDS it is
// reordered to p_lo = sum_{j < M} mu_j 9^j and transformed along digits 0..M-1, then written to
// v[q 9^M + p_lo] (REDUCE: summed instead).  M = min(N, 3).
template <typename T, int M, bool REDUCE>
__global__ __launch_bounds__(MIXED_NT) void k_mixed_first(const vec2<T> *__restrict__ rho, uint64_t D, uint64_t n_tiles,
                                                           vec2<T> *__restrict__ v, double *part) {
  constexpr int B = M == 1 ? 3 : M == 2 ? 9 : 27;  // 3^M
  constexpr int TILE = B * B;                       // 9^M
  __shared__ vec2<T> t[TILE];
  double acc[3] = {0.0, 0.0, 0.0};
  for (uint64_t b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    // neighbouring blocks share cache lines at their edges: keep them on one XCD's L2
    const uint64_t q = (uint64_t)xcd_tile((int64_t)b, (int64_t)n_tiles);
    // high row / column parts of the block
    uint64_t R = 0, C = 0, w3 = B, qq = q;
    while (qq) {
      const uint32_t mu = (uint32_t)(qq % 9);
      qq /= 9;
      R += (mu / 3) * w3;
      C += (mu % 3) * w3;
      w3 *= 3;
    }
    __syncthreads();  // the previous tile's LDS reads are done
    for (int e = threadIdx.x; e < TILE; e += MIXED_NT) {
      const int rl = e / B, cl = e % B;  // row-major within the block: B contiguous columns per row
      int p = 0, w9 = 1, r = rl, c = cl;
#pragma unroll
      for (int j = 0; j < M; ++j, w9 *= 9, r /= 3, c /= 3) p += (3 * (r % 3) + (c % 3)) * w9;
      t[p] = rho[(R + rl) * D + C + cl];
    }
    __syncthreads();
    lds_digit<T>(t, TILE / 9, 1);
    if constexpr (M >= 2) {
      __syncthreads();
      lds_digit<T>(t, TILE / 9, 9);
    }
    if constexpr (M >= 3) {
      __syncthreads();
      lds_digit<T>(t, TILE / 9, 81);
    }
    __syncthreads();
    if constexpr (REDUCE) {
      lds_sums<T>(t, TILE, acc);
    } else {
      vec2<T> *o = v + q * TILE;
      for (int e = threadIdx.x; e < TILE; e += MIXED_NT) o[e] = t[e];
    }
  }
  if constexpr (REDUCE) block_sums_out(acc, part);
}

// Pass B: digits k and k + 1 (ND = 2) or k alone (ND = 1), with the P lowest digits carried along
// so that a tile reads contiguous segments of 9^P values (144 B for P = 1, 1296 B for P = 2) and
// holds 9^(ND + P) = 729 values: tile q covers base + j + sum_{i < ND} mu_i 9^(k + i), j < 9^P,
// base = (q mod 9^(k-P)) 9^P + (q div 9^(k-P)) 9^(k+ND); LDS layout [mu_{k+1}][mu_k][j].  In place,
// or summed (REDUCE).
template <typename T, int ND, int P, bool REDUCE>
__global__ __launch_bounds__(MIXED_NT) void k_mixed_pair(vec2<T> *__restrict__ v, uint64_t n_tiles, uint64_t lo_span,
                                                          uint64_t stride_k, double *part) {
  constexpr int PS = P == 1 ? 9 : 81;           // 9^P
  constexpr int TILE = PS * (ND == 2 ? 81 : 9);  // 9^(ND + P)
  __shared__ vec2<T> t[TILE];
  double acc[3] = {0.0, 0.0, 0.0};
  auto off = [&](int e) -> uint64_t {
    const int j = e % PS, m = e / PS;  // m = mu_k + 9 mu_{k+1}
    return (uint64_t)j + (ND == 2 ? (uint64_t)(m % 9) * stride_k + (uint64_t)(m / 9) * stride_k * 9
                                  : (uint64_t)m * stride_k);
  };
  for (uint64_t b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    // consecutive tiles share the cache lines their segments straddle: keep them on one XCD's L2
    const uint64_t q = (uint64_t)xcd_tile((int64_t)b, (int64_t)n_tiles);
    const uint64_t base = (q % lo_span) * PS + (q / lo_span) * stride_k * (ND == 2 ? 81 : 9);
    __syncthreads();
    for (int e = threadIdx.x; e < TILE; e += MIXED_NT) t[e] = v[base + off(e)];
    __syncthreads();
    lds_digit<T>(t, TILE / 9, PS);
    if constexpr (ND == 2) {
      __syncthreads();
      lds_digit<T>(t, TILE / 9, PS * 9);
    }
    __syncthreads();
    if constexpr (REDUCE) {
      lds_sums<T>(t, TILE, acc);
    } else {
      for (int e = threadIdx.x; e < TILE; e += MIXED_NT) v[base + off(e)] = t[e];
    }
  }
  if constexpr (REDUCE) block_sums_out(acc, part);
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

// [partials][reordered vector 9^N values]
int mixed_workspace(int N, int dbl, size_t *bytes) {
  if (N < 1 || N > 10) return fail(E_SIZE, "mixed mana: n = %d outside [1, 10]", N);
  const uint64_t D = pow_u(3, N);
  *bytes = align256(MIXED_RED_BLOCKS * 3 * sizeof(double)) + align256(D * D * (dbl ? 16 : 8));
  return OK;
}

// One workgroup per tile, or a grid-stride loop over `cap` workgroups (a multiple of 8, so that the
// tiles a workgroup takes stay on its XCD's share).
static unsigned grid_of(uint64_t tiles, uint64_t cap) { return (unsigned)(tiles < cap ? tiles : cap); }

template <typename T, int M>
static void launch_first(bool reduce, const void *rho, uint64_t D, uint64_t tiles, vec2<T> *v, double *part,
                         unsigned *red_grid, hipStream_t st) {
  ProfScope prof(reduce ? "mixed_last" : "mixed_first", st);
  if (reduce) {
    *red_grid = grid_of(tiles, MIXED_RED_BLOCKS);
    hipLaunchKernelGGL((k_mixed_first<T, M, true>), dim3(*red_grid), dim3(MIXED_NT), 0, st, (const vec2<T> *)rho, D,
                       tiles, v, part);
  } else {
    hipLaunchKernelGGL((k_mixed_first<T, M, false>), dim3(grid_of(tiles, 1u << 20)), dim3(MIXED_NT), 0, st,
                       (const vec2<T> *)rho, D, tiles, v, part);
  }
}

template <typename T>
static int mixed_t(int N, const void *rho, double *out, void *ws, hipStream_t st) {
  const uint64_t D = pow_u(3, N), V = D * D;
  char *w = (char *)ws;
  double *part = (double *)w;
  vec2<T> *v = (vec2<T> *)(w + align256(MIXED_RED_BLOCKS * 3 * sizeof(double)));
  const int M = N < 3 ? N : 3;
  const uint64_t tiles_a = V / pow_u(9, M);
  unsigned red_grid = 0;
  if (M == 1) launch_first<T, 1>(N == M, rho, D, tiles_a, v, part, &red_grid, st);
  else if (M == 2) launch_first<T, 2>(N == M, rho, D, tiles_a, v, part, &red_grid, st);
  else launch_first<T, 3>(N == M, rho, D, tiles_a, v, part, &red_grid, st);
  for (int k = M; k < N;) {
    // two digits with digit 0 carried along, or (the last digit alone) one with digits 0 and 1
    const int nd = N - k >= 2 ? 2 : 1, P = nd == 2 ? 1 : 2;
    const bool last = k + nd == N;
    const uint64_t tiles = V / pow_u(9, nd + P), lo_span = pow_u(9, k - P), stride_k = pow_u(9, k);
    ProfScope prof(last ? "mixed_last" : "mixed_pair", st);
    if (last) {
      red_grid = grid_of(tiles, MIXED_RED_BLOCKS);
      if (nd == 2)
        hipLaunchKernelGGL((k_mixed_pair<T, 2, 1, true>), dim3(red_grid), dim3(MIXED_NT), 0, st, v, tiles, lo_span,
                           stride_k, part);
      else
        hipLaunchKernelGGL((k_mixed_pair<T, 1, 2, true>), dim3(red_grid), dim3(MIXED_NT), 0, st, v, tiles, lo_span,
                           stride_k, part);
    } else {
      hipLaunchKernelGGL((k_mixed_pair<T, 2, 1, false>), dim3(grid_of(tiles, 1u << 20)), dim3(MIXED_NT), 0, st, v, tiles,
                         lo_span, stride_k, part);
    }
    k += nd;
  }
  hipLaunchKernelGGL(k_mixed_total, dim3(1), dim3(256), 0, st, (const double *)part, (int)red_grid, N, out);
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
