// hm_sre_dev.h -- device pieces of the qubit SRE path shared by the forward and adjoint kernels:
// the round schedule of the row pass and the folded product step (see hm_sre.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hm_tile.h"

namespace hm {

__host__ __device__ constexpr int rp_S(int NL, int RB, int k) { return NL - RB * (k + 1) > 0 ? NL - RB * (k + 1) : 0; }
__host__ __device__ constexpr int rp_H(int NL, int RB, int k) { return RB < NL - RB * k ? RB : NL - RB * k; }

template <typename T>
__device__ __forceinline__ void cmul_conj(vec2<T> y, vec2<T> x, T &re, T &im) {
  // conj(y) * x
  re = fmaT(y.x, x.x, y.y * x.y);
  im = fmaT(y.x, x.y, -(y.y * x.x));
}

// Product step of the row pass: for the thread's R values (row-task ch, thread part tlo, register
// r at row position tlo + (r << S0)) form the folded vector u of shift a (see the file comment).
// CH bounds how many registers' loads may be in flight: a scheduling fence after every CH values
// keeps the compiler from hoisting all 2R gathers (register pressure decides occupancy).
template <typename T, int RB, int NL, int CH = (1 << RB)>
__device__ __forceinline__ void sre_product(const vec2<T> *__restrict__ psi, uint32_t half, uint64_t a, uint64_t ch,
                                            uint32_t tlo, bool active, T (&re)[1 << RB], T (&im)[1 << RB]) {
  constexpr int R = 1 << RB;
  constexpr int S0 = NL - RB;
  constexpr int SEG = 1 << S0;
  if (!active) {
#pragma unroll
    for (int r = 0; r < R; ++r) re[r] = im[r] = T(0);
  } else if (a == 0) {
    // a = 0: fold on the top qubit; u_c = (r0 + r1) + i (r0 - r1).
    const uint32_t cb = ((uint32_t)ch << NL) | tlo;
    const vec2<T> *p1b = psi + half;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t c = cb + ((uint32_t)r << S0);
      const vec2<T> p0 = ld32(psi, c), p1 = ld32(p1b, c);
      const T r0 = fmaT(p0.x, p0.x, p0.y * p0.y);
      const T r1 = fmaT(p1.x, p1.x, p1.y * p1.y);
      re[r] = r0 + r1;
      im[r] = r0 - r1;
      if constexpr (CH < R) {
        if ((r + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
    const int j = 63 - __builtin_clzll(a);
    if (j >= NL) {
      // fold bit inside the row index: columns are untouched, rows map c_h -> insert0(c_h, j - NL)
      const uint32_t xr = ins0_32((uint32_t)ch, j - NL);
      const uint32_t yr = xr ^ (uint32_t)(a >> NL);
      const uint32_t alo = (uint32_t)a & (SEG - 1);
      const uint32_t amid = ((uint32_t)(a >> S0)) & (R - 1);
      const uint32_t xb = (xr << NL) | tlo;
      const uint32_t yb = (yr << NL) | (tlo ^ alo);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const vec2<T> px = ld32(psi, xb + ((uint32_t)r << S0));
        const vec2<T> py = ld32(psi, yb + ((uint32_t)(r ^ amid) << S0));
        cmul_conj<T>(py, px, re[r], im[r]);
        if constexpr (CH < R) {
          if ((r + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else if (j >= S0) {
      // fold bit among the register bits of the first round
      const uint32_t base = (uint32_t)ch << (NL + 1);
      const int jj = j - S0;
      const uint32_t alo = (uint32_t)a & (SEG - 1);
      const uint32_t ahi = (uint32_t)(a >> S0);
      const uint32_t xb = base | tlo;
      const uint32_t yb = base | (tlo ^ alo);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t e = ins0_32((uint32_t)r, jj);
        const vec2<T> px = ld32(psi, xb + (e << S0));
        const vec2<T> py = ld32(psi, yb + ((e ^ ahi) << S0));
        cmul_conj<T>(py, px, re[r], im[r]);
        if constexpr (CH < R) {
          if ((r + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      // small shifts (a < 2^S0): generic index arithmetic
      const uint32_t base = (uint32_t)ch << (NL + 1);
      const uint32_t a32 = (uint32_t)a;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t c = tlo | ((uint32_t)r << S0);
        const uint32_t x = base | ins0_32(c, j);
        const vec2<T> px = ld32(psi, x);
        const vec2<T> py = ld32(psi, x ^ a32);
        cmul_conj<T>(py, px, re[r], im[r]);
        if constexpr (CH < R) {
          if ((r + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }

}

// Adjoint seed of one folded real value: |k x|^{2q-2} x (k = 2 for a != 0, 1 for a = 0).
template <typename T, bool Q2>
__device__ __forceinline__ T wfold(T x, T k, double q) {
  if (Q2) return (k * k) * (x * x) * x;
  const T ax = fabs(k * x);
  return ax > T(0) ? (T)pow(ax, (T)(2.0 * q - 2.0)) * x : T(0);
}

}  // namespace hm
