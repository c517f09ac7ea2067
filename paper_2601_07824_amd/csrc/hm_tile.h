// hm_tile.h -- device building blocks shared by the gfx950 kernels of libhmag.
//
// A "tile" is 2^TB complex values held by NT = 2^LT threads of one workgroup, R = 2^RB values per
// thread in registers.  A round layout with start S places the register index bits at tile-index
// positions [S, S+RB) and the thread index bits at the remaining positions, in order:
//     idx = (tau & (2^S - 1)) | (rho << S) | ((tau >> S) << (S + RB)).
// Butterflies act on register bits; moving to a layout with another S is one pass through LDS.
// LDS addresses are padded with one slot per R values (phys = idx + idx/R): for every layout above,
// any 32 consecutive lanes (8-byte values) or 16 lanes (16-byte values) then hit distinct banks, and
// the per-register part of the address stays a compile-time constant.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hm_internal.h"

namespace hm {

template <typename T> struct vec2_of;
template <> struct vec2_of<float> { using type = float2; };
template <> struct vec2_of<double> { using type = double2; };
template <typename T> using vec2 = typename vec2_of<T>::type;

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// Fused multiply-add in the precision of T (the plain builtin would promote floats to double).
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Load / store element idx of an array given by a uniform base pointer and a 32-bit element index
// (the byte offset stays in one 32-bit register; every buffer here is smaller than 4 GiB).
template <typename V>
__device__ __forceinline__ V ld32(const V *base, uint32_t idx) {
  return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + (uint32_t)(idx * (uint32_t)sizeof(V)));
}
template <typename V>
__device__ __forceinline__ void st32(V *base, uint32_t idx, V v) {
  *reinterpret_cast<V *>(reinterpret_cast<char *>(base) + (uint32_t)(idx * (uint32_t)sizeof(V))) = v;
}

template <int S, int RB>
__device__ __forceinline__ uint32_t lay(uint32_t tau, uint32_t rho) {
  return (tau & ((1u << S) - 1u)) | (rho << S) | ((tau >> S) << (S + RB));
}

template <int RB>
__host__ __device__ __forceinline__ constexpr uint32_t ldspad(uint32_t idx) { return idx + (idx >> RB); }

// lay<S, RB>(tau, rho) split into its thread part and its register part.  The two occupy disjoint
// bit fields, so lay = base + off and ldspad(lay) = ldspad(base) + ldspad(off): the register part
// is a compile-time constant that folds into the immediate offset of the LDS instruction.
template <int S, int RB>
__device__ __forceinline__ uint32_t lay_base(uint32_t tau) {
  return (tau & ((1u << S) - 1u)) | ((tau >> S) << (S + RB));
}
template <int S, int RB>
__host__ __device__ __forceinline__ constexpr uint32_t lay_off(int rho) { return (uint32_t)rho << S; }

// insert a zero bit at position j: bits >= j move up by one.
__device__ __forceinline__ uint64_t ins0(uint64_t c, int j) {
  uint64_t lo = c & ((1ull << j) - 1ull);
  return lo | ((c - lo) << 1);
}
__device__ __forceinline__ uint32_t ins0_32(uint32_t c, int j) {
  uint32_t lo = c & ((1u << j) - 1u);
  return lo | ((c - lo) << 1);
}

// Unnormalised Walsh-Hadamard butterflies over register bits [K0, K1).
template <typename T, int R, int K0, int K1>
__device__ __forceinline__ void wht_regs(T (&re)[R], T (&im)[R]) {
#pragma unroll
  for (int k = K0; k < K1; ++k) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (!((i >> k) & 1)) {
        const int j = i | (1 << k);
        T a = re[i], b = re[j];
        re[i] = a + b;
        re[j] = a - b;
        a = im[i];
        b = im[j];
        im[i] = a + b;
        im[j] = a - b;
      }
    }
  }
}

// Move the tile from layout SA to layout SB through LDS (all NT threads must call it).
// Threads with act == false (padding threads of a block larger than the tile) skip the LDS traffic.
template <typename T, int R, int RB, int SA, int SB>
__device__ __forceinline__ void relayout(T (&re)[R], T (&im)[R], vec2<T> *lds, uint32_t tau, bool act = true) {
  const uint32_t ba = ldspad<RB>(lay_base<SA, RB>(tau));
  const uint32_t bb = ldspad<RB>(lay_base<SB, RB>(tau));
  __syncthreads();  // earlier readers of lds are done
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vec2<T> v;
      v.x = re[r];
      v.y = im[r];
      lds[ba + ldspad<RB>(lay_off<SA, RB>(r))] = v;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vec2<T> v = lds[bb + ldspad<RB>(lay_off<SB, RB>(r))];
      re[r] = v.x;
      im[r] = v.y;
    }
  }
}

// Same as relayout, for tiles too large to stage both components at once: the real parts, then the
// imaginary parts, go through a scalar LDS buffer of 2^TB (+ padding) values.
// Same as relayout, for tiles too large to stage both components at once: the real parts, then the
// imaginary parts, go through a scalar LDS buffer of 2^TB (+ padding) values.
template <typename T, int R, int RB, int SA, int SB>
__device__ __forceinline__ void relayout_one(T (&v)[R], T *lds, uint32_t tau) {
  const uint32_t ba = ldspad<RB>(lay_base<SA, RB>(tau));
  const uint32_t bb = ldspad<RB>(lay_base<SB, RB>(tau));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) lds[ba + ldspad<RB>(lay_off<SA, RB>(r))] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = lds[bb + ldspad<RB>(lay_off<SB, RB>(r))];
}
template <typename T, int R, int RB, int SA, int SB>
__device__ __forceinline__ void relayout_split(T (&re)[R], T (&im)[R], T *lds, uint32_t tau) {
  relayout_one<T, R, RB, SA, SB>(re, lds, tau);
  relayout_one<T, R, RB, SA, SB>(im, lds, tau);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8).  This
// maps b in [0, n) to a tile so that XCD k takes the k-th contiguous share of [0, n) (a bijection
// for every n; shares differ by at most one tile): neighbouring tiles, which share cache lines of
// the exchange rows, are then read through the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t k = b & 7, m = b >> 3;
  int64_t start = 0;
  for (int64_t i = 0; i < k; ++i) start += (n - i + 7) >> 3;
  return start + m;
}

// Deterministic sum over aligned segments of SEG consecutive threads (SEG a power of two dividing
// NT).  Returns the segment total in the first thread of each segment (other threads: partial).
// lds must hold NT/64 doubles per value.
template <int NT, int SEG>
__device__ __forceinline__ double seg_sum(double v, double *lds, uint32_t tau) {
  constexpr int WSEG = SEG < 64 ? SEG : 64;
#pragma unroll
  for (int off = 1; off < WSEG; off <<= 1) v += __shfl_xor(v, off, 64);
  if constexpr (SEG > 64) {
    constexpr int NW = SEG / 64;
    __syncthreads();
    if ((tau & 63u) == 0) lds[tau >> 6] = v;
    __syncthreads();
    if ((tau & (SEG - 1)) == 0) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += lds[(tau >> 6) + w];
      v = s;
    }
  }
  return v;
}

// Arguments describing the Renyi indices of one call (passed by value to kernels).
struct QArgs {
  int nq;
  double q[HM_MAX_Q];
};

// Per-real-value accumulation of the reduction of Algorithm 2: t = x^2 = |<P>|^2 (folded form),
// acc[0] += t, acc[1+i] += t^{q_i} (q_i == 1: t log2 t).
template <typename T, int QM> struct Acc {
  static constexpr int N = (QM == 2) ? 2 : HM_MAX_Q + 1;
  T a[N];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = T(0);
  }
  __device__ __forceinline__ void add(T x, const QArgs &qa) {
    const T t = x * x;
    a[0] += t;
    if constexpr (QM == 2) {
      a[1] = fmaT(t, t, a[1]);
    } else {
#pragma unroll
      for (int i = 0; i < HM_MAX_Q; ++i) {
        if (i < qa.nq) {
          const double q = qa.q[i];
          T v;
          if (q == 1.0) v = t > T(0) ? t * (T)log2(t) : T(0);
          else if (q == 2.0) v = t * t;
          else if (q == 3.0) v = t * t * t;
          else if (q == 4.0) { T t2 = t * t; v = t2 * t2; }
          else v = t > T(0) ? (T)pow(t, (T)q) : T(0);
          a[1 + i] += v;
        }
      }
    }
  }
};

// Scale folded per-shift sums to the unfolded convention: a != 0 shifts were folded on one bit,
// |chi|^2 = f t with f = 4; the a == 0 shift is folded without the factor (f = 1).
__device__ __forceinline__ void unfold_scale(double *s, int nacc, const QArgs &qa, bool a_is_zero) {
  if (a_is_zero) return;
  const double f = 4.0;
  const double s0 = s[0];
  s[0] = f * s0;
  for (int i = 0; i < qa.nq && 1 + i < nacc; ++i) {
    const double q = qa.q[i];
    if (q == 1.0) s[1 + i] = f * (s[1 + i] + 2.0 * s0);  // f (sum t log2 t + log2(f) sum t)
    else s[1 + i] = exp2(2.0 * q) * s[1 + i];
  }
}

}  // namespace hm
