// hm_mana.hip -- gfx950 kernels for the mana of a pure qutrit state (Algorithm 4 of "Computing
// quantum magic of state vectors", Eqs. mana_FT, F3_unnorm_def).
//
// For a shift a in Z_3^N, alpha = X_a psi (alpha_x = psi_{x (-) a}, digit-wise mod 3),
// v_x = conj(alpha_x) alpha_{-x} and chi(a) = F_3^{(x)N} v with (F_3)_{jk} = omega^{2jk}.
// Because v_{-x} = conj(v_x), every chi_b(a) is real, so two shifts a, a' share one complex
// transform: F(v(a) + i v(a')) = chi(a) + i chi(a').  Each thread then accumulates, over its real
// values c: sum |c| (the mana sum), sum c and sum c^2 (normalisation and purity checks).
//
// Index layout: basis index x = sum_k x_k 3^k.  A row of 3^NL values holds the low NL trits; the
// radix-3 tile engine mirrors the qubit one: a thread holds R = 3^RT values whose index trits sit at
// positions [S, S+RT) of the row index, the thread's own index fills the other trits.  Strides in
// LDS are odd multiples of the element size, so no padding is needed against bank conflicts.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

__host__ __device__ constexpr int pow3c(int k) { return k <= 0 ? 1 : 3 * pow3c(k - 1); }
__host__ __device__ constexpr int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }
// largest power of 3 not above x (x >= 1)
__host__ __device__ constexpr int pow3floor(int x) { return x < 3 ? 1 : 3 * pow3floor(x / 3); }
// log3 of a power of 3
__host__ __device__ constexpr int log3c(int x) { return x < 3 ? 0 : 1 + log3c(x / 3); }

// Raw buffer view of n_bytes of global memory (gfx9 buffer descriptor: no stride, no format
// conversion).  Loads through it take a per-lane byte offset and a uniform byte offset (an SGPR), so
// an address that is a per-thread part plus a wave-uniform part costs no vector instruction; an
// offset past n_bytes reads zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void *p, uint32_t n_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n_bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld(float2 *, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double2 buf_ld(double2 *, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
// rows per row-pass tile: a power of 3 when rows are parts of a shift pair (WRITE), else as many
// whole rows (shift pairs) as the block holds
__host__ __device__ constexpr int mana_rows_per_tile(int NT, int TPR, bool write) {
  return write ? pow3floor(NT / TPR) : NT / TPR;
}

// digit-wise (x (-) a) mod 3 (neg = false) or ((-x) (-) a) mod 3 (neg = true) over k trits
__device__ __forceinline__ uint32_t dsub3(uint32_t x, uint32_t a, int k, bool neg) {
  uint32_t r = 0, p = 1;
  for (int i = 0; i < k; ++i) {
    const uint32_t xd = x % 3u, ad = a % 3u;
    x /= 3u;
    a /= 3u;
    const uint32_t d = neg ? (6u - xd - ad) % 3u : (3u + xd - ad) % 3u;
    r += d * p;
    p *= 3u;
  }
  return r;
}

// Radix-3 butterflies (F_3 with omega^{2jk}) over register trits [K0, K1) of R = 3^RT values.
template <typename T, int RT, int K0, int K1>
__device__ __forceinline__ void f3_regs(T (&re)[pow3c(RT)], T (&im)[pow3c(RT)]) {
  constexpr int R = pow3c(RT);
  const T c = T(0.86602540378443864676372317075294);  // sqrt(3)/2
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const int st = pow3c(k);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if ((i / st) % 3 == 0) {
        const int i1 = i + st, i2 = i + 2 * st;
        const T sr = re[i1] + re[i2], si = im[i1] + im[i2];
        const T dr = re[i1] - re[i2], di = im[i1] - im[i2];
        const T tr = fmaT(T(-0.5), sr, re[i]), ti = fmaT(T(-0.5), si, im[i]);
        re[i] = re[i] + sr;
        im[i] = im[i] + si;
        re[i1] = fmaT(c, di, tr);
        im[i1] = fmaT(-c, dr, ti);
        re[i2] = fmaT(-c, di, tr);
        im[i2] = fmaT(c, dr, ti);
      }
    }
  }
}

// row-local index of register rho for thread tp (thread index within its row) in layout S
template <int RT, int S>
__device__ __forceinline__ uint32_t lay3(uint32_t tp, uint32_t rho) {
  constexpr uint32_t P = pow3c(S);
  return (tp % P) + P * (rho + (uint32_t)pow3c(RT) * (tp / P));
}

// ------------------------------------------------------------------------------------------------
struct ManaRowArgs {
  const void *psi;
  int N;               // qutrits
  int nh;              // row-index trits per shift pair (0: workgroup-resident)
  uint32_t nhr;        // 3^nh rows per pair
  int64_t n_pairs;     // pairs in this launch
  uint64_t a0;         // first shift of pair 0
  uint64_t a_end;      // shifts >= a_end are absent
  void *exch;          // WRITE: [n_pairs][3^nh][3^NL]
  double *acc;         // REDUCE: per-block accumulators [gridDim][3], accumulated across launches
  int64_t n_tiles;
};

__host__ __device__ constexpr int mr_S(int NL, int RT, int k) { return imax(NL - RT * (k + 1), 0); }
__host__ __device__ constexpr int mr_H(int NL, int RT, int k) { return imin(RT, NL - RT * k); }

template <typename T, int RT, int SA, int SB, int ROWLEN>
__device__ __forceinline__ void relayout3(T (&re)[pow3c(RT)], T (&im)[pow3c(RT)], vec2<T> *lds, uint32_t g,
                                          uint32_t tp, bool act) {
  constexpr int R = pow3c(RT);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vec2<T> v;
      v.x = re[r];
      v.y = im[r];
      lds[g * ROWLEN + lay3<RT, SA>(tp, (uint32_t)r)] = v;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const vec2<T> v = lds[g * ROWLEN + lay3<RT, SB>(tp, (uint32_t)r)];
      re[r] = v.x;
      im[r] = v.y;
    }
  }
}

// The same, one component at a time through a scalar LDS buffer (half the LDS per workgroup).
template <typename T, int RT, int SA, int SB, int ROWLEN>
__device__ __forceinline__ void relayout3_one(T (&v)[pow3c(RT)], T *lds, uint32_t g, uint32_t tp, bool act) {
  constexpr int R = pow3c(RT);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) lds[g * ROWLEN + lay3<RT, SA>(tp, (uint32_t)r)] = v[r];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[g * ROWLEN + lay3<RT, SB>(tp, (uint32_t)r)];
  }
}
template <typename T, int RT, int SA, int SB, int ROWLEN>
__device__ __forceinline__ void relayout3_split(T (&re)[pow3c(RT)], T (&im)[pow3c(RT)], T *lds, uint32_t g,
                                                uint32_t tp, bool act) {
  relayout3_one<T, RT, SA, SB, ROWLEN>(re, lds, g, tp, act);
  relayout3_one<T, RT, SA, SB, ROWLEN>(im, lds, g, tp, act);
}
// Complex or split staging by a compile-time switch.
template <typename T, int RT, int SA, int SB, int ROWLEN, bool SPLIT, typename E>
__device__ __forceinline__ void relayout3_any(T (&re)[pow3c(RT)], T (&im)[pow3c(RT)], E *lds, uint32_t g, uint32_t tp,
                                              bool act) {
  if constexpr (SPLIT) relayout3_split<T, RT, SA, SB, ROWLEN>(re, im, lds, g, tp, act);
  else relayout3<T, RT, SA, SB, ROWLEN>(re, im, lds, g, tp, act);
}

// Block-wide FP64 sum of three per-thread values into acc[blockIdx] (added to what is there).
template <int NT>
__device__ __forceinline__ void block_acc3(double v0, double v1, double v2, double *red, double *acc, uint32_t tau) {
  double v[3] = {v0, v1, v2};
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = seg_sum<NT, NT>(v[k], red + k * (NT / 64 + 1), tau);
  if (tau == 0) {
    double *a = acc + (size_t)blockIdx.x * 3;
    a[0] += v[0];
    a[1] += v[1];
    a[2] += v[2];
  }
}

// Workgroup-resident tiles (n <= 8 for FP32, 7 for FP64): each row of G rows per tile is the whole
// vector of one shift pair, transformed and reduced in the workgroup.
template <typename T, int NT, int RT, int NL>
__global__ __launch_bounds__(NT) void k_mana_rowpass(ManaRowArgs A) {
  constexpr int R = pow3c(RT);
  constexpr int ROWLEN = pow3c(NL);
  constexpr int TPR = pow3c(NL - RT);         // threads per row
  constexpr int G = mana_rows_per_tile(NT, TPR, false);
  static_assert(NL >= RT && G >= 1, "tile shape");
  constexpr int S0 = NL - RT;
  constexpr int K = (NL + RT - 1) / RT;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = K > 1 ? G * ROWLEN : 1;

  __shared__ vec2<T> lds[LDS_N];
  __shared__ double red[3 * (NT / 64 + 1)];

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  const uint32_t tau = threadIdx.x;
  const uint32_t g = tau / TPR;
  const uint32_t tp = tau % TPR;
  const bool tact = g < (uint32_t)G;
  double m_acc = 0.0, s_acc = 0.0, q_acc = 0.0;

  for (int64_t b = blockIdx.x; b < A.n_tiles; b += gridDim.x) {
    const int64_t pair = b * G + g;
    const bool active = tact && pair < A.n_pairs;
    T re[R], im[R];
#pragma unroll
    for (int r = 0; r < R; ++r) re[r] = im[r] = T(0);
    if (active) {
#pragma unroll
      for (int which = 0; which < 2; ++which) {
        const uint64_t a64 = A.a0 + 2 * (uint64_t)pair + which;
        if (a64 >= A.a_end) continue;
        const uint32_t al = (uint32_t)a64;
        const uint32_t alo = al % (uint32_t)pow3c(S0), ahi = al / (uint32_t)pow3c(S0);
        const uint32_t xm = dsub3(tp, alo, S0, false);
        const uint32_t xn = dsub3(tp, alo, S0, true);
        // Register trit i of r contributes ((r_i - h_i) mod 3) 3^(S0+i) to the index of alpha_x and
        // ((-r_i - h_i) mod 3) 3^(S0+i) to that of alpha_{-x} (h = ahi).
        uint32_t om[RT][3], on[RT][3];
        {
          uint32_t h = ahi, p = (uint32_t)pow3c(S0);
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            const uint32_t hd = h % 3u;
            h /= 3u;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
              om[i][t] = ((3u + (uint32_t)t - hd) % 3u) * p;
              on[i][t] = ((6u - (uint32_t)t - hd) % 3u) * p;
            }
            p *= 3u;
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          uint32_t rm = 0, rn = 0;
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            const int t = (r / pow3c(i)) % 3;
            rm += om[i][t];
            rn += on[i][t];
          }
          const vec2<T> p = ld32(psi, xm + rm);  // alpha_x
          const vec2<T> q = ld32(psi, xn + rn);  // alpha_{-x}
          const T vr = fmaT(p.x, q.x, p.y * q.y);   // conj(p) q
          const T vi = fmaT(p.x, q.y, -(p.y * q.x));
          if (which == 0) {
            re[r] += vr;
            im[r] += vi;
          } else {  // + i v(a')
            re[r] -= vi;
            im[r] += vr;
          }
        }
      }
    }
    if constexpr (K >= 1) f3_regs<T, RT, 0, mr_H(NL, RT, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout3<T, RT, mr_S(NL, RT, 0), mr_S(NL, RT, 1), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout3<T, RT, mr_S(NL, RT, 1), mr_S(NL, RT, 2), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout3<T, RT, mr_S(NL, RT, 2), mr_S(NL, RT, 3), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 3)>(re, im);
    }
    T m = T(0), s = T(0), q = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      m += fabs(re[r]) + fabs(im[r]);
      s += re[r] + im[r];
      q = fmaT(re[r], re[r], fmaT(im[r], im[r], q));
    }
    m_acc += (double)m;
    s_acc += (double)s;
    q_acc += (double)q;
  }
  block_acc3<NT>(m_acc, s_acc, q_acc, red, A.acc, tau);
}

// ------------------------------------------------------------------------------------------------
// Two-pass row pass: for one shift pair (a, a + 1) and G consecutive rows xh of 3^NL values, the
// packed product v(a) + i v(a + 1) of each row followed by the NL radix-3 stages over the row index,
// written to the exchange buffer.
//
// The shift pair is uniform over the workgroup, so the source index of every register splits into
//   (row part: depends on the thread's row g) + (thread part: the thread's low S0 trits)
//   + (register part: the register's trits minus the shift's digits, the same for every lane),
// where every part is digit-wise (x - a) mod 3 or (-x - a) mod 3.  The register part is computed
// with scalar instructions and enters the loads as their uniform offset; the row and thread parts
// come from per-thread tables of the three possible digit results per trit (8 bits each), one
// bit-field extract per trit and shift.  So each packed value costs two loads per shift and no
// vector instruction for its address.
struct ManaWriteArgs {
  const void *psi;
  uint32_t psi_bytes;  // 3^N values
  int nhq;             // row-index trits above the tile's G rows (nh - log3 G)
  uint32_t nhr;        // 3^nh rows per pair
  int64_t n_pairs;     // pairs in this launch
  uint64_t a0;         // first shift of pair 0
  uint64_t a_end;      // shifts >= a_end are absent
  void *exch;          // [n_pairs][3^nh][3^NL]
  int64_t n_tiles;     // (3^nh / G) * n_pairs
};

// Table of the three results ((x - h) mod 3) p (neg: ((-x - h) mod 3) p) for h = 0, 1, 2, 8 bits each.
__device__ __forceinline__ uint32_t trit_table(uint32_t x, uint32_t p, bool neg) {
  uint32_t t = 0;
#pragma unroll
  for (uint32_t h = 0; h < 3; ++h) t |= ((neg ? (6u - x - h) : (3u + x - h)) % 3u) * p << (8u * h);
  return t;
}

// Register budget of the FP32 two-pass kernels: at least four waves per SIMD (row pass 118 and
// column pass 96 VGPRs, no spills; measured at n = 12 on MI355X: row pass 74.3 -> 71.3 us, column
// pass 38.2 -> 37.7 us per launch against the compiler's own budget; five or more waves spill).
template <typename T> struct ManaWaves {
  static constexpr int row = sizeof(T) == 4 ? 4 : 1;
  static constexpr int col = sizeof(T) == 4 ? 4 : 1;
};

template <typename T, int NT, int RT, int NL>
__global__ __launch_bounds__(NT, ManaWaves<T>::row) void k_mana_rowwrite(ManaWriteArgs A) {
  constexpr int R = pow3c(RT);
  constexpr int ROWLEN = pow3c(NL);
  constexpr int S0 = NL - RT;                // thread trits of the first layout
  constexpr int TPR = pow3c(S0);             // threads per row
  constexpr int G = mana_rows_per_tile(NT, TPR, true);
  constexpr int LG = log3c(G);
  static_assert(NL >= RT && G >= 1 && pow3c(LG) == G, "tile shape");
  static_assert(S0 <= 5 && LG <= 5, "8-bit digit tables");
  constexpr int K = (NL + RT - 1) / RT;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = K > 1 ? G * ROWLEN : 1;
  constexpr uint32_t VB = sizeof(vec2<T>);

  __shared__ T lds[LDS_N];

  const uint32_t tau = threadIdx.x;
  const uint32_t g = tau / TPR;
  const uint32_t tp = tau % TPR;
  const bool tact = g < (uint32_t)G;
  const __amdgpu_buffer_rsrc_t rs = buf_view(A.psi, A.psi_bytes);

  uint32_t tm[S0 > 0 ? S0 : 1], tn[S0 > 0 ? S0 : 1], gm[LG > 0 ? LG : 1], gn[LG > 0 ? LG : 1];
  {
    uint32_t x = tp, p = 1;
#pragma unroll
    for (int i = 0; i < S0; ++i, p *= 3u, x /= 3u) {
      tm[i] = trit_table(x % 3u, p, false);
      tn[i] = trit_table(x % 3u, p, true);
    }
    x = g;
    p = 1;
#pragma unroll
    for (int i = 0; i < LG; ++i, p *= 3u, x /= 3u) {
      gm[i] = trit_table(x % 3u, p, false);
      gn[i] = trit_table(x % 3u, p, true);
    }
  }

  // Per-shift address parts: lane byte offsets (row and thread parts) of alpha_x and alpha_{-x}, and
  // the uniform byte offsets of each register trit's three digit values.
  struct Shift {
    uint32_t vm, vn;
    uint32_t cm[RT][3], cn[RT][3];
  };
  auto shift_parts = [&](uint64_t a64, int64_t xb, Shift &S) {
    const uint32_t a = (uint32_t)a64;
    const uint32_t ah = a / (uint32_t)ROWLEN, al = a % (uint32_t)ROWLEN;
    // row part: xh = xb G + g, so (xh - ah) digit-wise = G (xb - ah / G) + (g - ah mod G)
    uint32_t rqm = 0, rqn = 0;
    {
      uint32_t x = (uint32_t)xb, h = ah / (uint32_t)G, p = 1;
      for (int i = 0; i < A.nhq; ++i, p *= 3u, x /= 3u, h /= 3u) {
        const uint32_t xd = x % 3u, hd = h % 3u;
        rqm += ((3u + xd - hd) % 3u) * p;
        rqn += ((6u - xd - hd) % 3u) * p;
      }
    }
    uint32_t rm = 0, rn = 0;
    {
      uint32_t h = ah;
#pragma unroll
      for (int i = 0; i < LG; ++i, h /= 3u) {
        const uint32_t sh = 8u * (h % 3u);
        rm += __builtin_amdgcn_ubfe(gm[i], sh, 8);
        rn += __builtin_amdgcn_ubfe(gn[i], sh, 8);
      }
    }
    uint32_t xm = 0, xn = 0;
    {
      uint32_t h = al;
#pragma unroll
      for (int i = 0; i < S0; ++i, h /= 3u) {
        const uint32_t sh = 8u * (h % 3u);
        xm += __builtin_amdgcn_ubfe(tm[i], sh, 8);
        xn += __builtin_amdgcn_ubfe(tn[i], sh, 8);
      }
    }
    S.vm = ((rqm * (uint32_t)G + rm) * (uint32_t)ROWLEN + xm) * VB;
    S.vn = ((rqn * (uint32_t)G + rn) * (uint32_t)ROWLEN + xn) * VB;
    uint32_t h = al / (uint32_t)TPR, p = (uint32_t)TPR * VB;
#pragma unroll
    for (int i = 0; i < RT; ++i, p *= 3u, h /= 3u) {
      const uint32_t hd = h % 3u;
#pragma unroll
      for (uint32_t t = 0; t < 3; ++t) {
        S.cm[i][t] = ((3u + t - hd) % 3u) * p;
        S.cn[i][t] = ((6u - t - hd) % 3u) * p;
      }
    }
  };

  vec2<T> *ex = (vec2<T> *)A.exch;
  for (int64_t b = blockIdx.x; b < A.n_tiles; b += gridDim.x) {
    const int64_t tile = xcd_tile(b, A.n_tiles);  // gridDim is a multiple of 8
    const int64_t xb = tile / A.n_pairs;          // row block (uniform)
    const int64_t pair = tile - xb * A.n_pairs;   // shift pair (uniform)
    const uint64_t a_first = A.a0 + 2 * (uint64_t)pair;
    const bool two = a_first + 1 < A.a_end;
    T re[R], im[R];
    if (tact) {
      Shift S0s, S1s;
      shift_parts(a_first, xb, S0s);
      if (two) {
        shift_parts(a_first + 1, xb, S1s);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          uint32_t om0 = 0, on0 = 0, om1 = 0, on1 = 0;
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            const int t = (r / pow3c(i)) % 3;
            om0 += S0s.cm[i][t];
            on0 += S0s.cn[i][t];
            om1 += S1s.cm[i][t];
            on1 += S1s.cn[i][t];
          }
          const vec2<T> p0 = buf_ld((vec2<T> *)nullptr, rs, S0s.vm, om0);  // alpha_x of a
          const vec2<T> q0 = buf_ld((vec2<T> *)nullptr, rs, S0s.vn, on0);  // alpha_{-x} of a
          const vec2<T> p1 = buf_ld((vec2<T> *)nullptr, rs, S1s.vm, om1);  // the same for a + 1
          const vec2<T> q1 = buf_ld((vec2<T> *)nullptr, rs, S1s.vn, on1);
          // conj(p0) q0 + i conj(p1) q1
          re[r] = fmaT(-p1.x, q1.y, fmaT(p1.y, q1.x, fmaT(p0.x, q0.x, p0.y * q0.y)));
          im[r] = fmaT(p1.x, q1.x, fmaT(p1.y, q1.y, fmaT(p0.x, q0.y, -(p0.y * q0.x))));
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          uint32_t om0 = 0, on0 = 0;
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            const int t = (r / pow3c(i)) % 3;
            om0 += S0s.cm[i][t];
            on0 += S0s.cn[i][t];
          }
          const vec2<T> p0 = buf_ld((vec2<T> *)nullptr, rs, S0s.vm, om0);
          const vec2<T> q0 = buf_ld((vec2<T> *)nullptr, rs, S0s.vn, on0);
          re[r] = fmaT(p0.x, q0.x, p0.y * q0.y);
          im[r] = fmaT(p0.x, q0.y, -(p0.y * q0.x));
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) re[r] = im[r] = T(0);
    }
    if constexpr (K >= 1) f3_regs<T, RT, 0, mr_H(NL, RT, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout3_split<T, RT, mr_S(NL, RT, 0), mr_S(NL, RT, 1), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout3_split<T, RT, mr_S(NL, RT, 1), mr_S(NL, RT, 2), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout3_split<T, RT, mr_S(NL, RT, 2), mr_S(NL, RT, 3), ROWLEN>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 3)>(re, im);
    }
    // Final layout S = 0: register r holds row position r + R * tp; stored at column r * TPR + tp
    // (a fixed column permutation) so that consecutive threads write consecutive addresses.
    if (tact) {
      const uint32_t xh = (uint32_t)xb * (uint32_t)G + g;
      const uint32_t ob = ((uint32_t)pair * A.nhr + xh) * ROWLEN + tp;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vec2<T> v;
        v.x = re[r];
        v.y = im[r];
        st32(ex, ob + (uint32_t)r * TPR, v);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
struct ManaColArgs {
  const void *exch;    // [n_pairs][3^NH][3^nl]
  uint32_t rowlen;     // 3^nl
  int64_t n_pairs;
  int64_t n_cb;        // column blocks per pair
  double *acc;         // per-block accumulators [gridDim][3]
  int64_t n_tiles;
};

__host__ __device__ constexpr int mc_S(int NH, int RT, int CT, int k) { return CT + imin(RT * k, NH - RT); }
__host__ __device__ constexpr int mc_L(int NH, int RT, int CT, int k) { return RT * k + CT - mc_S(NH, RT, CT, k); }
__host__ __device__ constexpr int mc_H(int NH, int RT, int CT, int k) {
  return imin(RT * (k + 1), NH) + CT - mc_S(NH, RT, CT, k);
}

// tile-local index (column trits first, then row trits) of register rho for thread tau in layout S
template <int RT, int S>
__device__ __forceinline__ uint32_t lay3t(uint32_t tau, uint32_t rho) { return lay3<RT, S>(tau, rho); }

// Column tiles stage through LDS one component at a time (half the LDS, more workgroups per CU).
template <typename T, int NT, int RT, int NH, int CT>
__global__ __launch_bounds__(NT, ManaWaves<T>::col) void k_mana_colpass(ManaColArgs A) {
  constexpr int R = pow3c(RT);
  constexpr int C = pow3c(CT);
  constexpr int TILE = pow3c(NH + CT);
  constexpr int NACT = TILE / R;  // active threads
  static_assert(NACT <= NT && NH >= RT, "column tile shape");
  constexpr int K = (NH + RT - 1) / RT;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = K > 1 ? TILE : 1;

  __shared__ T lds[LDS_N];
  __shared__ double red[3 * (NT / 64 + 1)];

  const vec2<T> *__restrict__ ex = (const vec2<T> *)A.exch;
  const uint32_t tau = threadIdx.x;
  const bool tact = tau < (uint32_t)NACT;
  const uint32_t col = tau % C;
  const uint32_t rowhi = tau / C;
  double m_acc = 0.0, s_acc = 0.0, q_acc = 0.0;

  for (int64_t b = blockIdx.x; b < A.n_tiles; b += gridDim.x) {
    const int64_t tile = xcd_tile(b, A.n_tiles);  // gridDim is a multiple of 8
    const int64_t pair = tile / A.n_cb;
    const int64_t cb = tile - pair * A.n_cb;
    T re[R], im[R];
    if (tact) {
      const uint32_t base = (uint32_t)pair * (uint32_t)pow3c(NH) * A.rowlen + (uint32_t)cb * C + col;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t row = (uint32_t)r + (uint32_t)R * rowhi;
        const vec2<T> v = ld32(ex, base + row * A.rowlen);
        re[r] = v.x;
        im[r] = v.y;
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) re[r] = im[r] = T(0);
    }
    f3_regs<T, RT, mc_L(NH, RT, CT, 0), mc_H(NH, RT, CT, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout3_split<T, RT, mc_S(NH, RT, CT, 0), mc_S(NH, RT, CT, 1), 0>(re, im, lds, 0, tau, tact);
      f3_regs<T, RT, mc_L(NH, RT, CT, 1), mc_H(NH, RT, CT, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout3_split<T, RT, mc_S(NH, RT, CT, 1), mc_S(NH, RT, CT, 2), 0>(re, im, lds, 0, tau, tact);
      f3_regs<T, RT, mc_L(NH, RT, CT, 2), mc_H(NH, RT, CT, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout3_split<T, RT, mc_S(NH, RT, CT, 2), mc_S(NH, RT, CT, 3), 0>(re, im, lds, 0, tau, tact);
      f3_regs<T, RT, mc_L(NH, RT, CT, 3), mc_H(NH, RT, CT, 3)>(re, im);
    }
    if (tact) {
      T m = T(0), s = T(0), q = T(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        m += fabs(re[r]) + fabs(im[r]);
        s += re[r] + im[r];
        q = fmaT(re[r], re[r], fmaT(im[r], im[r], q));
      }
      m_acc += (double)m;
      s_acc += (double)s;
      q_acc += (double)q;
    }
  }
  block_acc3<NT>(m_acc, s_acc, q_acc, red, A.acc, tau);
}

__global__ void k_mana_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Fixed-order sum of the per-block accumulators; sums = {m, sum chi, sum chi^2}; out = finalised.
__global__ __launch_bounds__(256) void k_mana_total(const double *acc, int64_t nblk, int N, double *sums, double *out) {
  __shared__ double red[256];
  __shared__ double tot[3];
  const uint32_t t = threadIdx.x;
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int64_t i = t; i < nblk; i += 256) s += acc[i * 3 + k];
    red[t] = s;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) tot[k] = red[0];
    __syncthreads();
  }
  if (t == 0) {
    if (sums)
      for (int k = 0; k < 3; ++k) sums[k] = tot[k];
    if (out) {
      double D = 1.0;
      for (int i = 0; i < N; ++i) D *= 3.0;
      out[0] = log2(tot[0] / D);  // Eq. mana2: log2(sum_u |<psi|A_u|psi>| / 3^N)
      out[1] = tot[1] / D;        // sum_u W(u)
      out[2] = tot[2] / D;        // 3^N sum_u W(u)^2
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
static constexpr int MANA_NT = 256;
static constexpr int MANA_GRID = 2048;  // fixed grid: per-block accumulators live across launches

struct ManaPlan {
  int N, dbl, path, nl, nh;
  int RT;   // register trits of the resident kernel (path 1) or of both two-pass kernels (path 2)
  int batch_pairs;
  int lanes;  // two-pass batches alternate over this many streams (own exchange and accumulators)
};

// Two-pass default: one lane.  Two lanes let the VALU-bound row pass of one batch overlap the
// memory-bound column pass of the other, but measured no faster at n = 12 (645 ms with 44-shift
// batches against 641 ms on one stream; 713 ms with two 192 MiB exchanges, which no longer fit the
// memory-side cache together).
static constexpr int MANA_STREAMS_DEFAULT = 1;

// batch: X-shifts per two-pass launch pair (0 = 192 MiB of exchange); streams: 0 (default), 1, 2.
// Two-pass tiles: rows of 3^nl values (nl <= 8), columns of 3^nh (nh <= 8); FP32 holds 3^3 values
// per thread, FP64 3^2 up to rows and columns of 3^7 and 3^3 at n = 15, 16.
static int mana_plan(int N, int dbl, int64_t batch, int streams, ManaPlan *p) {
  if (streams < 0 || streams > 2) return fail(E_ARG, "mana: streams = %d outside [0, 2]", streams);
  if (N < 1 || N > 16) return fail(E_SIZE, "mana: n = %d outside [1, 16]", N);
  ManaPlan P{};
  P.N = N;
  P.dbl = dbl;
  P.lanes = 1;
  P.RT = dbl ? 2 : 3;
  if (N < P.RT) P.RT = N;  // tiny states: one thread holds a whole vector
  const int onepass_max = dbl ? 7 : 8;  // one row of 3^N values per <= 243 threads
  if (N <= onepass_max) {
    P.path = 1;
    P.nl = N;
    P.nh = 0;
  } else {
    P.path = 2;
    if (dbl && N >= 15) P.RT = 3;
    const int row_max = P.RT == 3 ? 8 : 7;
    int nl = (N + 1) / 2, nh = N - nl;
    if (nl > row_max) nl = row_max, nh = N - nl;
    if (nh > row_max || nh < P.RT) return fail(E_SIZE, "mana: no two-pass split for n = %d", N);
    P.nl = nl;
    P.nh = nh;
    const size_t per_pair = (size_t)pow3c(N) * (dbl ? 16 : 8);
    // Untuned: 192 MiB of exchange per launch pair, inside the 256 MiB memory-side cache (at n = 12
    // on MI355X: 0.66 s against 0.68 s at 256 MiB and 0.77-0.79 s at 512 MiB - 1 GiB).
    int64_t b = batch > 0 ? (batch + 1) / 2 : (int64_t)((192ull << 20) / per_pair);
    if ((size_t)b * per_pair > (3ull << 30)) b = (int64_t)((3ull << 30) / per_pair);  // 32-bit offsets
    if (b < 1) b = 1;
    P.batch_pairs = (int)b;
    P.lanes = streams ? streams : MANA_STREAMS_DEFAULT;
  }
  *p = P;
  return OK;
}

static size_t mana_acc_bytes(const ManaPlan &P) { return align256((size_t)MANA_GRID * 3 * sizeof(double)); }

// [row accumulators][column accumulators x lanes][exchange x lanes]
int mana_workspace(int N, int dbl, int64_t batch, int streams, size_t *bytes) {
  ManaPlan P;
  const int e = mana_plan(N, dbl, batch, streams, &P);
  if (e) return e;
  size_t b = mana_acc_bytes(P) * (1 + P.lanes);
  if (P.path == 2) b += (size_t)P.lanes * align256((size_t)P.batch_pairs * (size_t)pow3c(N) * (dbl ? 16 : 8));
  *bytes = b;
  return OK;
}

template <typename T, int RT, int NL>
static void launch_mana_resident_nl(ManaRowArgs A, hipStream_t st) {
  constexpr int G = mana_rows_per_tile(MANA_NT, pow3c(NL - RT), false);
  A.n_tiles = (A.n_pairs + G - 1) / G;
  ProfScope prof("mana_rowpass_resident", st);
  hipLaunchKernelGGL((k_mana_rowpass<T, MANA_NT, RT, NL>), dim3(MANA_GRID), dim3(MANA_NT), 0, st, A);
}

template <typename T, int RT>
static int launch_mana_resident(int NL, ManaRowArgs A, hipStream_t st) {
#define HM_MROW(nl)                                  \
  case nl:                                           \
    launch_mana_resident_nl<T, RT, nl>(A, st);       \
    return OK;
  if constexpr (RT == 3) {
    switch (NL) { HM_MROW(3) HM_MROW(4) HM_MROW(5) HM_MROW(6) HM_MROW(7) HM_MROW(8) default: break; }
  } else if constexpr (RT == 2) {
    switch (NL) { HM_MROW(2) HM_MROW(3) HM_MROW(4) HM_MROW(5) HM_MROW(6) HM_MROW(7) default: break; }
  } else {
    switch (NL) { HM_MROW(1) default: break; }
  }
#undef HM_MROW
  return fail(E_UNSUPPORTED, "mana: no resident kernel for 3^%d values (RT %d)", NL, RT);
}

template <typename T, int RT, int NL>
static int launch_mana_write_nl(ManaWriteArgs A, int nh, hipStream_t st) {
  constexpr int G = mana_rows_per_tile(MANA_NT, pow3c(NL - RT), true);
  constexpr int LG = log3c(G);
  if (nh < LG) return fail(E_UNSUPPORTED, "mana: 3^%d rows per pair, fewer than one tile of %d rows", nh, G);
  A.nhq = nh - LG;
  A.n_tiles = (int64_t)(A.nhr / (uint32_t)G) * A.n_pairs;
  ProfScope prof("mana_rowpass_write", st);
  hipLaunchKernelGGL((k_mana_rowwrite<T, MANA_NT, RT, NL>), dim3(MANA_GRID), dim3(MANA_NT), 0, st, A);
  return OK;
}

template <typename T, int RT>
static int launch_mana_write(int NL, int nh, ManaWriteArgs A, hipStream_t st) {
#define HM_MWR(nl) \
  case nl:         \
    return launch_mana_write_nl<T, RT, nl>(A, nh, st);
  if constexpr (sizeof(T) == 4 && RT == 3) {
    switch (NL) { HM_MWR(4) HM_MWR(5) HM_MWR(6) HM_MWR(7) HM_MWR(8) default: break; }
  } else if constexpr (sizeof(T) == 8 && RT == 2) {
    switch (NL) { HM_MWR(4) HM_MWR(5) HM_MWR(6) HM_MWR(7) default: break; }
  } else if constexpr (sizeof(T) == 8 && RT == 3) {
    switch (NL) { HM_MWR(8) default: break; }
  }
#undef HM_MWR
  return fail(E_UNSUPPORTED, "mana: no row-pass kernel for rows of 3^%d (RT %d)", NL, RT);
}

template <typename T, int RT, int NH, int CT>
static int launch_mana_col_ct(ManaColArgs A, int nl, hipStream_t st) {
  if (nl < CT) return fail(E_UNSUPPORTED, "mana: rows of 3^%d shorter than column blocks of 3^%d", nl, CT);
  A.n_cb = pow3c(nl - CT);
  A.n_tiles = A.n_pairs * A.n_cb;
  ProfScope prof("mana_colpass", st);
  hipLaunchKernelGGL((k_mana_colpass<T, MANA_NT, RT, NH, CT>), dim3(MANA_GRID), dim3(MANA_NT), 0, st, A);
  return OK;
}

template <typename T, int RT>
static int launch_mana_col(int NH, int nl, ManaColArgs A, hipStream_t st) {
  // column blocks of C = 3^CT columns with 3^(NH-RT) * C <= 256 threads
#define HM_MCOL(nh)                                                   \
  case nh: {                                                          \
    constexpr int CT = (nh - RT >= 5) ? 0 : 5 - (nh - RT);            \
    return launch_mana_col_ct<T, RT, nh, CT>(A, nl, st);              \
  }
  if constexpr (sizeof(T) == 4 && RT == 3) {
    switch (NH) { HM_MCOL(3) HM_MCOL(4) HM_MCOL(5) HM_MCOL(6) HM_MCOL(7) HM_MCOL(8) default: break; }
  } else if constexpr (sizeof(T) == 8 && RT == 2) {
    switch (NH) { HM_MCOL(2) HM_MCOL(3) HM_MCOL(4) HM_MCOL(5) HM_MCOL(6) HM_MCOL(7) default: break; }
  } else if constexpr (sizeof(T) == 8 && RT == 3) {
    switch (NH) { HM_MCOL(7) HM_MCOL(8) default: break; }
  }
#undef HM_MCOL
  return fail(E_UNSUPPORTED, "mana: no column kernel for 3^%d rows", NH);
}

template <typename T>
static int mana_t(const ManaPlan &P, const void *psi, uint64_t a0, uint64_t a1, double *sums, double *out, void *ws,
                  hipStream_t st) {
  char *w = (char *)ws;
  const size_t accb = mana_acc_bytes(P);
  double *acc_row = (double *)w;
  double *acc_col = (double *)(w + accb);  // lane l: acc_col + l * MANA_GRID * 3 (contiguous)
  {
    const int64_t nz = (int64_t)(accb * (1 + P.lanes) / sizeof(double));
    hipLaunchKernelGGL(k_mana_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, acc_row, nz);
  }
  const int64_t n_pairs = (int64_t)((a1 - a0 + 1) / 2);
  int e = OK;
  if (P.path == 1) {
    ManaRowArgs A{};
    A.psi = psi;
    A.N = P.N;
    A.nh = 0;
    A.nhr = 1;
    A.n_pairs = n_pairs;
    A.a0 = a0;
    A.a_end = a1;
    A.acc = acc_row;
    if constexpr (sizeof(T) == 4) {
      if (P.RT == 3) e = launch_mana_resident<T, 3>(P.nl, A, st);
      else if (P.RT == 2) e = launch_mana_resident<T, 2>(P.nl, A, st);
      else e = launch_mana_resident<T, 1>(P.nl, A, st);
    } else {
      if (P.RT == 2) e = launch_mana_resident<T, 2>(P.nl, A, st);
      else e = launch_mana_resident<T, 1>(P.nl, A, st);
    }
    if (e) return e;
    hipLaunchKernelGGL(k_mana_total, dim3(1), dim3(256), 0, st, acc_row, (int64_t)MANA_GRID, P.N, sums, out);
    return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "mana launch: %s", hipGetErrorString(hipGetLastError()));
  }
  // Two-pass: batch k runs on lane k mod lanes (lane 0 = the caller's stream, lane 1 = the internal
  // side stream, forked after the zeroing and joined before the totals), with that lane's exchange
  // buffer and column accumulators, so lanes share no memory they write.
  const size_t xb = align256((size_t)P.batch_pairs * (size_t)pow3c(P.N) * (P.dbl ? 16 : 8));
  char *exch0 = w + accb * (1 + P.lanes);
  const int64_t n_batches = (n_pairs + P.batch_pairs - 1) / P.batch_pairs;
  const int L = (P.lanes > 1 && n_batches > 1) ? 2 : 1;
  hipStream_t lst[2] = {st, st};
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  if (L == 2) {
    if ((e = side_stream(&lst[1]))) return e;
    if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess) {
      if (ev_fork) (void)hipEventDestroy(ev_fork);
      return fail(E_HIP, "mana: event creation failed");
    }
    if (hipEventRecord(ev_fork, st) != hipSuccess || hipStreamWaitEvent(lst[1], ev_fork, 0) != hipSuccess) {
      (void)hipEventDestroy(ev_fork);
      (void)hipEventDestroy(ev_join);
      return fail(E_HIP, "mana: stream fork failed");
    }
  }
  for (int64_t k = 0; k < n_batches && !e; ++k) {
    const int l = (int)(k % L);
    const int64_t p0 = k * P.batch_pairs;
    const int64_t nb = (n_pairs - p0) < P.batch_pairs ? (n_pairs - p0) : P.batch_pairs;
    void *ex_l = exch0 + (size_t)l * xb;
    ManaWriteArgs A{};
    A.psi = psi;
    A.psi_bytes = (uint32_t)((size_t)pow3c(P.N) * sizeof(vec2<T>));
    A.nhr = (uint32_t)pow3c(P.nh);
    A.n_pairs = nb;
    A.a0 = a0 + 2 * (uint64_t)p0;
    A.a_end = a1;
    A.exch = ex_l;
    if (P.RT == 3) e = launch_mana_write<T, 3>(P.nl, P.nh, A, lst[l]);
    else e = launch_mana_write<T, 2>(P.nl, P.nh, A, lst[l]);
    if (e) break;
    ManaColArgs C{};
    C.exch = ex_l;
    C.rowlen = (uint32_t)pow3c(P.nl);
    C.n_pairs = nb;
    C.acc = acc_col + (size_t)l * MANA_GRID * 3;
    if (P.RT == 3) e = launch_mana_col<T, 3>(P.nh, P.nl, C, lst[l]);
    else e = launch_mana_col<T, 2>(P.nh, P.nl, C, lst[l]);
  }
  if (L == 2) {
    const bool ok = hipEventRecord(ev_join, lst[1]) == hipSuccess && hipStreamWaitEvent(st, ev_join, 0) == hipSuccess;
    (void)hipEventDestroy(ev_fork);
    (void)hipEventDestroy(ev_join);
    if (!ok && !e) e = fail(E_HIP, "mana: stream join failed");
  }
  if (e) return e;
  // fixed-order sum over the lanes' per-block accumulators (contiguous)
  hipLaunchKernelGGL(k_mana_total, dim3(1), dim3(256), 0, st, acc_col, (int64_t)MANA_GRID * P.lanes, P.N, sums, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "mana launch: %s", hipGetErrorString(hipGetLastError()));
}

int mana_launch(int N, int dbl, int64_t batch, int streams, const void *psi, uint64_t a0, uint64_t a1, double *sums,
                double *out, void *ws, size_t ws_bytes, hipStream_t st) {
  ManaPlan P;
  int e = mana_plan(N, dbl, batch, streams, &P);
  if (e) return e;
  size_t need = 0;
  if ((e = mana_workspace(N, dbl, batch, streams, &need))) return e;
  if (ws_bytes < need) return fail(E_WORKSPACE, "mana workspace too small");
  return dbl ? mana_t<double>(P, psi, a0, a1, sums, out, ws, st) : mana_t<float>(P, psi, a0, a1, sums, out, ws, st);
}

}  // namespace hm
