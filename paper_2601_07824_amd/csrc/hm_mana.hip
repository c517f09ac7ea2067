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

// Two-pass row tiles (WRITE) stage through LDS one component at a time.
template <typename T, int NT, int RT, int NL, bool WRITE>
__global__ __launch_bounds__(NT) void k_mana_rowpass(ManaRowArgs A) {
  constexpr bool SPLIT = WRITE;
  constexpr int R = pow3c(RT);
  constexpr int ROWLEN = pow3c(NL);
  constexpr int TPR = pow3c(NL - RT);         // threads per row
  constexpr int G = mana_rows_per_tile(NT, TPR, WRITE);
  static_assert(NL >= RT && G >= 1, "tile shape");
  constexpr int S0 = NL - RT;
  constexpr int K = (NL + RT - 1) / RT;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = K > 1 ? G * ROWLEN : 1;

  __shared__ typename std::conditional<SPLIT, T, vec2<T>>::type lds[LDS_N];
  __shared__ double red[3 * (NT / 64 + 1)];

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  const uint32_t tau = threadIdx.x;
  const uint32_t g = tau / TPR;
  const uint32_t tp = tau % TPR;
  const bool tact = g < (uint32_t)G;
  double m_acc = 0.0, s_acc = 0.0, q_acc = 0.0;

  // WRITE: row-tasks are numbered xh-major (rt = xh * n_pairs + pair) and each XCD takes a
  // contiguous share of the tiles, so an XCD works on a fixed set of rows xh for every shift pair of
  // the launch and reads a fixed eighth-or-so of the state through its L2.
  for (int64_t b = blockIdx.x; b < A.n_tiles; b += gridDim.x) {
    const int64_t tile = WRITE ? xcd_tile(b, A.n_tiles) : b;  // gridDim is a multiple of 8
    const int64_t rt = tile * G + g;
    int64_t pair;
    uint32_t xh;
    if constexpr (WRITE) {
      xh = (uint32_t)(rt / A.n_pairs);
      pair = rt - (int64_t)xh * A.n_pairs;
    } else {
      pair = rt / A.nhr;
      xh = (uint32_t)(rt - pair * A.nhr);
    }
    const bool active = tact && (WRITE ? rt < A.n_pairs * A.nhr : pair < A.n_pairs);
    T re[R], im[R];
#pragma unroll
    for (int r = 0; r < R; ++r) re[r] = im[r] = T(0);
    if (active) {
#pragma unroll
      for (int which = 0; which < 2; ++which) {
        const uint64_t a64 = A.a0 + 2 * (uint64_t)pair + which;
        if (a64 >= A.a_end) continue;
        const uint32_t a = (uint32_t)a64;
        const uint32_t ah = a / ROWLEN, al = a % ROWLEN;
        const uint32_t alo = al % (uint32_t)pow3c(S0), ahi = al / (uint32_t)pow3c(S0);
        const uint32_t xm = dsub3(xh, ah, A.nh, false) * ROWLEN + dsub3(tp, alo, S0, false);
        const uint32_t xn = dsub3(xh, ah, A.nh, true) * ROWLEN + dsub3(tp, alo, S0, true);
        // Register trit i of r contributes ((r_i - h_i) mod 3) 3^(S0+i) to the index of alpha_x and
        // ((-r_i - h_i) mod 3) 3^(S0+i) to that of alpha_{-x} (h = ahi): tables of the three
        // possible contributions per trit, so that each register's offset is a sum of table entries
        // picked by its (compile-time) digits.
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
      relayout3_any<T, RT, mr_S(NL, RT, 0), mr_S(NL, RT, 1), ROWLEN, SPLIT>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout3_any<T, RT, mr_S(NL, RT, 1), mr_S(NL, RT, 2), ROWLEN, SPLIT>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout3_any<T, RT, mr_S(NL, RT, 2), mr_S(NL, RT, 3), ROWLEN, SPLIT>(re, im, lds, g, tp, tact);
      f3_regs<T, RT, 0, mr_H(NL, RT, 3)>(re, im);
    }
    if constexpr (WRITE) {
      // Final layout S = 0: register r holds row position r + R * tp; stored at column r * TPR + tp
      // (a fixed column permutation) so that consecutive threads write consecutive addresses.
      if (active) {
        vec2<T> *ex = (vec2<T> *)A.exch;
        const uint32_t ob = ((uint32_t)pair * (uint32_t)A.nhr + xh) * ROWLEN + tp;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          vec2<T> v;
          v.x = re[r];
          v.y = im[r];
          st32(ex, ob + (uint32_t)r * TPR, v);
        }
      }
    } else {
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
  if constexpr (!WRITE) block_acc3<NT>(m_acc, s_acc, q_acc, red, A.acc, tau);
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
__global__ __launch_bounds__(NT) void k_mana_colpass(ManaColArgs A) {
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
  int N, dbl, path, nl, nh, RT, batch_pairs;
  int lanes;  // two-pass batches alternate over this many streams (own exchange and accumulators)
};

// Two-pass default: one lane.  Two lanes let the VALU-bound row pass of one batch overlap the
// memory-bound column pass of the other, but measured no faster at n = 12 (645 ms with 44-shift
// batches against 641 ms on one stream; 713 ms with two 192 MiB exchanges, which no longer fit the
// memory-side cache together).
static constexpr int MANA_STREAMS_DEFAULT = 1;

// batch: X-shifts per two-pass launch pair (0 = 192 MiB of exchange); streams: 0 (default), 1, 2.
static int mana_plan(int N, int dbl, int64_t batch, int streams, ManaPlan *p) {
  if (streams < 0 || streams > 2) return fail(E_ARG, "mana: streams = %d outside [0, 2]", streams);
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
    const int row_max = dbl ? 7 : 8;
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
size_t mana_workspace(int N, int dbl, int64_t batch, int streams, uint64_t n_shifts) {
  (void)n_shifts;
  ManaPlan P;
  if (N < 1 || N > 16 || mana_plan(N, dbl, batch, streams, &P) != OK) return 256;
  size_t b = mana_acc_bytes(P) * (1 + P.lanes);
  if (P.path == 2) b += (size_t)P.lanes * align256((size_t)P.batch_pairs * (size_t)pow3c(N) * (dbl ? 16 : 8));
  return b;
}

template <typename T, int RT, int NL, bool WRITE>
static void launch_mana_row_nl(ManaRowArgs A, hipStream_t st) {
  constexpr int G = mana_rows_per_tile(MANA_NT, pow3c(NL - RT), WRITE);
  const int64_t rts = A.n_pairs * (int64_t)A.nhr;
  A.n_tiles = (rts + G - 1) / G;
  ProfScope prof(WRITE ? "mana_rowpass_write" : "mana_rowpass_resident", st);
  hipLaunchKernelGGL((k_mana_rowpass<T, MANA_NT, RT, NL, WRITE>), dim3(MANA_GRID), dim3(MANA_NT), 0, st, A);
}

template <typename T, int RT, bool WRITE>
static int launch_mana_row(int NL, ManaRowArgs A, hipStream_t st) {
#define HM_MROW(nl)                                  \
  case nl:                                           \
    launch_mana_row_nl<T, RT, nl, WRITE>(A, st);     \
    return OK;
  if constexpr (RT == 3) {
    switch (NL) { HM_MROW(3) HM_MROW(4) HM_MROW(5) HM_MROW(6) HM_MROW(7) HM_MROW(8) default: break; }
  } else if constexpr (RT == 2) {
    switch (NL) { HM_MROW(2) HM_MROW(3) HM_MROW(4) HM_MROW(5) HM_MROW(6) HM_MROW(7) default: break; }
  } else {
    switch (NL) { HM_MROW(1) default: break; }
  }
#undef HM_MROW
  return fail(E_UNSUPPORTED, "mana: no row kernel for 3^%d values (RT %d)", NL, RT);
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
  if constexpr (RT == 3) {
    switch (NH) { HM_MCOL(3) HM_MCOL(4) HM_MCOL(5) HM_MCOL(6) HM_MCOL(7) HM_MCOL(8) default: break; }
  } else {
    switch (NH) { HM_MCOL(2) HM_MCOL(3) HM_MCOL(4) HM_MCOL(5) HM_MCOL(6) HM_MCOL(7) default: break; }
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
      if (P.RT == 3) e = launch_mana_row<T, 3, false>(P.nl, A, st);
      else if (P.RT == 2) e = launch_mana_row<T, 2, false>(P.nl, A, st);
      else e = launch_mana_row<T, 1, false>(P.nl, A, st);
    } else {
      if (P.RT == 2) e = launch_mana_row<T, 2, false>(P.nl, A, st);
      else e = launch_mana_row<T, 1, false>(P.nl, A, st);
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
    ManaRowArgs A{};
    A.psi = psi;
    A.N = P.N;
    A.nh = P.nh;
    A.nhr = (uint32_t)pow3c(P.nh);
    A.n_pairs = nb;
    A.a0 = a0 + 2 * (uint64_t)p0;
    A.a_end = a1;
    A.exch = exch0 + (size_t)l * xb;
    if constexpr (sizeof(T) == 4) e = launch_mana_row<T, 3, true>(P.nl, A, lst[l]);
    else e = launch_mana_row<T, 2, true>(P.nl, A, lst[l]);
    if (e) break;
    ManaColArgs C{};
    C.exch = A.exch;
    C.rowlen = (uint32_t)pow3c(P.nl);
    C.n_pairs = nb;
    C.acc = acc_col + (size_t)l * MANA_GRID * 3;
    if constexpr (sizeof(T) == 4) e = launch_mana_col<T, 3>(P.nh, P.nl, C, lst[l]);
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
  if (ws_bytes < mana_workspace(N, dbl, batch, streams, a1 - a0)) return fail(E_WORKSPACE, "mana workspace too small");
  return dbl ? mana_t<double>(P, psi, a0, a1, sums, out, ws, st) : mana_t<float>(P, psi, a0, a1, sums, out, ws, st);
}

}  // namespace hm
