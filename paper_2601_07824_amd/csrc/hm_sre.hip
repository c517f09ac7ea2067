// hm_sre.hip -- gfx950 kernels for the qubit stabilizer Renyi entropy (Algorithm 2 of "Computing
// quantum magic of state vectors", Eqs. Z_FT_qubits / Z_ovN).
//
// Every X-shift a gives chi_b(a) = sum_x conj(psi_{x^a}) psi_x (-1)^{b.x}, the Walsh-Hadamard
// transform of v_x = conj(psi_{x^a}) psi_x.  Since v_{x^a} = conj(v_x), the transform is computed
// on half the length ("folded" form): with j the top set bit of a and u_c = v_{x(c)} over the
// 2^{N-1} indices x(c) with x_j = 0 (c = x with bit j removed), U = H^{(x)(N-1)} u gives
// |chi_b|^2 in {4 (Re U_c)^2, 4 (Im U_c)^2} for the two b that project onto c.  For a = 0,
// u_c = (r0 + r1) + i (r0 - r1) with r0, r1 = |psi|^2 on the two halves of the top qubit, and
// |chi|^2 in {(Re U_c)^2, (Im U_c)^2}.  The sum over b of |chi_b|^{2q} is therefore the sum of
// f^q t^q over the 2^N real values t = (Re U)^2, (Im U)^2 with f = 4 (a != 0) or 1 (a = 0).
//
// Kernel families
//   * row pass: a workgroup tile holds G whole rows of 2^NL folded values; it forms the product
//     (gathering psi_x and psi_{x^a} from global memory), runs all NL butterfly stages in
//     registers + LDS relayouts, then either reduces (workgroup-resident path: a row is a whole
//     shift) or writes the row to the exchange buffer (two-pass path).
//   * column pass: a tile holds 2^NH rows x 2^CB columns of the exchange buffer of one shift,
//     runs the remaining NH stages and reduces.
//   * shift reduce / final reduce: fixed-order FP64 sums (bitwise reproducible).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hm_sre_dev.h"
#include "hm_tile.h"

namespace hm {

// ------------------------------------------------------------------------------------------------
// Row pass
// ------------------------------------------------------------------------------------------------
struct RowPassArgs {
  const void *psi;      // 2^(nf+1) amplitudes
  int nf;               // folded bits = N - 1
  int nh;               // row-task index bits per shift (0 on the workgroup-resident path)
  int64_t n_slots;      // shifts covered by this launch
  uint64_t a0;          // shift of slot 0 when rows == nullptr
  const uint64_t *rows; // explicit shifts (slot s -> rows[s])
  void *exch;           // WRITE: [n_slots][2^nh][2^NL] values
  double *shift_sums;   // REDUCE: [n_slots][nacc]
  int nacc;
  int64_t n_tiles;
  QArgs qa;
};

template <typename T, int NT, int RB, int NL, bool WRITE, int QM>
__global__ __launch_bounds__(NT) void k_sre_rowpass(RowPassArgs A) {
  constexpr int R = 1 << RB;
  constexpr int LT = ilog2c(NT);
  constexpr int TB = LT + RB;
  static_assert(TB >= NL && NL >= RB, "tile must hold whole rows");
  constexpr int S0 = NL - RB;
  constexpr int K = RB == 0 ? 0 : (NL + RB - 1) / RB;
  static_assert(K <= 4, "at most four rounds");
  constexpr int SEG = 1 << S0;           // threads per row-task
  constexpr int G = 1 << (TB - NL);      // row-tasks per tile
  constexpr bool WAVE_UNIFORM = SEG >= 64;
  constexpr int LDS_N = (K > 1) ? ((1 << TB) + (1 << (TB - RB))) : 1;

  __shared__ vec2<T> lds[LDS_N];
  __shared__ double red[NT / 64 + 1];

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  const uint32_t tau = threadIdx.x;
  const uint32_t tlo = tau & (SEG - 1);
  const uint32_t g = tau >> S0;
  const uint32_t half = 1u << A.nf;

  for (int64_t tile = blockIdx.x; tile < A.n_tiles; tile += gridDim.x) {
    const int64_t rt = tile * G + g;
    const int64_t slot = rt >> A.nh;
    const uint64_t ch = (uint64_t)rt & ((1ull << A.nh) - 1ull);
    const bool active = slot < A.n_slots;
    uint64_t a = 0;
    bool bad = false;
    if (active) {
      a = A.rows ? A.rows[slot] : A.a0 + (uint64_t)slot;
      if (a >> (A.nf + 1)) {
        bad = true;
        a = 0;
      }
    }
    if constexpr (WAVE_UNIFORM) {
      uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
      uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
      a = ((uint64_t)hi << 32) | lo;
    }

    T re[R], im[R];
    sre_product<T, RB, NL>(psi, half, a, ch, tlo, active, re, im);

    // NL butterfly stages: K rounds, round k holds tile bits [S_k, S_k + RB) in registers.
    if constexpr (K >= 1) wht_regs<T, R, 0, rp_H(NL, RB, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout<T, R, RB, rp_S(NL, RB, 0), rp_S(NL, RB, 1)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 2)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 3)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(re, im);
    }

    if constexpr (WRITE) {
      // Final layout has S = 0: register r holds row position b = r | (tlo << RB).  It is stored at
      // column (r << S0) | tlo (a fixed permutation of the columns; the column pass only needs each
      // column to stay a column), so consecutive lanes write consecutive addresses.
      if (active) {
        vec2<T> *ex = (vec2<T> *)A.exch;
        const uint32_t ob = ((uint32_t)rt << NL) | tlo;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          vec2<T> v;
          v.x = re[r];
          v.y = im[r];
          st32(ex, ob + ((uint32_t)r << S0), v);
        }
      }
    } else {
      Acc<T, QM> acc;
      acc.zero();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc.add(re[r], A.qa);
        acc.add(im[r], A.qa);
      }
      double s[Acc<T, QM>::N];
#pragma unroll
      for (int k = 0; k < Acc<T, QM>::N; ++k) s[k] = seg_sum<NT, SEG>((double)acc.a[k], red, tau);
      if (active && tlo == 0) {
        unfold_scale(s, A.nacc, A.qa, a == 0);
        double *o = A.shift_sums + slot * A.nacc;
        for (int k = 0; k < A.nacc; ++k) o[k] = bad ? __builtin_nan("") : s[k];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Column pass
// ------------------------------------------------------------------------------------------------
struct ColPassArgs {
  const void *exch;   // [n_slots][2^NH][2^nl]
  int nl;
  int64_t n_slots;
  int64_t n_cb;       // column blocks per shift = 2^(nl - CB)
  double *partials;   // [n_slots][n_cb][nacc]
  int nacc;
  int64_t n_tiles;
  QArgs qa;
  // per-shift reduction of the previous batch's partials (written by the previous launch)
  const double *prev_partials;
  int64_t prev_n_slots;
  uint64_t prev_a0;
  const uint64_t *prev_rows;
  double *prev_shift_sums;
  int nf;
};

// Per-shift sum over column blocks (fixed order), unfolded and scaled.
__device__ __forceinline__ void reduce_shift(const double *partials, int64_t slot, int64_t n_cb, int nacc, uint64_t a0,
                                             const uint64_t *rows, int nf, const QArgs &qa, double *shift_sums) {
  double s[HM_MAX_Q + 1];
  for (int k = 0; k < nacc; ++k) s[k] = 0.0;
  const double *p = partials + slot * n_cb * nacc;
  for (int64_t c = 0; c < n_cb; ++c)
    for (int k = 0; k < nacc; ++k) s[k] += p[c * nacc + k];
  const uint64_t a = rows ? rows[slot] : a0 + (uint64_t)slot;
  const bool bad = (a >> (nf + 1)) != 0;
  unfold_scale(s, nacc, qa, a == 0);
  for (int k = 0; k < nacc; ++k) shift_sums[slot * nacc + k] = bad ? __builtin_nan("") : s[k];
}

__host__ __device__ constexpr int cp_S(int NH, int RB, int CB, int k) {
  return CB + (RB * k < NH - RB ? RB * k : NH - RB);
}
__host__ __device__ constexpr int cp_L(int NH, int RB, int CB, int k) { return RB * k + CB - cp_S(NH, RB, CB, k); }
__host__ __device__ constexpr int cp_H(int NH, int RB, int CB, int k) {
  return (RB * (k + 1) < NH ? RB * (k + 1) : NH) + CB - cp_S(NH, RB, CB, k);
}

template <typename T, int NT, int RB, int NH, int CB, int QM>
__global__ __launch_bounds__(NT) void k_sre_colpass(ColPassArgs A) {
  constexpr int R = 1 << RB;
  constexpr int LT = ilog2c(NT);
  constexpr int TB = LT + RB;
  static_assert(TB == NH + CB && NH >= RB, "column tile shape");
  constexpr int K = (NH + RB - 1) / RB;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = (K > 1) ? ((1 << TB) + (1 << (TB - RB))) : 1;

  __shared__ vec2<T> lds[LDS_N];
  __shared__ double red[NT / 64 + 1];

  const vec2<T> *__restrict__ ex = (const vec2<T> *)A.exch;
  const uint32_t tau = threadIdx.x;
  const uint32_t col = tau & ((1u << CB) - 1u);
  const uint32_t rowhi = tau >> CB;

  for (int64_t s = (int64_t)blockIdx.x * NT + tau; s < A.prev_n_slots; s += (int64_t)gridDim.x * NT)
    reduce_shift(A.prev_partials, s, A.n_cb, A.nacc, A.prev_a0, A.prev_rows, A.nf, A.qa, A.prev_shift_sums);

  for (int64_t tile = blockIdx.x; tile < A.n_tiles; tile += gridDim.x) {
    const int64_t slot = tile / A.n_cb;
    const int64_t cb = tile - slot * A.n_cb;
    T re[R], im[R];
    {
      const uint32_t base = ((uint32_t)slot << (NH + A.nl)) + ((uint32_t)cb << CB) + col;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t row = (uint32_t)r | (rowhi << RB);
        const vec2<T> v = ld32(ex, base + (row << A.nl));
        re[r] = v.x;
        im[r] = v.y;
      }
    }
    wht_regs<T, R, cp_L(NH, RB, CB, 0), cp_H(NH, RB, CB, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout<T, R, RB, cp_S(NH, RB, CB, 0), cp_S(NH, RB, CB, 1)>(re, im, lds, tau);
      wht_regs<T, R, cp_L(NH, RB, CB, 1), cp_H(NH, RB, CB, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout<T, R, RB, cp_S(NH, RB, CB, 1), cp_S(NH, RB, CB, 2)>(re, im, lds, tau);
      wht_regs<T, R, cp_L(NH, RB, CB, 2), cp_H(NH, RB, CB, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout<T, R, RB, cp_S(NH, RB, CB, 2), cp_S(NH, RB, CB, 3)>(re, im, lds, tau);
      wht_regs<T, R, cp_L(NH, RB, CB, 3), cp_H(NH, RB, CB, 3)>(re, im);
    }
    Acc<T, QM> acc;
    acc.zero();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc.add(re[r], A.qa);
      acc.add(im[r], A.qa);
    }
    double s[Acc<T, QM>::N];
#pragma unroll
    for (int k = 0; k < Acc<T, QM>::N; ++k) s[k] = seg_sum<NT, NT>((double)acc.a[k], red, tau);
    if (tau == 0) {
      double *o = A.partials + (slot * A.n_cb + cb) * A.nacc;
      for (int k = 0; k < A.nacc; ++k) o[k] = s[k];
    }
  }
}

// per-shift sums from column-pass partials of the last batch
__global__ void k_sre_shift_reduce(const double *partials, int64_t n_slots, int64_t n_cb, int nacc, uint64_t a0,
                                   const uint64_t *rows, int nf, QArgs qa, double *shift_sums) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot < n_slots) reduce_shift(partials, slot, n_cb, nacc, a0, rows, nf, qa, shift_sums);
}

// Fixed-order sum over all per-shift sums; optionally finalise (Eq. sre).
__global__ __launch_bounds__(256) void k_sre_total(const double *shift_sums, int64_t n_slots, int nacc, QArgs qa,
                                                   int N, double *sums, double *out) {
  __shared__ double red[256];
  __shared__ double tot[HM_MAX_Q + 1];
  const uint32_t t = threadIdx.x;
  for (int k = 0; k < nacc; ++k) {
    double s = 0.0;
    for (int64_t i = t; i < n_slots; i += 256) s += shift_sums[i * nacc + k];
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
      for (int k = 0; k < nacc; ++k) sums[k] = tot[k];
    if (out) {
      const double D = ldexp(1.0, N);
      for (int i = 0; i < qa.nq; ++i) {
        const double q = qa.q[i];
        out[i] = (q == 1.0) ? -tot[1 + i] / D : log2(tot[1 + i] / D) / (1.0 - q);
      }
      out[qa.nq] = 1.0 - tot[0] / D;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------------
static inline int nacc_of(const QArgs &qa) { return qa.nq + 1; }
static inline bool is_q2(const QArgs &qa) { return qa.nq == 1 && qa.q[0] == 2.0; }

template <typename T> struct Cfg;
template <> struct Cfg<float> {
  static constexpr int RB = 5, ROW_NT = 128, COL_NT = 256;
};
template <> struct Cfg<double> {
  static constexpr int RB = 4, ROW_NT = 128, COL_NT = 256;
};

static int64_t grid_for(int64_t tiles) { return tiles < 65536 ? tiles : 65536; }

template <typename T, int NT, int RB, int NL, bool WRITE>
static void launch_row_q(const RowPassArgs &A, bool q2, hipStream_t st) {
  const dim3 grid((unsigned)grid_for(A.n_tiles)), block(NT);
  ProfScope prof(WRITE ? "sre_rowpass_write" : "sre_rowpass_resident", st);
  if (WRITE || !q2) hipLaunchKernelGGL((k_sre_rowpass<T, NT, RB, NL, WRITE, 0>), grid, block, 0, st, A);
  else hipLaunchKernelGGL((k_sre_rowpass<T, NT, RB, NL, WRITE, 2>), grid, block, 0, st, A);
}

// Dispatch over the row length NL (compile-time in the kernels).
template <typename T, bool WRITE>
static int launch_rowpass(int NL, RowPassArgs A, bool q2, hipStream_t st) {
  constexpr int RB = Cfg<T>::RB;
  constexpr int NT = Cfg<T>::ROW_NT;
  constexpr int TB = ilog2c(NT) + RB;
  auto tiles = [&](int nt, int rb) {
    const int G = 1 << (ilog2c(nt) + rb - NL);
    const int64_t rts = A.n_slots << A.nh;
    return (rts + G - 1) / G;
  };
#define HM_ROW_SMALL(nl)                                       \
  case nl:                                                     \
    A.n_tiles = tiles(64, nl);                                 \
    launch_row_q<T, 64, nl, nl, WRITE>(A, q2, st);             \
    return OK;
#define HM_ROW(nl)                                             \
  case nl:                                                     \
    A.n_tiles = tiles(NT, RB);                                 \
    launch_row_q<T, NT, RB, nl, WRITE>(A, q2, st);             \
    return OK;
#define HM_ROW_BIG(nl)                                         \
  case nl:                                                     \
    A.n_tiles = tiles(2 * NT, RB);                             \
    launch_row_q<T, 2 * NT, RB, nl, WRITE>(A, q2, st);         \
    return OK;
  if constexpr (RB == 5) {
    switch (NL) {
      HM_ROW_SMALL(0) HM_ROW_SMALL(1) HM_ROW_SMALL(2) HM_ROW_SMALL(3) HM_ROW_SMALL(4)
      HM_ROW(5) HM_ROW(6) HM_ROW(7) HM_ROW(8) HM_ROW(9) HM_ROW(10) HM_ROW(11) HM_ROW(12)
      HM_ROW_BIG(13)
      default: break;
    }
  } else {
    switch (NL) {
      HM_ROW_SMALL(0) HM_ROW_SMALL(1) HM_ROW_SMALL(2) HM_ROW_SMALL(3)
      HM_ROW(4) HM_ROW(5) HM_ROW(6) HM_ROW(7) HM_ROW(8) HM_ROW(9) HM_ROW(10) HM_ROW(11)
      HM_ROW_BIG(12)
      default: break;
    }
  }
#undef HM_ROW_SMALL
#undef HM_ROW
#undef HM_ROW_BIG
  (void)TB;
  return fail(E_UNSUPPORTED, "row pass: no kernel for row length 2^%d", NL);
}

template <typename T, int NT, int NH>
static void launch_col_nh(ColPassArgs A, bool q2, hipStream_t st) {
  constexpr int RB = Cfg<T>::RB;
  constexpr int CB = ilog2c(NT) + RB - NH;
  A.n_cb = (int64_t)1 << (A.nl - CB);
  A.n_tiles = A.n_slots * A.n_cb;
  const dim3 grid((unsigned)grid_for(A.n_tiles)), block(NT);
  ProfScope prof("sre_colpass", st);
  if (q2) hipLaunchKernelGGL((k_sre_colpass<T, NT, RB, NH, CB, 2>), grid, block, 0, st, A);
  else hipLaunchKernelGGL((k_sre_colpass<T, NT, RB, NH, CB, 0>), grid, block, 0, st, A);
}

// Column tiles: 256 threads (2^(8+RB) values) on the large sizes, 64 threads on the small ones.
template <typename T>
static int launch_colpass(int col_tb, int NH, ColPassArgs &A, bool q2, hipStream_t st) {
  constexpr int RB = Cfg<T>::RB;
  if (A.nl < col_tb - NH) return fail(E_UNSUPPORTED, "column pass: rows of 2^%d too short for 2^%d-row tiles", A.nl, NH);
#define HM_COLB(nh) \
  case nh:          \
    launch_col_nh<T, 256, nh>(A, q2, st); \
    return OK;
#define HM_COLS(nh) \
  case nh:          \
    launch_col_nh<T, 64, nh>(A, q2, st); \
    return OK;
  if (col_tb != 8 + RB && col_tb != 6 + RB) return fail(E_UNSUPPORTED, "column pass: tile of 2^%d values", col_tb);
  if constexpr (RB == 5) {
    if (col_tb == 8 + RB) {
      switch (NH) { HM_COLB(5) HM_COLB(6) HM_COLB(7) HM_COLB(8) HM_COLB(9) HM_COLB(10) HM_COLB(11) HM_COLB(12) HM_COLB(13) default: break; }
    } else {
      switch (NH) { HM_COLS(5) HM_COLS(6) HM_COLS(7) HM_COLS(8) HM_COLS(9) HM_COLS(10) HM_COLS(11) default: break; }
    }
  } else {
    if (col_tb == 8 + RB) {
      switch (NH) { HM_COLB(4) HM_COLB(5) HM_COLB(6) HM_COLB(7) HM_COLB(8) HM_COLB(9) HM_COLB(10) HM_COLB(11) HM_COLB(12) default: break; }
    } else {
      switch (NH) { HM_COLS(4) HM_COLS(5) HM_COLS(6) HM_COLS(7) HM_COLS(8) HM_COLS(9) HM_COLS(10) default: break; }
    }
  }
#undef HM_COLB
#undef HM_COLS
  return fail(E_UNSUPPORTED, "column pass: no kernel for 2^%d rows", NH);
}

// ---- planning -------------------------------------------------------------------------------------
int sre_plan(int N, int dbl, int force_path, int64_t batch_opt, SrePlan *p) {
  if (N < 1 || N > 26) return fail(E_SIZE, "SRE: n = %d outside [1, 26]", N);
  SrePlan P{};
  P.N = N;
  P.nf = N - 1;
  P.dbl = dbl;
  const int RB = dbl ? 4 : 5;
  const int onepass_max = dbl ? 12 : 13;  // folded bits one workgroup tile can hold
  const int twopass_min = 6 + RB;         // smallest column tile is 64 threads x 2^RB values
  int path = force_path;
  if (path == 0) path = (P.nf <= onepass_max) ? 1 : 2;
  if (path != 1 && path != 2) return fail(E_ARG, "SRE: path %d unknown", path);
  if (path == 1 && P.nf > onepass_max)
    return fail(E_UNSUPPORTED, "SRE: workgroup-resident path holds at most 2^%d folded values (n = %d)", onepass_max, N);
  if (path == 2 && P.nf < twopass_min)
    return fail(E_UNSUPPORTED, "SRE: two-pass path needs n >= %d", twopass_min + 1);
  P.path = path;
  if (path == 2) {
    const int col_tb = (P.nf >= 8 + RB) ? 8 + RB : 6 + RB;
    const int nl_max = dbl ? 12 : 13;
    int nl = (P.nf + 1) / 2;
    int nh = P.nf - nl;
    if (nh < RB) { nh = RB; nl = P.nf - nh; }
    if (nl < col_tb - nh) { nl = col_tb - nh; nh = P.nf - nl; }
    if (nl > nl_max) { nl = nl_max; nh = P.nf - nl; }
    if (nh < RB || nh > col_tb || nl < col_tb - nh || nl > nl_max)
      return fail(E_SIZE, "SRE: no two-pass split for n = %d", N);
    P.nl = nl;
    P.nh = nh;
    P.col_tb = col_tb;
    // The exchange of one batch (batch x 2^nf values) is sized to stay resident in the 256 MiB
    // memory-side cache (MALL) while giving each launch enough tiles to fill the 256 CUs.
    const size_t per_shift = ((size_t)1 << P.nf) * (dbl ? 16 : 8);
    int64_t b = batch_opt > 0 ? batch_opt : (int64_t)((128ull << 20) / per_shift);
    if ((size_t)b * per_shift > (3ull << 30)) b = (int64_t)((3ull << 30) / per_shift);  // 32-bit offsets
    if (b < 1) b = 1;
    if (b > ((int64_t)1 << N)) b = (int64_t)1 << N;
    P.batch = (int)b;
  }
  *p = P;
  return OK;
}

// Workspace layout: [per-shift sums, unless the caller supplies them] [exchange] [column partials].
static size_t exch_bytes(const SrePlan &p) {
  return p.path == 2 ? align256((size_t)p.batch * ((size_t)1 << p.nf) * (p.dbl ? 16 : 8)) : 0;
}
static int64_t col_blocks(const SrePlan &p) { return (int64_t)1 << (p.nl - (p.col_tb - p.nh)); }

size_t sre_workspace(const SrePlan &p, int nq, int64_t n_internal_slots) {
  const size_t nacc = (size_t)nq + 1;
  size_t b = align256((size_t)n_internal_slots * nacc * sizeof(double));
  if (p.path == 2) {
    b += exch_bytes(p);
    b += 2 * align256((size_t)p.batch * (size_t)col_blocks(p) * nacc * sizeof(double));  // double-buffered
  }
  return b < 256 ? 256 : b;
}

template <typename T>
static int shift_sums_t(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                        int64_t n_slots, double *shift_sums, char *w, hipStream_t st) {
  const bool q2 = is_q2(qa);
  const int nacc = nacc_of(qa);
  if (n_slots <= 0) return OK;
  if (p.path == 1) {
    RowPassArgs A{};
    A.psi = psi;
    A.nf = p.nf;
    A.nh = 0;
    A.n_slots = n_slots;
    A.a0 = a0;
    A.rows = rows;
    A.shift_sums = shift_sums;
    A.nacc = nacc;
    A.qa = qa;
    int e = launch_rowpass<T, false>(p.nf, A, q2, st);
    if (e) return e;
    return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE row pass launch: %s", hipGetErrorString(hipGetLastError()));
  }
  // Two-pass: per batch, row pass (writes the exchange) then column pass (reads it, writes per
  // column-block partials and reduces the previous batch's partials to per-shift sums).
  const int64_t n_cb = col_blocks(p);
  void *exch = w;
  const size_t pbytes = align256((size_t)p.batch * (size_t)n_cb * nacc * sizeof(double));
  double *partials[2] = {(double *)(w + exch_bytes(p)), (double *)(w + exch_bytes(p) + pbytes)};
  int64_t prev_s0 = 0, prev_nb = 0;
  int k = 0;
  for (int64_t s0 = 0; s0 < n_slots; s0 += p.batch, ++k) {
    const int64_t nb = (n_slots - s0) < p.batch ? (n_slots - s0) : p.batch;
    RowPassArgs A{};
    A.psi = psi;
    A.nf = p.nf;
    A.nh = p.nh;
    A.n_slots = nb;
    A.a0 = a0 + (uint64_t)s0;
    A.rows = rows ? rows + s0 : nullptr;
    A.exch = exch;
    A.nacc = nacc;
    A.qa = qa;
    int e = launch_rowpass<T, true>(p.nl, A, q2, st);
    if (e) return e;
    ColPassArgs C{};
    C.exch = exch;
    C.nl = p.nl;
    C.n_slots = nb;
    C.partials = partials[k & 1];
    C.nacc = nacc;
    C.qa = qa;
    C.nf = p.nf;
    C.prev_partials = partials[(k + 1) & 1];
    C.prev_n_slots = prev_nb;
    C.prev_a0 = a0 + (uint64_t)prev_s0;
    C.prev_rows = rows ? rows + prev_s0 : nullptr;
    C.prev_shift_sums = shift_sums + prev_s0 * nacc;
    e = launch_colpass<T>(p.col_tb, p.nh, C, q2, st);
    if (e) return e;
    prev_s0 = s0;
    prev_nb = nb;
  }
  {
    const int thr = 128;
    ProfScope prof("sre_shift_reduce", st);
    hipLaunchKernelGGL(k_sre_shift_reduce, dim3((unsigned)((prev_nb + thr - 1) / thr)), dim3(thr), 0, st,
                       partials[(k + 1) & 1], prev_nb, n_cb, nacc, a0 + (uint64_t)prev_s0,
                       rows ? rows + prev_s0 : nullptr, p.nf, qa, shift_sums + prev_s0 * nacc);
  }
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE two-pass launch: %s", hipGetErrorString(hipGetLastError()));
}

int sre_run(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows, int64_t n_slots,
            double *ext_shift_sums, double *sums, double *out, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  double *ss = ext_shift_sums;
  if (!ss) {
    ss = (double *)w;
    w += align256((size_t)n_slots * (size_t)nacc_of(qa) * sizeof(double));
  }
  int e = p.dbl ? shift_sums_t<double>(p, psi, qa, a0, rows, n_slots, ss, w, st)
                : shift_sums_t<float>(p, psi, qa, a0, rows, n_slots, ss, w, st);
  if (e) return e;
  if (sums || out) return sre_reduce_shifts(ss, n_slots, qa, p.N, sums, out, st);
  return OK;
}

int sre_reduce_shifts(const double *shift_sums, int64_t n_slots, const QArgs &qa, int N, double *sums, double *out,
                      hipStream_t st) {
  ProfScope prof("sre_total", st);
  hipLaunchKernelGGL(k_sre_total, dim3(1), dim3(256), 0, st, shift_sums, n_slots, nacc_of(qa), qa, N, sums, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE reduce launch: %s", hipGetErrorString(hipGetLastError()));
}

__global__ void k_sre_finalize(int N, QArgs qa, const double *sums, double *out) {
  if (threadIdx.x != 0) return;
  const double D = ldexp(1.0, N);
  for (int i = 0; i < qa.nq; ++i) {
    const double q = qa.q[i];
    out[i] = (q == 1.0) ? -sums[1 + i] / D : log2(sums[1 + i] / D) / (1.0 - q);
  }
  out[qa.nq] = 1.0 - sums[0] / D;
}

int sre_finalize_launch(int N, const QArgs &qa, const double *sums, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sre_finalize, dim3(1), dim3(64), 0, st, N, qa, sums, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE finalize launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace hm
