// hm_sre_kern.h -- qubit SRE kernels (row pass, column pass, per-shift reduction) and their
// templated launchers.  Included by one translation unit per dtype (hm_sre_f32.hip,
// hm_sre_f64.hip); everything here has internal linkage.
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
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_sre_dev.h"
#include "hm_tile.h"

namespace hm {
namespace {

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
  int64_t tile0;        // first tile of this launch (launches of one workgroup per tile, in chunks)
  QArgs qa;
  // batched mode (n_states > 0): slot s is shift s mod 2^state_bits of state s >> state_bits
  int n_states;
  int state_bits;
  const void *psis[HM_BATCH_PTRS];
};

// Row-pass tile shape and LDS needs (shared by the stand-alone and the pipelined kernels).
template <typename T, int NT, int RB, int NL, bool SPLIT>
struct RowShape {
  static constexpr int TB = ilog2c(NT) + RB;
  static constexpr int K = RB == 0 ? 0 : (NL + RB - 1) / RB;
  static constexpr int LDS_N = (K > 1) ? ((1 << TB) + (1 << (TB - RB))) : 1;
  using Elem = typename std::conditional<SPLIT, T, vec2<T>>::type;
  static constexpr size_t LDS_BYTES = (size_t)LDS_N * sizeof(Elem);
};

// Arguments of one state's workgroup-resident tiles inside a persistent launch: the fields of
// RowPassArgs that a single-state, all-shifts, reducing row pass reads (no pointer table).
struct StateTileArgs {
  const void *psi;
  int nf;
  static constexpr int nh = 0;
  int64_t n_slots;
  static constexpr uint64_t a0 = 0;
  static constexpr const uint64_t *rows = nullptr;
  static constexpr void *exch = nullptr;
  double *shift_sums;
  int nacc;
  int64_t n_tiles;
  const QArgs &qa;  // the launch's Renyi indices (kernel argument), not copied
  static constexpr int n_states = 0;
  static constexpr int state_bits = 0;
  static constexpr const void *psis[1] = {nullptr};
  __device__ StateTileArgs(const void *psi_, int nf_, double *ss, int nacc_, int64_t n_tiles_, const QArgs &qa_)
      : psi(psi_), nf(nf_), n_slots((int64_t)1 << (nf_ + 1)), shift_sums(ss), nacc(nacc_), n_tiles(n_tiles_),
        qa(qa_) {}
};

// Row tiles t0, t0 + tstep, ... < A.n_tiles; ONE: the tile t0 only (launches of one workgroup per
// tile).  Without the loop the compiler does not keep every fold case's addresses live across
// tiles: the tile needs far fewer registers (measured at n = 12: 162 -> 98 VGPRs, 18.6 -> 12.6 us
// per launch on MI355X).
template <typename T, int NT, int RB, int NL, bool WRITE, int QM, bool SPLIT, typename Args = RowPassArgs,
          bool ONE = false>
__device__ __forceinline__ void rowpass_tiles(const Args &A, int64_t t0, int64_t tstep,
                                              typename RowShape<T, NT, RB, NL, SPLIT>::Elem *lds, double *red,
                                              uint32_t tau = threadIdx.x) {
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

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  const uint32_t tlo = tau & (SEG - 1);
  const uint32_t g = tau >> S0;
  const uint32_t half = 1u << A.nf;

  for (int64_t tile = t0; tile < A.n_tiles; tile += tstep) {
    const int64_t rt = tile * G + g;
    const int64_t slot = rt >> A.nh;
    const uint64_t ch = (uint64_t)rt & ((1ull << A.nh) - 1ull);
    const bool active = slot < A.n_slots;
    uint64_t a = 0;
    bool bad = false;
    const vec2<T> *__restrict__ ps = psi;
    if (active) {
      if (A.n_states > 0) {
        ps = (const vec2<T> *)A.psis[A.n_states > 0 ? slot >> A.state_bits : 0];
        a = (uint64_t)slot & ((1ull << A.state_bits) - 1ull);
      } else {
        a = A.rows ? A.rows[slot] : A.a0 + (uint64_t)slot;
      }
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
    sre_product<T, RB, NL, (SPLIT || WRITE) ? 8 : R>(ps, half, a, ch, tlo, active, re, im);

    // NL butterfly stages: K rounds, round k holds tile bits [S_k, S_k + RB) in registers.
    if constexpr (K >= 1) wht_regs<T, R, 0, rp_H(NL, RB, 0)>(re, im);
    if constexpr (K >= 2) {
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 0), rp_S(NL, RB, 1)>(re, im, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 0), rp_S(NL, RB, 1)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 2)>(re, im, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 2)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 3)>(re, im, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 3)>(re, im, lds, tau);
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(re, im);
    }

    if constexpr (WRITE) {
      // Final layout has S = 0: register r holds row position b = r | (tlo << RB).  It is stored at
      // column (r << S0) | tlo (a fixed permutation of the columns; the column pass only needs each
      // column to stay a column), so consecutive lanes write consecutive addresses.
      if (active) {
        vec2<T> *ex = (vec2<T> *)A.exch;
        if constexpr (sizeof(T) == 4 && RB == 5) {
          // 16-byte stores: registers r, r + 1 of thread tlo go to columns 2 c, 2 c + 1 with
          // c = ((r / 2) << S0) | tlo (another fixed column permutation)
          float4 *ex4 = (float4 *)A.exch;
          const uint32_t ob4 = ((uint32_t)rt << (NL - 1)) | tlo;
#pragma unroll
          for (int r = 0; r < R; r += 2) {
            float4 v;
            v.x = re[r];
            v.y = im[r];
            v.z = re[r + 1];
            v.w = im[r + 1];
            st32(ex4, ob4 + ((uint32_t)(r >> 1) << S0), v);
          }
        } else {
          const uint32_t ob = ((uint32_t)rt << NL) | tlo;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            vec2<T> v;
            v.x = re[r];
            v.y = im[r];
            st32(ex, ob + ((uint32_t)r << S0), v);
          }
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
    if constexpr (ONE) break;
  }
}

// Split-staged FP32 row-pass tiles keep to a register budget of four waves per SIMD (the column
// pass would spill under it).
template <typename T, bool SPLIT>
struct TwoPassWaves { static constexpr int value = (SPLIT && sizeof(T) == 4) ? 4 : 1; };

// One workgroup per tile (grid = n_tiles).
template <typename T, int NT, int RB, int NL, bool WRITE, int QM, bool SPLIT = false>
__global__ __launch_bounds__(NT, (WRITE ? TwoPassWaves<T, SPLIT>::value : 1)) void k_sre_rowpass(RowPassArgs A) {
  using Sh = RowShape<T, NT, RB, NL, SPLIT>;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  __shared__ double red[NT / 64 + 1];
  rowpass_tiles<T, NT, RB, NL, WRITE, QM, SPLIT, RowPassArgs, true>(A, A.tile0 + blockIdx.x, gridDim.x, lds, red);
}

// The same with a register budget for at least MINW waves per SIMD (resident tiles of <= 2^13
// values with split LDS staging, so that LDS does not cap the occupancy either).
template <typename T, int NT, int RB, int NL, int QM, int MINW>
__global__ __launch_bounds__(NT, MINW) void k_sre_rowpass_occ(RowPassArgs A) {
  using Sh = RowShape<T, NT, RB, NL, true>;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  __shared__ double red[NT / 64 + 1];
  rowpass_tiles<T, NT, RB, NL, false, QM, true, RowPassArgs, true>(A, A.tile0 + blockIdx.x, gridDim.x, lds, red);
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
  int64_t tile0;      // first tile of this launch (launches of one workgroup per tile, in chunks)
  QArgs qa;
  // per-shift reduction of the previous batch's partials (written by the previous launch)
  const double *prev_partials;
  int64_t prev_n_slots;
  uint64_t prev_a0;
  const uint64_t *prev_rows;
  double *prev_shift_sums;
  int nf;
  uint64_t a0;  // shift of slot 0 (adjoint column pass only)
};

// Per-shift sum over the column blocks, unfolded and scaled, by the 64 lanes of one wave (all of
// them must call it): lane l adds blocks l, l + 64, ... in order, then a fixed shuffle tree adds the
// lanes, so the result does not depend on timing.  (One thread per shift would walk 2^10 blocks per
// shift serially at n = 24.)
__device__ __forceinline__ void reduce_shift_wave(const double *partials, int64_t slot, int64_t n_cb, int nacc,
                                                  uint64_t a0, const uint64_t *rows, int nf, const QArgs &qa,
                                                  double *shift_sums, uint32_t lane) {
  double s[HM_MAX_Q + 1];
#pragma unroll
  for (int k = 0; k < HM_MAX_Q + 1; ++k) s[k] = 0.0;
  const double *p = partials + slot * n_cb * nacc;
  for (int64_t c = lane; c < n_cb; c += 64)
#pragma unroll
    for (int k = 0; k < HM_MAX_Q + 1; ++k)
      if (k < nacc) s[k] += p[c * nacc + k];
#pragma unroll
  for (int k = 0; k < HM_MAX_Q + 1; ++k)
    if (k < nacc)
      for (int off = 32; off > 0; off >>= 1) s[k] += __shfl_down(s[k], off, 64);
  if (lane == 0) {
    const uint64_t a = rows ? rows[slot] : a0 + (uint64_t)slot;
    const bool bad = (a >> (nf + 1)) != 0;
    unfold_scale(s, nacc, qa, a == 0);
    for (int k = 0; k < nacc; ++k) shift_sums[slot * nacc + k] = bad ? __builtin_nan("") : s[k];
  }
}

// Slots s0, s0 + step, ... < n of the previous batch, one wave each (wave w of the workgroup takes
// the w-th of the workgroup's slots).
__device__ __forceinline__ void reduce_prev_shifts(const ColPassArgs &C, int64_t first_wave, int64_t wave_step) {
  const uint32_t lane = threadIdx.x & 63;
  for (int64_t s = first_wave + (threadIdx.x >> 6); s < C.prev_n_slots; s += wave_step)
    reduce_shift_wave(C.prev_partials, s, C.n_cb, C.nacc, C.prev_a0, C.prev_rows, C.nf, C.qa, C.prev_shift_sums, lane);
}

__host__ __device__ constexpr int cp_S(int NH, int RB, int CB, int k) {
  return CB + (RB * k < NH - RB ? RB * k : NH - RB);
}
__host__ __device__ constexpr int cp_L(int NH, int RB, int CB, int k) { return RB * k + CB - cp_S(NH, RB, CB, k); }
__host__ __device__ constexpr int cp_H(int NH, int RB, int CB, int k) {
  return (RB * (k + 1) < NH ? RB * (k + 1) : NH) + CB - cp_S(NH, RB, CB, k);
}

template <typename T, int NT, int RB, int NH, int CB, bool SPLIT>
struct ColShape {
  static constexpr int TB = ilog2c(NT) + RB;
  static constexpr int K = (NH + RB - 1) / RB;
  static constexpr int LDS_N = (K > 1) ? ((1 << TB) + (1 << (TB - RB))) : 1;
  using Elem = typename std::conditional<SPLIT, T, vec2<T>>::type;
  static constexpr size_t LDS_BYTES = (size_t)LDS_N * sizeof(Elem);
};

// Column tiles t0, t0 + tstep, ... < A.n_tiles (the previous batch's per-shift reduction is done by
// the caller).
// ADJ (gradient): after the sums, each value is replaced by its adjoint seed |k U|^{2q-2} U, the
// column stages run again in reverse order (the transform is its own adjoint) and the tile is
// written back in place.
// XCD: tiles t0, t0 + tstep, ... are taken through xcd_tile (tstep a multiple of 8).
template <typename T, int NT, int RB, int NH, int CB, int QM, bool SPLIT, bool ADJ = false, bool XCD = false,
          bool ONE = false>
__device__ __forceinline__ void colpass_tiles(const ColPassArgs &A, int64_t t0, int64_t tstep,
                                              typename ColShape<T, NT, RB, NH, CB, SPLIT>::Elem *lds, double *red) {
  constexpr int R = 1 << RB;
  constexpr int LT = ilog2c(NT);
  constexpr int TB = LT + RB;
  static_assert(TB == NH + CB && NH >= RB, "column tile shape");
  constexpr int K = (NH + RB - 1) / RB;
  static_assert(K <= 4, "at most four rounds");

  const vec2<T> *__restrict__ ex = (const vec2<T> *)A.exch;
  const uint32_t tau = threadIdx.x;
  const uint32_t col = tau & ((1u << CB) - 1u);
  const uint32_t rowhi = tau >> CB;

  for (int64_t b = t0; b < A.n_tiles; b += tstep) {
    const int64_t tile = XCD ? xcd_tile(b, A.n_tiles) : b;
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
      if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 0), cp_S(NH, RB, CB, 1)>(re, im, lds, tau);
      else relayout<T, R, RB, cp_S(NH, RB, CB, 0), cp_S(NH, RB, CB, 1)>(re, im, lds, tau);
      wht_regs<T, R, cp_L(NH, RB, CB, 1), cp_H(NH, RB, CB, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 1), cp_S(NH, RB, CB, 2)>(re, im, lds, tau);
      else relayout<T, R, RB, cp_S(NH, RB, CB, 1), cp_S(NH, RB, CB, 2)>(re, im, lds, tau);
      wht_regs<T, R, cp_L(NH, RB, CB, 2), cp_H(NH, RB, CB, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 2), cp_S(NH, RB, CB, 3)>(re, im, lds, tau);
      else relayout<T, R, RB, cp_S(NH, RB, CB, 2), cp_S(NH, RB, CB, 3)>(re, im, lds, tau);
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
    if constexpr (ADJ) {
      const T kf = (A.a0 + (uint64_t)slot == 0) ? T(1) : T(2);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        re[r] = wfold<T, QM == 2>(re[r], kf, A.qa.q[0]);
        im[r] = wfold<T, QM == 2>(im[r], kf, A.qa.q[0]);
      }
      if constexpr (K >= 4) {
        wht_regs<T, R, cp_L(NH, RB, CB, 3), cp_H(NH, RB, CB, 3)>(re, im);
        if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 3), cp_S(NH, RB, CB, 2)>(re, im, lds, tau);
        else relayout<T, R, RB, cp_S(NH, RB, CB, 3), cp_S(NH, RB, CB, 2)>(re, im, lds, tau);
      }
      if constexpr (K >= 3) {
        wht_regs<T, R, cp_L(NH, RB, CB, 2), cp_H(NH, RB, CB, 2)>(re, im);
        if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 2), cp_S(NH, RB, CB, 1)>(re, im, lds, tau);
        else relayout<T, R, RB, cp_S(NH, RB, CB, 2), cp_S(NH, RB, CB, 1)>(re, im, lds, tau);
      }
      if constexpr (K >= 2) {
        wht_regs<T, R, cp_L(NH, RB, CB, 1), cp_H(NH, RB, CB, 1)>(re, im);
        if constexpr (SPLIT) relayout_split<T, R, RB, cp_S(NH, RB, CB, 1), cp_S(NH, RB, CB, 0)>(re, im, lds, tau);
        else relayout<T, R, RB, cp_S(NH, RB, CB, 1), cp_S(NH, RB, CB, 0)>(re, im, lds, tau);
      }
      wht_regs<T, R, cp_L(NH, RB, CB, 0), cp_H(NH, RB, CB, 0)>(re, im);
      vec2<T> *exw = (vec2<T> *)A.exch;
      uint32_t base = ((uint32_t)slot << (NH + A.nl)) + ((uint32_t)cb << CB) + col;
      // recompute the write addresses instead of keeping the loads' 64-bit addresses live across
      // the transforms (an empty asm hides that base equals the load base)
      asm volatile("" : "+v"(base));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t row = (uint32_t)r | (rowhi << RB);
        vec2<T> v;
        v.x = re[r];
        v.y = im[r];
        st32(exw, base + (row << A.nl), v);
      }
    }
    if constexpr (ONE) break;
  }
}

template <typename T, int NT, int RB, int NH, int CB, int QM, bool SPLIT = false>
__global__ __launch_bounds__(NT) void k_sre_colpass(ColPassArgs A) {
  using Sh = ColShape<T, NT, RB, NH, CB, SPLIT>;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  __shared__ double red[NT / 64 + 1];
  if (A.tile0 == 0) reduce_prev_shifts(A, (int64_t)blockIdx.x * (NT / 64), (int64_t)gridDim.x * (NT / 64));
  colpass_tiles<T, NT, RB, NH, CB, QM, SPLIT, false, true, true>(A, A.tile0 + blockIdx.x, gridDim.x, lds, red);
}

// per-shift sums from column-pass partials of the last batch: one wave per shift (launch
// SHIFT_REDUCE_NT threads per workgroup, ceil(n_slots / (SHIFT_REDUCE_NT / 64)) workgroups)
constexpr int SHIFT_REDUCE_NT = 256;
__global__ __launch_bounds__(SHIFT_REDUCE_NT) void k_sre_shift_reduce(const double *partials, int64_t n_slots,
                                                                     int64_t n_cb, int nacc, uint64_t a0,
                                                                     const uint64_t *rows, int nf, QArgs qa,
                                                                     double *shift_sums) {
  const int64_t slot = (int64_t)blockIdx.x * (SHIFT_REDUCE_NT / 64) + (threadIdx.x >> 6);
  if (slot < n_slots) reduce_shift_wave(partials, slot, n_cb, nacc, a0, rows, nf, qa, shift_sums, threadIdx.x & 63);
}
static inline unsigned shift_reduce_grid(int64_t n_slots) {
  return (unsigned)((n_slots + SHIFT_REDUCE_NT / 64 - 1) / (SHIFT_REDUCE_NT / 64));
}


static inline int nacc_of(const QArgs &qa) { return qa.nq + 1; }
static inline bool is_q2(const QArgs &qa) { return qa.nq == 1 && qa.q[0] == 2.0; }
// One workgroup per tile: the row and column kernels take tile tile0 + blockIdx.x only, in launches
// of at most MAX_GRID workgroups (gridDim.x x blockDim.x must stay below 2^32; a multiple of 8, so
// the XCD of a workgroup is blockIdx.x mod 8 in every chunk).
static constexpr int64_t MAX_GRID = (int64_t)1 << 21;
static inline int64_t grid_for(int64_t tiles) { return tiles < MAX_GRID ? tiles : MAX_GRID; }

// Register-tile bits of the workgroup-resident kernels (values per thread = 2^RB).
template <typename T> struct ResidentRB;
template <> struct ResidentRB<float> { static constexpr int value = 5; };
template <> struct ResidentRB<double> { static constexpr int value = 4; };

template <typename T, int NT, int RB, int NL, bool WRITE, bool SPLIT = false>
static void launch_row_q(RowPassArgs A, bool q2, hipStream_t st) {
  ProfScope prof(WRITE ? "sre_rowpass_write" : "sre_rowpass_resident", st);
  for (A.tile0 = 0; A.tile0 < A.n_tiles; A.tile0 += MAX_GRID) {
    const dim3 grid((unsigned)grid_for(A.n_tiles - A.tile0)), block(NT);
    if (WRITE || !q2) hipLaunchKernelGGL((k_sre_rowpass<T, NT, RB, NL, WRITE, 0, SPLIT>), grid, block, 0, st, A);
    else hipLaunchKernelGGL((k_sre_rowpass<T, NT, RB, NL, WRITE, 2, SPLIT>), grid, block, 0, st, A);
  }
}

template <int NT, int RB, int NL>
static int64_t row_tiles(const RowPassArgs &A) {
  constexpr int G = 1 << (ilog2c(NT) + RB - NL);
  const int64_t rts = A.n_slots << A.nh;
  return (rts + G - 1) / G;
}

// Workgroup-resident row pass (one row = one whole folded shift vector of 2^NL values).
template <typename T, int NT, int RB, int NL, int MINW>
static void launch_row_occ(RowPassArgs A, bool q2, hipStream_t st) {
  ProfScope prof("sre_rowpass_resident", st);
  for (A.tile0 = 0; A.tile0 < A.n_tiles; A.tile0 += MAX_GRID) {
    const dim3 grid((unsigned)grid_for(A.n_tiles - A.tile0)), block(NT);
    if (q2) hipLaunchKernelGGL((k_sre_rowpass_occ<T, NT, RB, NL, 2, MINW>), grid, block, 0, st, A);
    else hipLaunchKernelGGL((k_sre_rowpass_occ<T, NT, RB, NL, 0, (MINW > 3 ? 3 : MINW)>), grid, block, 0, st, A);  // general q: more accumulators
  }
}

// split: tiles of 2^10..2^14 (FP32) / 2^10..2^13 (FP64) values use split LDS staging and a register
// budget of at least 3 waves per SIMD (4 for 2^14 FP32 values: 512 threads x 32 values in 128
// registers); one tile per workgroup, the tiles use about 100 registers.
template <typename T>
static int launch_resident(int NL, RowPassArgs A, bool q2, hipStream_t st, bool split = false) {
  constexpr int RB = ResidentRB<T>::value;
  if (split && NL >= 10 && NL <= 14) {
#define HM_RO(nl, nt, w)                                            \
  case nl:                                                          \
    A.n_tiles = row_tiles<nt, RB, nl>(A);                           \
    launch_row_occ<T, nt, RB, nl, w>(A, q2, st);                    \
    return OK;
    if constexpr (RB == 5) {
      // one shift per workgroup from 2^11 values on (a one-wave workgroup at 2^11: measured 18.6 ->
      // 12.6 us at n = 12 against two shifts per 128-thread workgroup)
      switch (NL) { HM_RO(10, 64, 3) HM_RO(11, 64, 3) HM_RO(12, 128, 3) HM_RO(13, 256, 3) HM_RO(14, 512, 4) default: break; }
    } else {
      switch (NL) { HM_RO(10, 64, 3) HM_RO(11, 128, 3) HM_RO(12, 256, 3) HM_RO(13, 512, 3) default: break; }
    }
#undef HM_RO
  }
#define HM_RS(nl)                                                   \
  case nl:                                                          \
    A.n_tiles = row_tiles<64, nl, nl>(A);                           \
    launch_row_q<T, 64, nl, nl, false>(A, q2, st);                  \
    return OK;
#define HM_RR(nl, nt)                                               \
  case nl:                                                          \
    A.n_tiles = row_tiles<nt, RB, nl>(A);                           \
    launch_row_q<T, nt, RB, nl, false>(A, q2, st);                  \
    return OK;
#define HM_RX(nl, nt)                                               \
  case nl:                                                          \
    A.n_tiles = row_tiles<nt, RB, nl>(A);                           \
    launch_row_q<T, nt, RB, nl, false, true>(A, q2, st);            \
    return OK;
  if constexpr (RB == 5) {
    switch (NL) {
      HM_RS(0) HM_RS(1) HM_RS(2) HM_RS(3) HM_RS(4)
      HM_RR(5, 128) HM_RR(6, 128) HM_RR(7, 128) HM_RR(8, 128) HM_RR(9, 128) HM_RR(10, 128) HM_RR(11, 128)
      HM_RR(12, 128) HM_RR(13, 256) HM_RX(14, 512) HM_RX(15, 1024)
      default: break;
    }
  } else {
    switch (NL) {
      HM_RS(0) HM_RS(1) HM_RS(2) HM_RS(3)
      HM_RR(4, 128) HM_RR(5, 128) HM_RR(6, 128) HM_RR(7, 128) HM_RR(8, 128) HM_RR(9, 128) HM_RR(10, 128)
      HM_RR(11, 128) HM_RR(12, 256) HM_RX(13, 512) HM_RX(14, 1024)
      default: break;
    }
  }
#undef HM_RS
#undef HM_RR
#undef HM_RX
  return fail(E_UNSUPPORTED, "resident row pass: no kernel for 2^%d values", NL);
}

// Two-pass row pass: rows of 2^NL values, tiles of 2^12 values (2^13 for NL = 13), RB register bits.
template <typename T, int RB, bool SPLIT>
static int launch_rowwrite_rb(int NL, RowPassArgs A, hipStream_t st) {
  constexpr int NT12 = 1 << (12 - RB), NT13 = 1 << (13 - RB), NT14 = 1 << (14 - RB), NT15 = 1 << (15 - RB);
#define HM_RW(nl, nt)                                               \
  case nl:                                                          \
    A.n_tiles = row_tiles<nt, RB, nl>(A);                           \
    launch_row_q<T, nt, RB, nl, true, SPLIT>(A, false, st);         \
    return OK;
  switch (NL) {
    HM_RW(6, NT12) HM_RW(7, NT12) HM_RW(8, NT12) HM_RW(9, NT12) HM_RW(10, NT12) HM_RW(11, NT12) HM_RW(12, NT12)
    HM_RW(13, NT13)
    // rows of 2^14 / 2^15 values (workgroups of 512 / 1024 threads with 2^5-value FP32 tiles): the
    // long rows that keep the column tiles wide from 2^21 folded values on
    case 14:
      if constexpr (sizeof(T) == 4 && NT14 <= 1024) {
        A.n_tiles = row_tiles<NT14, RB, 14>(A);
        launch_row_q<T, NT14, RB, 14, true, SPLIT>(A, false, st);
        return OK;
      }
      break;
    case 15:  // split staging only: whole-complex staging needs more registers than 1024 threads have
      if constexpr (sizeof(T) == 4 && NT15 <= 1024 && SPLIT) {
        A.n_tiles = row_tiles<NT15, RB, 15>(A);
        launch_row_q<T, NT15, RB, 15, true, SPLIT>(A, false, st);
        return OK;
      }
      break;
    default: break;
  }
#undef HM_RW
  return fail(E_UNSUPPORTED, "row pass: no kernel for rows of 2^%d values (RB %d)", NL, RB);
}

// Split LDS staging is built for 2^5 and 2^4 FP32 and 2^4 FP64 register tiles.
template <typename T>
static int launch_rowwrite(int rb, int NL, RowPassArgs A, bool split, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (rb == 5) return split ? launch_rowwrite_rb<T, 5, true>(NL, A, st) : launch_rowwrite_rb<T, 5, false>(NL, A, st);
    if (rb == 4) return split ? launch_rowwrite_rb<T, 4, true>(NL, A, st) : launch_rowwrite_rb<T, 4, false>(NL, A, st);
  } else {
    if (rb == 4) return split ? launch_rowwrite_rb<T, 4, true>(NL, A, st) : launch_rowwrite_rb<T, 4, false>(NL, A, st);
  }
  return fail(E_UNSUPPORTED, "row pass: register tile 2^%d (split %d) not built for this dtype", rb, (int)split);
}

template <typename T, int NT, int RB, int NH, bool SPLIT>
static void launch_col_nh(ColPassArgs A, bool q2, hipStream_t st) {
  constexpr int CB = ilog2c(NT) + RB - NH;
  A.n_cb = (int64_t)1 << (A.nl - CB);
  A.n_tiles = A.n_slots * A.n_cb;
  ProfScope prof("sre_colpass", st);
  for (A.tile0 = 0; A.tile0 < A.n_tiles; A.tile0 += MAX_GRID) {  // the first chunk also sums the previous batch
    const dim3 grid((unsigned)grid_for(A.n_tiles - A.tile0)), block(NT);
    if (q2) hipLaunchKernelGGL((k_sre_colpass<T, NT, RB, NH, CB, 2, SPLIT>), grid, block, 0, st, A);
    else hipLaunchKernelGGL((k_sre_colpass<T, NT, RB, NH, CB, 0, SPLIT>), grid, block, 0, st, A);
  }
}

// Column tiles of 2^col_tb values (col_tb - rb thread bits), RB register bits.
template <typename T, int RB, int TBC, bool SPLIT>
static int launch_col_tb(int NH, ColPassArgs &A, bool q2, hipStream_t st) {
  constexpr int NT = 1 << (TBC - RB);
#define HM_C(nh)                                                    \
  case nh:                                                          \
    if constexpr (nh >= RB && nh <= TBC) {                          \
      launch_col_nh<T, NT, RB, nh, SPLIT>(A, q2, st);               \
      return OK;                                                    \
    }                                                               \
    break;
  switch (NH) { HM_C(4) HM_C(5) HM_C(6) HM_C(7) HM_C(8) HM_C(9) HM_C(10) HM_C(11) HM_C(12) HM_C(13) default: break; }
#undef HM_C
  return fail(E_UNSUPPORTED, "column pass: no kernel for 2^%d rows (tile 2^%d, RB %d)", NH, TBC, RB);
}

template <typename T>
static int launch_colpass(int rb, int col_tb, int NH, ColPassArgs &A, bool q2, bool split, hipStream_t st) {
  if (A.nl < col_tb - NH) return fail(E_UNSUPPORTED, "column pass: rows of 2^%d too short for 2^%d-row tiles", A.nl, NH);
  if constexpr (sizeof(T) == 4) {
    if (rb == 5 && col_tb == 13)
      return split ? launch_col_tb<T, 5, 13, true>(NH, A, q2, st) : launch_col_tb<T, 5, 13, false>(NH, A, q2, st);
    if (rb == 5 && col_tb == 11)
      return split ? launch_col_tb<T, 5, 11, true>(NH, A, q2, st) : launch_col_tb<T, 5, 11, false>(NH, A, q2, st);
    if (rb == 4 && col_tb == 13 && !split) return launch_col_tb<T, 4, 13, false>(NH, A, q2, st);
    if (rb == 4 && col_tb == 11 && !split) return launch_col_tb<T, 4, 11, false>(NH, A, q2, st);
  } else {
    if (rb == 4 && col_tb == 12)
      return split ? launch_col_tb<T, 4, 12, true>(NH, A, q2, st) : launch_col_tb<T, 4, 12, false>(NH, A, q2, st);
    if (rb == 4 && col_tb == 10)
      return split ? launch_col_tb<T, 4, 10, true>(NH, A, q2, st) : launch_col_tb<T, 4, 10, false>(NH, A, q2, st);
  }
  return fail(E_UNSUPPORTED, "column pass: tile 2^%d with RB %d (split %d) not built for this dtype", col_tb, rb,
              (int)split);
}

template <typename T>
int shift_sums_t(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
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
    int e = launch_resident<T>(p.nf, A, q2, st, p.split != 0);
    if (e) return e;
    return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE row pass launch: %s", hipGetErrorString(hipGetLastError()));
  }
  // Two-pass: per batch, row pass (writes the exchange) then column pass (reads it, writes per
  // column-block partials and reduces the previous batch's partials to per-shift sums).
  if (p.pipe) return sizeof(T) == 4 ? sre_pipe_f32(p, psi, qa, a0, rows, n_slots, shift_sums, w, st)
                                    : sre_pipe_f64(p, psi, qa, a0, rows, n_slots, shift_sums, w, st);
  // Sequential launches on one or two streams.  With two streams, batch k goes to stream k mod 2
  // (the caller's stream and an internal one forked from it), each with its own exchange buffer and
  // partials, so one stream's row pass (exchange writes) overlaps the other's column pass (reads).
  const int64_t n_cb = sre_col_blocks(p);
  const int L = p.streams == 2 && n_slots > p.batch ? 2 : 1;
  const size_t xb = sre_exch_bytes(p);
  const size_t pbytes = align256((size_t)p.batch * (size_t)n_cb * nacc * sizeof(double));
  struct Lane {
    hipStream_t st;
    void *exch;
    double *partials[2];
    int64_t prev_s0, prev_nb;
    int k;
  } lane[2];
  for (int l = 0; l < L; ++l) {
    char *b = w + (size_t)l * (xb + 2 * pbytes);
    lane[l].exch = b;
    lane[l].partials[0] = (double *)(b + xb);
    lane[l].partials[1] = (double *)(b + xb + pbytes);
    lane[l].prev_s0 = lane[l].prev_nb = 0;
    lane[l].k = 0;
  }
  lane[0].st = st;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  if (L == 2) {
    int e = side_stream(&lane[1].st);
    if (e) return e;
    if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess)
      return fail(E_HIP, "SRE: event creation failed");
    if (hipEventRecord(ev_fork, st) != hipSuccess || hipStreamWaitEvent(lane[1].st, ev_fork, 0) != hipSuccess)
      return fail(E_HIP, "SRE: stream fork failed");
  }
  int64_t bi = 0;
  for (int64_t s0 = 0; s0 < n_slots; s0 += p.batch, ++bi) {
    Lane &ln = lane[bi % L];
    const int64_t nb = (n_slots - s0) < p.batch ? (n_slots - s0) : p.batch;
    RowPassArgs A{};
    A.psi = psi;
    A.nf = p.nf;
    A.nh = p.nh;
    A.n_slots = nb;
    A.a0 = a0 + (uint64_t)s0;
    A.rows = rows ? rows + s0 : nullptr;
    A.exch = ln.exch;
    A.nacc = nacc;
    A.qa = qa;
    int e = launch_rowwrite<T>(p.row_rb, p.nl, A, p.split != 0, ln.st);
    if (e) return e;
    ColPassArgs C{};
    C.exch = ln.exch;
    C.nl = p.nl;
    C.n_slots = nb;
    C.partials = ln.partials[ln.k & 1];
    C.nacc = nacc;
    C.qa = qa;
    C.nf = p.nf;
    C.prev_partials = ln.partials[(ln.k + 1) & 1];
    C.prev_n_slots = ln.prev_nb;
    C.prev_a0 = a0 + (uint64_t)ln.prev_s0;
    C.prev_rows = rows ? rows + ln.prev_s0 : nullptr;
    C.prev_shift_sums = shift_sums + ln.prev_s0 * nacc;
    e = launch_colpass<T>(p.col_rb, p.col_tb, p.nh, C, q2, p.split != 0, ln.st);
    if (e) return e;
    ln.prev_s0 = s0;
    ln.prev_nb = nb;
    ++ln.k;
  }
  for (int l = 0; l < L; ++l) {
    Lane &ln = lane[l];
    ProfScope prof("sre_shift_reduce", ln.st);
    hipLaunchKernelGGL(k_sre_shift_reduce, dim3(shift_reduce_grid(ln.prev_nb)), dim3(SHIFT_REDUCE_NT), 0, ln.st,
                       ln.partials[(ln.k + 1) & 1], ln.prev_nb, n_cb, nacc, a0 + (uint64_t)ln.prev_s0,
                       rows ? rows + ln.prev_s0 : nullptr, p.nf, qa, shift_sums + ln.prev_s0 * nacc);
  }
  if (L == 2) {
    const bool ok = hipEventRecord(ev_join, lane[1].st) == hipSuccess && hipStreamWaitEvent(st, ev_join, 0) == hipSuccess;
    (void)hipEventDestroy(ev_fork);
    (void)hipEventDestroy(ev_join);
    if (!ok) return fail(E_HIP, "SRE: stream join failed");
  }
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE two-pass launch: %s", hipGetErrorString(hipGetLastError()));
}


// ------------------------------------------------------------------------------------------------
// Pipelined two-pass: launch k runs the row pass of batch k (into exchange buffer k & 1) and the
// column pass of batch k - 1 (from buffer (k - 1) & 1) side by side, so exchange writes and reads
// are in flight together and the number of launches is halved.  Kernel boundaries order everything:
// buffer k & 1 is rewritten by launch k + 2, after launch k + 1 has read it.  Blocks alternate
// between the two parts while both have tiles left.
// ------------------------------------------------------------------------------------------------
struct PairArgs {
  RowPassArgs row;  // row.n_tiles = 0 in the last launch
  ColPassArgs col;  // col.n_tiles = 0 in the first launch
};

template <typename T, int NT, int RB, int NL, int NH, int CB, int QM, bool SPLIT>
__global__ __launch_bounds__(NT) void k_sre_pair(PairArgs P) {
  using RS = RowShape<T, NT, RB, NL, SPLIT>;
  using CS = ColShape<T, NT, RB, NH, CB, SPLIT>;
  constexpr size_t LB = RS::LDS_BYTES > CS::LDS_BYTES ? RS::LDS_BYTES : CS::LDS_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[LB];
  __shared__ double red[NT / 64 + 1];
  const int64_t nr = P.row.n_tiles, nc = P.col.n_tiles;
  const int64_t m = nr < nc ? nr : nc;
  const int64_t b = blockIdx.x;
  bool is_row;
  int64_t t;
  if (b < 2 * m) {
    is_row = (b & 1) == 0;
    t = b >> 1;
  } else {
    is_row = nr > nc;
    t = b - m;
  }
  if (is_row) {
    rowpass_tiles<T, NT, RB, NL, true, 0, SPLIT>(P.row, t, nr, (typename RS::Elem *)lds_raw, red);
  } else {
    const ColPassArgs &C = P.col;
    reduce_prev_shifts(C, t * (NT / 64), nc * (NT / 64));
    colpass_tiles<T, NT, RB, NH, CB, QM, SPLIT>(C, t, nc, (typename CS::Elem *)lds_raw, red);
  }
}

template <typename T, int RB, int NF, bool SPLIT>
static void launch_pair_nf(PairArgs &P, bool q2, hipStream_t st) {
  constexpr int TB = sre_default_col_tb(NF, sizeof(T) == 8, RB);
  constexpr int NL = sre_default_nl(NF, TB, RB);
  constexpr int NH = NF - NL;
  constexpr int CB = TB - NH;
  constexpr int NT = 1 << (TB - RB);
  static_assert(NH >= RB && CB >= 0 && NL >= CB && NL <= TB, "pipelined tile shape");
  P.row.n_tiles = P.row.n_slots > 0 ? row_tiles<NT, RB, NL>(P.row) : 0;
  P.col.n_cb = (int64_t)1 << (P.col.nl - CB);
  P.col.n_tiles = P.col.n_slots * P.col.n_cb;
  const dim3 grid((unsigned)(P.row.n_tiles + P.col.n_tiles)), block(NT);
  ProfScope prof("sre_pair", st);
  if (q2) hipLaunchKernelGGL((k_sre_pair<T, NT, RB, NL, NH, CB, 2, SPLIT>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((k_sre_pair<T, NT, RB, NL, NH, CB, 0, SPLIT>), grid, block, 0, st, P);
}

template <typename T, bool SPLIT>
static int launch_pair(int nf, PairArgs &P, bool q2, hipStream_t st) {
  constexpr int RB = ResidentRB<T>::value;
#define HM_P(nf_)                                                   \
  case nf_:                                                         \
    launch_pair_nf<T, RB, nf_, SPLIT>(P, q2, st);                   \
    return OK;
  switch (nf) {
    HM_P(11) HM_P(12) HM_P(13) HM_P(14) HM_P(15) HM_P(16) HM_P(17) HM_P(18) HM_P(19) HM_P(20) HM_P(21) HM_P(22)
    HM_P(23) HM_P(24)
    case 25:
      if constexpr (sizeof(T) == 4) {  // FP64 rows of 2^13 do not fit its 2^12-value tiles
        launch_pair_nf<T, RB, 25, SPLIT>(P, q2, st);
        return OK;
      }
      break;
    default: break;
  }
#undef HM_P
  return fail(E_UNSUPPORTED, "pipelined SRE: no kernel for 2^%d folded values", nf);
}

template <typename T>
int pipe_shift_sums_t(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                      int64_t n_slots, double *shift_sums, char *w, hipStream_t st) {
  if (!sre_pipe_built(p)) return fail(E_UNSUPPORTED, "pipelined SRE: plan not built (n = %d)", p.N);
  const bool q2 = is_q2(qa);
  const int nacc = nacc_of(qa);
  const int64_t n_cb = sre_col_blocks(p);
  const size_t xb = sre_exch_bytes(p) / 2;
  void *exch[2] = {w, w + xb};
  const size_t pbytes = align256((size_t)p.batch * (size_t)n_cb * nacc * sizeof(double));
  double *partials[2] = {(double *)(w + 2 * xb), (double *)(w + 2 * xb + pbytes)};
  const int64_t nbat = (n_slots + p.batch - 1) / p.batch;
  auto b0 = [&](int64_t k) { return k * (int64_t)p.batch; };
  auto bn = [&](int64_t k) { return (n_slots - b0(k)) < p.batch ? (n_slots - b0(k)) : (int64_t)p.batch; };
  for (int64_t k = 0; k <= nbat; ++k) {
    PairArgs P{};
    if (k < nbat) {
      RowPassArgs &A = P.row;
      A.psi = psi;
      A.nf = p.nf;
      A.nh = p.nh;
      A.n_slots = bn(k);
      A.a0 = a0 + (uint64_t)b0(k);
      A.rows = rows ? rows + b0(k) : nullptr;
      A.exch = exch[k & 1];
      A.nacc = nacc;
      A.qa = qa;
    }
    if (k >= 1) {
      ColPassArgs &C = P.col;
      C.exch = exch[(k - 1) & 1];
      C.nl = p.nl;
      C.n_slots = bn(k - 1);
      C.partials = partials[(k - 1) & 1];
      C.nacc = nacc;
      C.qa = qa;
      C.nf = p.nf;
      if (k >= 2) {
        C.prev_partials = partials[k & 1];
        C.prev_n_slots = bn(k - 2);
        C.prev_a0 = a0 + (uint64_t)b0(k - 2);
        C.prev_rows = rows ? rows + b0(k - 2) : nullptr;
        C.prev_shift_sums = shift_sums + b0(k - 2) * nacc;
      }
    }
    const int e = p.split ? launch_pair<T, true>(p.nf, P, q2, st) : launch_pair<T, false>(p.nf, P, q2, st);
    if (e) return e;
  }
  {
    const int64_t k = nbat - 1;
    ProfScope prof("sre_shift_reduce", st);
    hipLaunchKernelGGL(k_sre_shift_reduce, dim3(shift_reduce_grid(bn(k))), dim3(SHIFT_REDUCE_NT), 0, st,
                       partials[k & 1], bn(k), n_cb, nacc, a0 + (uint64_t)b0(k), rows ? rows + b0(k) : nullptr, p.nf,
                       qa, shift_sums + b0(k) * nacc);
  }
  return hipPeekAtLastError() == hipSuccess ? OK
                                            : fail(E_HIP, "SRE pipelined launch: %s", hipGetErrorString(hipGetLastError()));
}

// Batched states of one size on the workgroup-resident path (one launch for up to HM_BATCH_PTRS states).
template <typename T>
int states_t(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *shift_sums,
             hipStream_t st) {
  RowPassArgs A{};
  A.psi = psis[0];
  A.nf = p.nf;
  A.nh = 0;
  A.n_slots = (int64_t)n_states << p.N;
  A.shift_sums = shift_sums;
  A.nacc = nacc_of(qa);
  A.qa = qa;
  A.n_states = n_states;
  A.state_bits = p.N;
  for (int i = 0; i < n_states; ++i) A.psis[i] = psis[i];
  int e = launch_resident<T>(p.nf, A, is_q2(qa), st, p.split != 0);
  if (e) return e;
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE batched launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace
}  // namespace hm
