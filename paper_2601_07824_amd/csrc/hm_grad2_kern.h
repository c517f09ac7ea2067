// hm_grad2_kern.h -- two-pass fused forward + adjoint of M_q for states too large for one
// workgroup (the gradient formulas are those of hm_grad.hip).  Per batch of X-shifts:
//   1. row pass (forward, as for M_q): product and the row stages, into the exchange buffer;
//   2. column pass with ADJ: the column stages, the sums of |chi|^2 and |chi|^{2q}, the adjoint
//      seed |k U|^{2q-2} U, the column stages again in reverse order, written back in place;
//   3. backward row pass: the row stages in reverse order, leaving Z = H^{(x)(N-1)} w in natural
//      folded order (in place);
//   4. accumulation: each workgroup owns a block of y and a group of the batch's shifts and adds
//      2q psi_{y^a} [Z or conj Z]_{c(y)} (the unfolded form of the folded update) in registers,
//      then into its own FP64 partial of G; no two workgroups write the same partial element, so
//      no atomics are needed and the result is deterministic.
// After the last batch, a fixed-order sum over the groups' partials, times 2 / ((1-q) S_q ln 2),
// gives the gradient.
#pragma once
#include "hm_sre_kern.h"

namespace hm {
namespace {

// Adjoint column pass (step 2), with the per-shift reduction of the previous batch's partials.
template <typename T, int NT, int RB, int NH, int CB, int QM, bool SPLIT>
__global__ __launch_bounds__(NT) void k_sre_colpass_adj(ColPassArgs A) {
  using Sh = ColShape<T, NT, RB, NH, CB, SPLIT>;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  __shared__ double red[NT / 64 + 1];
  if (A.tile0 == 0) reduce_prev_shifts(A, (int64_t)blockIdx.x * (NT / 64), (int64_t)gridDim.x * (NT / 64));
  colpass_tiles<T, NT, RB, NH, CB, QM, SPLIT, true, true, true>(A, A.tile0 + blockIdx.x, gridDim.x, lds, red);
}

// Backward row pass: rows of 2^NL adjoint values, read in the row pass's output layout (register
// r of thread tlo holds row position r | (tlo << RB) at column (r << S0) | tlo), stages in reverse
// round order, written back in natural order (position tlo + (r << S0)).
template <typename T, int NT, int RB, int NL, bool SPLIT>
__global__ __launch_bounds__(NT) void k_sre_rowback(RowPassArgs A) {
  using Sh = RowShape<T, NT, RB, NL, SPLIT>;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  constexpr int R = 1 << RB;
  constexpr int LT = ilog2c(NT);
  constexpr int TB = LT + RB;
  static_assert(TB >= NL && NL >= RB, "tile must hold whole rows");
  constexpr int S0 = NL - RB;
  constexpr int K = (NL + RB - 1) / RB;
  static_assert(K >= 2 && K <= 4, "two to four rounds");
  constexpr int SEG = 1 << S0;
  constexpr int G = 1 << (TB - NL);
  vec2<T> *__restrict__ ex = (vec2<T> *)A.exch;
  const uint32_t tau = threadIdx.x;
  const uint32_t tlo = tau & (SEG - 1);
  const uint32_t g = tau >> S0;
  for (int64_t tile = blockIdx.x; tile < A.n_tiles; tile += gridDim.x) {
    const int64_t rt = tile * G + g;
    const bool active = (rt >> A.nh) < A.n_slots;
    const uint32_t ob = ((uint32_t)rt << NL) | tlo;
    T re[R], im[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vec2<T> v{T(0), T(0)};
      if (active) v = ld32(ex, ob + ((uint32_t)r << S0));
      re[r] = v.x;
      im[r] = v.y;
    }
    if constexpr (K >= 4) {
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(re, im);
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 3), rp_S(NL, RB, 2)>(re, im, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 3), rp_S(NL, RB, 2)>(re, im, lds, tau);
    }
    if constexpr (K >= 3) {
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(re, im);
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 1)>(re, im, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 1)>(re, im, lds, tau);
    }
    wht_regs<T, R, 0, rp_H(NL, RB, 1)>(re, im);
    if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 0)>(re, im, lds, tau);
    else relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 0)>(re, im, lds, tau);
    wht_regs<T, R, 0, rp_H(NL, RB, 0)>(re, im);
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vec2<T> v;
        v.x = re[r];
        v.y = im[r];
        st32(ex, ob + ((uint32_t)r << S0), v);
      }
    }
  }
}

// ---- fused backward row pass + accumulation ------------------------------------------------------
// For a batch whose shifts a share their top bit j (and, when j >= NL, their bits above NL), row ch
// of the folded vector maps, for every shift of the batch, onto the same two sets of gradient
// entries: the x side y = x(c) (bit j clear) and the partner side y = x(c) ^ a (bit j set), with
// the partner's position inside its block permuted by the shift's low bits.  One workgroup takes one
// row for a group of the batch's shifts (G shifts at a time, one per row task), runs the backward row
// stages, and accumulates the x side in registers and the partner side in per-row-task LDS slices;
// the slices are then summed in fixed order and added to the group's FP64 partial of G.  Rows own
// disjoint entries, so there are no atomics and the result is deterministic.
struct FusedArgs {
  const void *psi;
  const void *exch;   // adjoint rows after the column pass, row-pass output layout
  int nf, nh;
  int64_t n_slots;
  uint64_t a0;
  double q;
  int j;              // common top bit of the batch's shifts
  uint32_t ah;        // common a >> NL (used when j >= NL)
  double2 *gpart;     // [groups][2^N]
  int groups;
};

// RBW: register tile of the row pass that wrote the exchange (its column permutation: row position
// P sits at column (P mod 2^RBW) 2^(NL-RBW) + P / 2^RBW).  RB <= RBW is this kernel's own tile.
// Waves per SIMD the fused kernel is compiled for (the grid's own depth at the gradient's largest
// batches): four (at most 128 VGPRs) for 2^3-value FP32 tiles, two (at most 256) for 2^4-value
// FP32 and 2^3-value FP64 tiles, one otherwise.
constexpr int fused_waves(int rb, int tbytes) { return (tbytes << rb) <= 32 ? 4 : (tbytes << rb) <= 64 ? 2 : 1; }

template <typename T, int NT, int RB, int RBW, int NL, bool SPLIT>
__global__ __launch_bounds__(NT, fused_waves(RB, sizeof(T))) void k_grad_rowback_accum(FusedArgs F) {
  using Sh = RowShape<T, NT, RB, NL, SPLIT>;
  constexpr int R = 1 << RB;
  constexpr int LT = ilog2c(NT);
  constexpr int TB = LT + RB;
  static_assert(TB >= NL && NL >= RB, "tile must hold whole rows");
  constexpr int S0 = NL - RB;
  constexpr int K = (NL + RB - 1) / RB;
  static_assert(K >= 2 && K <= 4, "two to four rounds");
  constexpr int SEG = 1 << S0;       // threads per row task
  constexpr int G = 1 << (TB - NL);  // row tasks (shifts in flight) per workgroup
  constexpr int ROW = 1 << NL;
  __shared__ typename Sh::Elem lds[Sh::LDS_N];
  __shared__ vec2<T> slice[G * ROW];

  const vec2<T> *__restrict__ ex = (const vec2<T> *)F.exch;
  const vec2<T> *__restrict__ psi = (const vec2<T> *)F.psi;
  const uint32_t tau = threadIdx.x;
  const uint32_t tlo = tau & (SEG - 1);
  const uint32_t g = tau >> S0;
  const int64_t nrows = (int64_t)1 << F.nh;
  const uint32_t ch = (uint32_t)((int64_t)blockIdx.x % nrows);
  const int grp = (int)((int64_t)blockIdx.x / nrows);
  const int64_t per = (F.n_slots + F.groups - 1) / F.groups;
  const int64_t s_lo = (int64_t)grp * per;
  const int64_t s_hi = (s_lo + per) < F.n_slots ? (s_lo + per) : F.n_slots;
  const int j = F.j;
  const bool jhi = j >= NL;
  // x side: y = x(c) for c = ch * ROW + p; partner block origin
  const uint32_t xh = jhi ? (uint32_t)ins0_32(ch, j - NL) : 0u;
  const T q4 = (T)(4.0 * F.q);

  for (uint32_t i = tau; i < (uint32_t)(G * ROW); i += NT) slice[i] = vec2<T>{T(0), T(0)};
  T axr[R], axi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) axr[r] = axi[r] = T(0);

  static_assert(RB <= RBW && RBW <= NL, "reader tile within the writer's");
  // Adjoint row of shift slot s in this kernel's layout S = 0: register r of thread tlo holds row
  // position P = r + R tlo, which the forward row pass stored at column
  // (P mod 2^RBW) 2^(NL-RBW) + P / 2^RBW.
  auto load_row = [&](int64_t s, T(&xr)[R], T(&xi)[R]) {
    const uint32_t ob = (((uint32_t)s << F.nh) + ch) << NL;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t P = (uint32_t)r + (tlo << RB);
      const uint32_t col = ((P & ((1u << RBW) - 1u)) << (NL - RBW)) | (P >> RBW);
      const vec2<T> v = ld32(ex, ob + col);
      xr[r] = v.x;
      xi[r] = v.y;
    }
  };
  auto backward_stages = [&](T(&xr)[R], T(&xi)[R]) {
    if constexpr (K >= 4) {
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(xr, xi);
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 3), rp_S(NL, RB, 2)>(xr, xi, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 3), rp_S(NL, RB, 2)>(xr, xi, lds, tau);
    }
    if constexpr (K >= 3) {
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(xr, xi);
      if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 1)>(xr, xi, lds, tau);
      else relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 1)>(xr, xi, lds, tau);
    }
    wht_regs<T, R, 0, rp_H(NL, RB, 1)>(xr, xi);
    if constexpr (SPLIT) relayout_split<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 0)>(xr, xi, lds, tau);
    else relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 0)>(xr, xi, lds, tau);
    wht_regs<T, R, 0, rp_H(NL, RB, 0)>(xr, xi);
  };
  // x-side gradient entry of register r (after the stages: row position p = tlo + r 2^S0); it does
  // not depend on the shift
  auto xpos = [&](int r) -> uint32_t {
    const uint32_t p = tlo + ((uint32_t)r << S0);
    return jhi ? ((xh << NL) | p) : ((ch << (NL + 1)) | ins0_32(p, j));
  };
  // Tiles of at most 64 B per register array (2^3 or 2^4 FP32, 2^3 FP64 values): the x-side state
  // values stay in registers for the whole loop, the next shift's row is loaded during the current
  // shift's stages, and the partner-side state values are gathered together.  2^4-value FP64 tiles
  // keep the one-value-at-a-time form (the pipelined arrays would need more than 256 VGPRs).
  constexpr bool PF = R * sizeof(T) <= 64;
  if constexpr (PF) {
    if (s_lo < s_hi) {  // uniform
      const int64_t s_last = s_hi - 1;
      T re[R], im[R];
      vec2<T> px[R];
      // row tasks past the group's last shift load that shift's row (valid data, not accumulated)
      load_row((s_lo + g) < s_last ? (s_lo + g) : s_last, re, im);
#pragma unroll
      for (int r = 0; r < R; ++r) px[r] = ld32(psi, xpos(r));
      for (int64_t sb = s_lo; sb < s_hi; sb += G) {
        const int64_t s = sb + g;
        const bool active = s < s_hi;
        const uint32_t a = (uint32_t)(F.a0 + (uint64_t)(active ? s : s_last));
        // next row (past the end: the last shift's row again, an L2 hit; no branch, so that the
        // loads stay in flight through the stages)
        T nre[R], nim[R];
        load_row((s + G) < s_last ? (s + G) : s_last, nre, nim);
        backward_stages(re, im);
        if (active) {
          const uint32_t m = jhi ? (a & (uint32_t)(ROW - 1)) : (a & ((1u << j) - 1u));  // partner position = p ^ m
          vec2<T> *sl = slice + g * ROW;
          vec2<T> py[R], o[R];
#pragma unroll
          for (int r = 0; r < R; ++r) py[r] = ld32(psi, xpos(r) ^ a);
#pragma unroll
          for (int r = 0; r < R; ++r) o[r] = sl[(tlo + ((uint32_t)r << S0)) ^ m];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const T zr = q4 * re[r], zi = q4 * im[r];
            // G_x += 4q psi_{x^a} Z ;  G_{x^a} += 4q psi_x conj(Z)
            axr[r] += fmaT(py[r].x, zr, -(py[r].y * zi));
            axi[r] += fmaT(py[r].x, zi, py[r].y * zr);
            o[r].x += fmaT(px[r].x, zr, px[r].y * zi);
            o[r].y += fmaT(px[r].y, zr, -(px[r].x * zi));
          }
#pragma unroll
          for (int r = 0; r < R; ++r) sl[(tlo + ((uint32_t)r << S0)) ^ m] = o[r];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          re[r] = nre[r];
          im[r] = nim[r];
        }
      }
    }
  } else {
    for (int64_t sb = s_lo; sb < s_hi; sb += G) {
      const int64_t s = sb + g;
      const bool active = s < s_hi;
      T re[R], im[R];
      load_row(active ? s : s_hi - 1, re, im);
      backward_stages(re, im);
      if (active) {
        const uint32_t a = (uint32_t)(F.a0 + (uint64_t)s);
        const uint32_t m = jhi ? (a & (uint32_t)(ROW - 1)) : (a & ((1u << j) - 1u));
        vec2<T> *sl = slice + g * ROW;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t p = tlo + ((uint32_t)r << S0);
          const uint32_t x = xpos(r);
          const vec2<T> py = ld32(psi, x ^ a), px = ld32(psi, x);
          const T zr = q4 * re[r], zi = q4 * im[r];
          axr[r] += fmaT(py.x, zr, -(py.y * zi));
          axi[r] += fmaT(py.x, zi, py.y * zr);
          vec2<T> o = sl[p ^ m];
          o.x += fmaT(px.x, zr, px.y * zi);
          o.y += fmaT(px.y, zr, -(px.x * zi));
          sl[p ^ m] = o;
          if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // keep the state gathers in groups of four
        }
      }
    }
  }
  if (s_lo >= s_hi) return;  // uniform: no shifts in this group
  double2 *gp = F.gpart + ((size_t)grp << (F.nf + 1));
  const uint32_t ah_sh = jhi ? ((xh ^ F.ah) << NL) : 0u;
  __syncthreads();
  // partner side: fixed-order sum over the row tasks' slices
  for (uint32_t p = tau; p < (uint32_t)ROW; p += NT) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < G; ++k) {
      const vec2<T> v = slice[k * ROW + p];
      sr += (double)v.x;
      si += (double)v.y;
    }
    const uint32_t y = jhi ? (ah_sh | p) : ((ch << (NL + 1)) | ins0_32(p, j) | (1u << j));
    double2 o = gp[y];
    o.x += sr;
    o.y += si;
    gp[y] = o;
  }
  __syncthreads();
  // x side: registers through the slices, then the same fixed-order sum
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t p = tlo + ((uint32_t)r << S0);
    slice[g * ROW + p] = vec2<T>{axr[r], axi[r]};
  }
  __syncthreads();
  for (uint32_t p = tau; p < (uint32_t)ROW; p += NT) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < G; ++k) {
      const vec2<T> v = slice[k * ROW + p];
      sr += (double)v.x;
      si += (double)v.y;
    }
    const uint32_t y = jhi ? ((xh << NL) | p) : ((ch << (NL + 1)) | ins0_32(p, j));
    double2 o = gp[y];
    o.x += sr;
    o.y += si;
    gp[y] = o;
  }
}

struct AccumArgs {
  const void *psi;
  const void *z;       // [n_slots][2^nf] adjoint values in natural folded order
  int nf;
  int64_t n_slots;
  uint64_t a0;
  double q;
  double2 *gpart;      // [groups][2^N]
  int groups;
  int64_t y_tiles;
};

// Gradient accumulation: block b -> y-tile b % y_tiles, shift group b / y_tiles; thread tau holds
// y = tile * (256 * V) + v * 256 + tau for v < V.
template <typename T, int V>
__global__ __launch_bounds__(256) void k_grad_accum(AccumArgs A) {
  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  const int64_t tile = (int64_t)blockIdx.x % A.y_tiles;
  const int grp = (int)((int64_t)blockIdx.x / A.y_tiles);
  const int64_t per = (A.n_slots + A.groups - 1) / A.groups;
  const int64_t s_lo = (int64_t)grp * per;
  const int64_t s_hi = (s_lo + per) < A.n_slots ? (s_lo + per) : A.n_slots;
  const uint32_t half = 1u << A.nf;
  const T q2 = (T)(2.0 * A.q), q4 = (T)(4.0 * A.q);
  uint32_t y[V];
  T gr[V], gi[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    y[v] = (uint32_t)(tile * (256 * V)) + (uint32_t)(v * 256) + threadIdx.x;
    gr[v] = gi[v] = T(0);
  }
  for (int64_t s = s_lo; s < s_hi; ++s) {
    const uint64_t a = A.a0 + (uint64_t)s;
    const vec2<T> *__restrict__ z = (const vec2<T> *)A.z + ((size_t)s << A.nf);
    if (a == 0) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint32_t c = y[v] & (half - 1u);
        const vec2<T> zc = ld32(z, c);
        const vec2<T> p = ld32(psi, y[v]);
        const T f = q2 * ((y[v] & half) ? (zc.x - zc.y) : (zc.x + zc.y));
        gr[v] = fmaT(f, p.x, gr[v]);
        gi[v] = fmaT(f, p.y, gi[v]);
      }
    } else {
      const int j = 63 - __builtin_clzll(a);
      const uint32_t lomask = (1u << j) - 1u;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint32_t yj = (y[v] >> j) & 1u;
        const uint32_t x = yj ? (y[v] ^ (uint32_t)a) : y[v];
        const uint32_t c = (x & lomask) | ((x >> (j + 1)) << j);
        vec2<T> zc = ld32(z, c);
        if (yj) zc.y = -zc.y;
        const vec2<T> p = ld32(psi, y[v] ^ (uint32_t)a);
        // G_y += 4q psi_{y^a} zc
        gr[v] = fmaT(q4, fmaT(p.x, zc.x, -(p.y * zc.y)), gr[v]);
        gi[v] = fmaT(q4, fmaT(p.x, zc.y, p.y * zc.x), gi[v]);
      }
    }
  }
  if (s_lo >= s_hi) return;
  double2 *gp = A.gpart + ((size_t)grp << (A.nf + 1));
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double2 o = gp[y[v]];
    o.x += (double)gr[v];
    o.y += (double)gi[v];
    gp[y[v]] = o;
  }
}

// grad[y] = scale * sum over the groups' partials: a workgroup takes 64 consecutive y (one per lane)
// x 16 strided sets of groups (one per wave), then wave 0 adds the 16 set sums in order.
template <typename T>
__global__ __launch_bounds__(1024) void k_grad2_final(const double2 *gpart, int groups, int64_t n, const double *scale,
                                                      vec2<T> *grad) {
  constexpr int FY = 64, FG = 16;
  __shared__ double sr[FG][FY], si[FG][FY];
  const uint32_t ly = threadIdx.x % FY, g = threadIdx.x / FY;
  const int64_t y = (int64_t)blockIdx.x * FY + ly;
  double gr = 0.0, gi = 0.0;
  if (y < n) {
    for (int k = (int)g; k < groups; k += FG) {
      const double2 v = gpart[(size_t)k * n + y];
      gr += v.x;
      gi += v.y;
    }
  }
  sr[g][ly] = gr;
  si[g][ly] = gi;
  __syncthreads();
  if (g == 0 && y < n) {
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int k = 0; k < FG; ++k) {
      tr += sr[k][ly];
      ti += si[k][ly];
    }
    vec2<T> o;
    o.x = (T)(scale[0] * tr);
    o.y = (T)(scale[0] * ti);
    grad[y] = o;
  }
}

__global__ void k_zero2(double2 *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = double2{0.0, 0.0};
}

// Register tile of the fused backward-row + accumulation kernel: 2^3 values per thread for rows of
// 2^8 and 2^9 (half the registers of 2^4, so twice the waves; measured faster there), 2^4 otherwise
// (rows of 2^10 would need a fourth round).
constexpr int fused_rb(int nl) { return nl == 8 || nl == 9 ? 3 : 4; }
// Workgroup size of the fused kernel: 256 threads for FP32 rows of 2^8..2^10 values and FP64 rows of
// 2^8..2^9 (twice the shifts in flight per workgroup; the launch then uses half as many shift
// groups, so the waves in flight stay the same and the FP64 partials of G read and written per
// launch halve), 128 otherwise.
constexpr int fused_nt(int nl, int tbytes) {
  return (tbytes == 4 && nl >= 8 && nl <= 10) || (tbytes == 8 && nl >= 8 && nl <= 9) ? 256 : 128;
}
// Register tile of the gradient's forward row pass (the plan's row_rb), which fixes the exchange's
// column permutation.
constexpr int GRAD_ROW_RB = 4;

// ---- launchers (default two-pass split only) -----------------------------------------------------
template <typename T, int RB, int NF, bool SPLIT>
static void grad2_launch_nf(int step, RowPassArgs &A, ColPassArgs &C, const FusedArgs *F, bool q2, hipStream_t st) {
  constexpr int TB = sre_default_col_tb(NF, sizeof(T) == 8, RB);
  constexpr int NL = sre_default_nl(NF, TB, RB);
  constexpr int NH = NF - NL;
  constexpr int CB = TB - NH;
  // Register tile of the adjoint column pass: 2^4 values per thread (four waves per SIMD); for FP32
  // columns of 2^9 rows 2^5 (two waves per SIMD, more loads in flight per wave; measured on one
  // MI355X at n = 19 / 20: 116.0 -> 113.7 / 115.9 -> 110.6 us per launch, fwd+grad 2 % faster; at
  // 2^8 rows 2^4 stays faster).
  constexpr int RBC = (sizeof(T) == 4 && NH >= 9) ? 5 : 4;
  constexpr int NTC = 1 << (TB - RBC);
  if (step == 2) {
    C.n_cb = (int64_t)1 << (C.nl - CB);
    C.n_tiles = C.n_slots * C.n_cb;
    ProfScope prof("sre_grad_colpass", st);
    for (C.tile0 = 0; C.tile0 < C.n_tiles; C.tile0 += MAX_GRID) {
      const dim3 grid((unsigned)grid_for(C.n_tiles - C.tile0)), block(NTC);
      if (q2) hipLaunchKernelGGL((k_sre_colpass_adj<T, NTC, RBC, NH, CB, 2, SPLIT>), grid, block, 0, st, C);
      else hipLaunchKernelGGL((k_sre_colpass_adj<T, NTC, RBC, NH, CB, 0, SPLIT>), grid, block, 0, st, C);
    }
  } else if (step == 3) {
    // row tiles of 2^4 values per thread on the row side of the gradient (the plan's row_rb)
    constexpr int RBR = 4;
    constexpr int TBR = NL > 12 ? 13 : 12;
    constexpr int NTR = 1 << (TBR - RBR);
    A.n_tiles = row_tiles<NTR, RBR, NL>(A);
    const dim3 grid((unsigned)grid_for(A.n_tiles)), block(NTR);
    ProfScope prof("sre_grad_rowback", st);
    hipLaunchKernelGGL((k_sre_rowback<T, NTR, RBR, NL, SPLIT>), grid, block, 0, st, A);
  } else {
    // fused backward rows + accumulation: NTF threads x 2^RBR values, NTF 2^RBR / 2^NL shifts in
    // flight
    constexpr int RBR = fused_rb(NL);
    constexpr int NTF = fused_nt(NL, sizeof(T));
    static_assert(ilog2c(NTF) + RBR >= NL, "fused tile must hold a whole row");
    const dim3 grid((unsigned)(((int64_t)1 << F->nh) * F->groups)), block(NTF);
    ProfScope prof("sre_grad_rowback_accum", st);
    hipLaunchKernelGGL((k_grad_rowback_accum<T, NTF, RBR, GRAD_ROW_RB, NL, SPLIT>), grid, block, 0, st, *F);
  }
}

template <typename T, bool SPLIT>
static int grad2_launch(int nf, int step, RowPassArgs &A, ColPassArgs &C, const FusedArgs *F, bool q2,
                        hipStream_t st) {
  constexpr int RB = ResidentRB<T>::value;
#define HM_G2(nf_)                                                  \
  case nf_:                                                         \
    grad2_launch_nf<T, RB, nf_, SPLIT>(step, A, C, F, q2, st);      \
    return OK;
  switch (nf) {
    HM_G2(11) HM_G2(12) HM_G2(13) HM_G2(14) HM_G2(15) HM_G2(16) HM_G2(17) HM_G2(18) HM_G2(19)
    default: break;
  }
#undef HM_G2
  return fail(E_UNSUPPORTED, "two-pass gradient: no kernels for 2^%d folded values", nf);
}

static inline int grad2_groups(int N) {
  const int64_t tiles = ((int64_t)1 << N) / 1024;
  int64_t g = 2048 / (tiles > 0 ? tiles : 1);
  return (int)(g < 1 ? 1 : g > 256 ? 256 : g);
}

static inline size_t grad2_workspace(const SrePlan &p) {
  const size_t n = (size_t)1 << p.N;
  return align256(n * 2 * sizeof(double)) + sre_exch_bytes(p) +
         2 * align256((size_t)p.batch * (size_t)sre_col_blocks(p) * 2 * sizeof(double)) +
         align256((size_t)grad2_groups(p.N) * n * sizeof(double2)) + 256;
}

template <typename T>
int grad2_t(const SrePlan &p, const void *psi, double q, double *out, void *grad, char *w, hipStream_t st) {
  const int N = p.N, nf = p.nf;
  const int64_t n_shifts = (int64_t)1 << N;
  QArgs qa{};
  qa.nq = 1;
  qa.q[0] = q;
  const bool q2 = q == 2.0;
  const int nacc = 2;
  const int groups = grad2_groups(N);
  const int64_t n_cb = sre_col_blocks(p);
  // workspace: [shift sums][exchange][partials x 2][G partials][scale]
  double *shift_sums = (double *)w;
  w += align256((size_t)n_shifts * nacc * sizeof(double));
  void *exch = w;
  w += sre_exch_bytes(p);
  const size_t pbytes = align256((size_t)p.batch * (size_t)n_cb * nacc * sizeof(double));
  double *partials[2] = {(double *)w, (double *)(w + pbytes)};
  w += 2 * pbytes;
  double2 *gpart = (double2 *)w;
  w += align256((size_t)groups * (size_t)n_shifts * sizeof(double2));
  double *scale = (double *)w;
  {
    const int64_t n = (int64_t)groups * n_shifts;
    hipLaunchKernelGGL(k_zero2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gpart, n);
  }
  int64_t prev_s0 = 0, prev_nb = 0;
  int k = 0;
  for (int64_t s0 = 0; s0 < n_shifts; s0 += p.batch, ++k) {
    const int64_t nb = (n_shifts - s0) < p.batch ? (n_shifts - s0) : p.batch;
    RowPassArgs A{};
    A.psi = psi;
    A.nf = nf;
    A.nh = p.nh;
    A.n_slots = nb;
    A.a0 = (uint64_t)s0;
    A.exch = exch;
    A.nacc = nacc;
    A.qa = qa;
    int e = launch_rowwrite<T>(p.row_rb, p.nl, A, p.split != 0, st);
    if (e) return e;
    ColPassArgs C{};
    C.exch = exch;
    C.nl = p.nl;
    C.n_slots = nb;
    C.partials = partials[k & 1];
    C.nacc = nacc;
    C.qa = qa;
    C.nf = nf;
    C.a0 = (uint64_t)s0;
    C.prev_partials = partials[(k + 1) & 1];
    C.prev_n_slots = prev_nb;
    C.prev_a0 = (uint64_t)prev_s0;
    C.prev_shift_sums = shift_sums + prev_s0 * nacc;
    e = p.split ? grad2_launch<T, true>(nf, 2, A, C, nullptr, q2, st)
                : grad2_launch<T, false>(nf, 2, A, C, nullptr, q2, st);
    if (e) return e;
    // Fused backward rows + accumulation when every shift of the batch has the same top bit j and,
    // for j >= nl, the same bits above nl (so each row owns fixed gradient entries).
    const uint64_t a_first = (uint64_t)s0, a_last = (uint64_t)(s0 + nb - 1);
    const int j0 = a_first ? 63 - __builtin_clzll(a_first) : -1;
    const int j1 = 63 - __builtin_clzll(a_last | 1);
    const bool fuse = a_first != 0 && j0 == j1 && (j0 < p.nl || (a_first >> p.nl) == (a_last >> p.nl));
    if (fuse && p.row_rb != GRAD_ROW_RB) return fail(E_UNSUPPORTED, "fused gradient kernel: row tile %d", p.row_rb);
    if (fuse) {
      FusedArgs F{};
      F.psi = psi;
      F.exch = exch;
      F.nf = nf;
      F.nh = p.nh;
      F.n_slots = nb;
      F.a0 = a_first;
      F.q = q;
      F.j = j0;
      F.ah = (uint32_t)(a_first >> p.nl);
      F.gpart = gpart;
      // shift groups: at least one round of the shifts a workgroup holds at a time
      const int64_t gf = nb >> (ilog2c(fused_nt(p.nl, sizeof(T))) + fused_rb(p.nl) - p.nl);
      const int gdiv = fused_nt(p.nl, sizeof(T)) / 128;
      const int gcap = groups / gdiv > 0 ? groups / gdiv : 1;
      F.groups = (int)(gf < 1 ? 1 : gf < gcap ? gf : gcap);
      e = p.split ? grad2_launch<T, true>(nf, 4, A, C, &F, q2, st) : grad2_launch<T, false>(nf, 4, A, C, &F, q2, st);
      if (e) return e;
      prev_s0 = s0;
      prev_nb = nb;
      continue;
    }
    e = p.split ? grad2_launch<T, true>(nf, 3, A, C, nullptr, q2, st)
                : grad2_launch<T, false>(nf, 3, A, C, nullptr, q2, st);
    if (e) return e;
    AccumArgs G{};
    G.psi = psi;
    G.z = exch;
    G.nf = nf;
    G.n_slots = nb;
    G.a0 = (uint64_t)s0;
    G.q = q;
    G.gpart = gpart;
    G.groups = groups;
    G.y_tiles = n_shifts / 1024;
    {
      ProfScope prof("sre_grad_accum", st);
      hipLaunchKernelGGL((k_grad_accum<T, 4>), dim3((unsigned)(G.y_tiles * groups)), dim3(256), 0, st, G);
    }
    prev_s0 = s0;
    prev_nb = nb;
  }
  {
    hipLaunchKernelGGL(k_sre_shift_reduce, dim3(shift_reduce_grid(prev_nb)), dim3(SHIFT_REDUCE_NT), 0, st,
                       partials[(k + 1) & 1], prev_nb, n_cb, nacc, (uint64_t)prev_s0, nullptr, nf, qa,
                       shift_sums + prev_s0 * nacc);
  }
  int e = grad_totals_launch(shift_sums, n_shifts, N, q, out, scale, st);
  if (e) return e;
  hipLaunchKernelGGL(k_grad2_final<T>, dim3((unsigned)((n_shifts + 63) / 64)), dim3(1024), 0, st,
                     (const double2 *)gpart, groups, n_shifts, (const double *)scale, (vec2<T> *)grad);
  return hipPeekAtLastError() == hipSuccess ? OK
                                            : fail(E_HIP, "two-pass gradient launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace
}  // namespace hm
