// hm_grad.hip -- fused forward + adjoint of the stabilizer Renyi entropy, dM_q/dpsi (q != 1).
//
// Differentiating chi_b(a) = sum_x conj(psi_{x^a}) psi_x (-1)^{b.x} (Eq. Z_FT_qubits) and using that
// chi_b(a) is real for even a.b and imaginary for odd a.b gives
//     dS_q/dpsi*_y = 2q sum_a psi_{y^a} [H^{(x)N} w(a)]_y,   w_b(a) = |chi_b(a)|^{2q-2} chi_b(a),
// and g = dM/dRe psi + i dM/dIm psi = 2 dS_q/dpsi* / ((1-q) S_q ln 2) (Eq. sre).
//
// Folded form (the forward kernels' notation: U = H^{(x)(N-1)} u for shift a, fold bit j):
// for a != 0, w_b is 2 R_c or 2i I_c with R_c = |2 Re U_c|^{2q-2} Re U_c, I_c = |2 Im U_c|^{2q-2} Im U_c,
// and with Z = H^{(x)(N-1)} (R + i I) the update is, for every folded index c with x = x(c):
//     G_x += 4q psi_{x^a} Z_c,     G_{x^a} += 4q psi_x conj(Z_c).
// For a = 0 (R_c = |Re U_c|^{2q-2} Re U_c, I_c = |Im U_c|^{2q-2} Im U_c):
//     G_c += 2q psi_c (Re Z_c + Im Z_c),   G_{c + 2^{N-1}} += 2q psi_{c + 2^{N-1}} (Re Z_c - Im Z_c).
// The transform is self-adjoint, so the backward runs the forward rounds in reverse order and ends in
// the layout of the product step: the same thread updates the same index pairs it gathered.
//
// Workgroup-resident kernel: one shift per tile, the whole gradient accumulator G (2^N values) in LDS,
// written once per workgroup as a partial; a fixed-order reduction over workgroups follows.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_sre_dev.h"
#include "hm_tile.h"

namespace hm {

// One launch covers gridDim.y states of one size; blockIdx.y selects the state, blockIdx.x a
// strided share of its shifts.
struct GradArgs {
  const void *psis[HM_BATCH_PTRS];
  int nf;              // N - 1
  int64_t n_shifts;    // 2^N
  double q;
  void *gpart;         // [gridDim.y][gridDim.x][2^N] vec2<T>
  double *spart;       // [gridDim.y][gridDim.x][2]: sum |chi|^2, sum |chi|^{2q}
};

struct GradOuts {
  void *g[HM_BATCH_PTRS];
};


// G index pair of register r (a != 0): x = x(c), y = x ^ a, c = tlo + (r << S0), resident path.
template <int RB, int NL>
__device__ __forceinline__ void pair_index(uint64_t a, int j, uint32_t tlo, int r, uint32_t &x, uint32_t &y) {
  constexpr int S0 = NL - RB;
  const uint32_t c = tlo + ((uint32_t)r << S0);
  if (j >= NL) x = c;  // fold on the top qubit: x has bit NL clear, x ^ a sets it
  else x = ins0_32(c, j);
  y = x ^ (uint32_t)a;
}

template <typename T, int RB, int NL, bool Q2>
__global__ __launch_bounds__((1 << (NL - RB)) < 64 ? 64 : (1 << (NL - RB))) void k_sre_grad_resident(GradArgs A) {
  constexpr int R = 1 << RB;
  constexpr int NT = 1 << (NL - RB);  // threads holding the tile (one shift)
  constexpr int S0 = NL - RB;
  constexpr int K = RB == 0 ? 0 : (NL + RB - 1) / RB;
  static_assert(K <= 4, "at most four rounds");
  constexpr int LDS_N = (K > 1) ? ((1 << NL) + (1 << (NL - RB))) : 1;
  constexpr int GN = 2 << NL;  // 2^N

  __shared__ vec2<T> lds[LDS_N];
  __shared__ vec2<T> gacc[GN];
  __shared__ double red[2 * (NT / 64 + 2)];

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psis[blockIdx.y];
  const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
  const uint32_t tau = threadIdx.x;
  const bool tact = tau < (uint32_t)NT;
  const uint32_t tlo = tau & (NT - 1);
  const uint32_t half = 1u << A.nf;
  const T q2 = (T)(2.0 * A.q), q4 = (T)(4.0 * A.q);

  for (uint32_t i = tau; i < (uint32_t)GN; i += blockDim.x) gacc[i] = vec2<T>{T(0), T(0)};
  __syncthreads();
  double s1 = 0.0, sq = 0.0;

  for (int64_t sh = blockIdx.x; sh < A.n_shifts; sh += gridDim.x) {
    const uint64_t a = (uint64_t)sh;
    T re[R], im[R];
    sre_product<T, RB, NL>(psi, half, a, 0, tlo, tact, re, im);
    // forward rounds
    if constexpr (K >= 1) wht_regs<T, R, 0, rp_H(NL, RB, 0)>(re, im);
    if constexpr (K >= 2) {
      relayout<T, R, RB, rp_S(NL, RB, 0), rp_S(NL, RB, 1)>(re, im, lds, tau, tact);
      wht_regs<T, R, 0, rp_H(NL, RB, 1)>(re, im);
    }
    if constexpr (K >= 3) {
      relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 2)>(re, im, lds, tau, tact);
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(re, im);
    }
    if constexpr (K >= 4) {
      relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 3)>(re, im, lds, tau, tact);
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(re, im);
    }
    // sums and the adjoint seed w
    const T kf = (a == 0) ? T(1) : T(2);
    T l1 = T(0), lq = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T tr = re[r] * re[r], ti = im[r] * im[r];
      l1 += tr + ti;
      if (Q2) lq = fmaT(tr, tr, fmaT(ti, ti, lq));
      else lq += (tr > T(0) ? (T)pow(tr, (T)A.q) : T(0)) + (ti > T(0) ? (T)pow(ti, (T)A.q) : T(0));
      re[r] = wfold<T, Q2>(re[r], kf, A.q);
      im[r] = wfold<T, Q2>(im[r], kf, A.q);
    }
    if (tact) {
      const double f = (a == 0) ? 1.0 : 4.0;
      s1 += f * (double)l1;
      sq += pow(f, A.q) * (double)lq;
    }
    // backward rounds (the transform is its own adjoint): reverse order, ending in layout S0
    if constexpr (K >= 4) {
      wht_regs<T, R, 0, rp_H(NL, RB, 3)>(re, im);
      relayout<T, R, RB, rp_S(NL, RB, 3), rp_S(NL, RB, 2)>(re, im, lds, tau, tact);
    }
    if constexpr (K >= 3) {
      wht_regs<T, R, 0, rp_H(NL, RB, 2)>(re, im);
      relayout<T, R, RB, rp_S(NL, RB, 2), rp_S(NL, RB, 1)>(re, im, lds, tau, tact);
    }
    if constexpr (K >= 2) {
      wht_regs<T, R, 0, rp_H(NL, RB, 1)>(re, im);
      relayout<T, R, RB, rp_S(NL, RB, 1), rp_S(NL, RB, 0)>(re, im, lds, tau, tact);
    }
    if constexpr (K >= 1) wht_regs<T, R, 0, rp_H(NL, RB, 0)>(re, im);
    // scatter-accumulate into G (distinct addresses within one shift)
    if (tact) {
      if (a == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t c = tlo + ((uint32_t)r << S0);
          const vec2<T> p0 = ld32(psi, c), p1 = ld32(psi, c + half);
          const T u = re[r] + im[r], v = re[r] - im[r];
          vec2<T> g0 = gacc[c], g1 = gacc[c + half];
          g0.x = fmaT(q2 * u, p0.x, g0.x);
          g0.y = fmaT(q2 * u, p0.y, g0.y);
          g1.x = fmaT(q2 * v, p1.x, g1.x);
          g1.y = fmaT(q2 * v, p1.y, g1.y);
          gacc[c] = g0;
          gacc[c + half] = g1;
        }
      } else {
        const int j = 63 - __builtin_clzll(a);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          uint32_t x, y;
          pair_index<RB, NL>(a, j, tlo, r, x, y);
          const vec2<T> px = ld32(psi, x), py = ld32(psi, y);
          const T zr = q4 * re[r], zi = q4 * im[r];
          vec2<T> gx = gacc[x], gy = gacc[y];
          // G_x += 4q psi_y Z;  G_y += 4q psi_x conj(Z)
          gx.x += fmaT(py.x, zr, -(py.y * zi));
          gx.y += fmaT(py.x, zi, py.y * zr);
          gy.x += fmaT(px.x, zr, px.y * zi);
          gy.y += fmaT(px.y, zr, -(px.x * zi));
          gacc[x] = gx;
          gacc[y] = gy;
        }
      }
    }
    __syncthreads();
  }
  vec2<T> *gp = (vec2<T> *)A.gpart + blk * GN;
  for (uint32_t i = tau; i < (uint32_t)GN; i += blockDim.x) gp[i] = gacc[i];
  // block sums of s1, sq (fixed order)
  constexpr int BT = NT < 64 ? 64 : NT;
  const double t1 = seg_sum<BT, BT>(s1, red, tau);
  const double tq = seg_sum<BT, BT>(sq, red + (BT / 64 + 1), tau);
  if (tau == 0) {
    A.spart[2 * blk] = t1;
    A.spart[2 * blk + 1] = tq;
  }
}

// totals over blocks -> out = {M_q, lost_norm}; scale = 2 / ((1 - q) S_q ln 2) for the gradient.
// Workgroup s handles state s: spart[s][nblk][2] -> out[2 s .. 2 s + 1], scale[s].  Fixed order:
// thread t sums entries t, t + TOT_T, ... in turn, then a tree over the threads.
static constexpr int TOT_T = 1024;
__global__ __launch_bounds__(TOT_T) void k_grad_totals(const double *spart, int nblk, int N, double q, double *out,
                                                      double *scale) {
  __shared__ double r1[TOT_T], rq[TOT_T];
  const uint32_t t = threadIdx.x;
  const double2 *sp = (const double2 *)spart + (size_t)blockIdx.x * nblk;
  out += 2 * blockIdx.x;
  scale += blockIdx.x;
  double a = 0.0, b = 0.0;
#pragma unroll 4
  for (int i = t; i < nblk; i += TOT_T) {
    const double2 v = sp[i];
    a += v.x;
    b += v.y;
  }
  r1[t] = a;
  rq[t] = b;
  __syncthreads();
  for (uint32_t w = TOT_T / 2; w > 0; w >>= 1) {
    if (t < w) {
      r1[t] += r1[t + w];
      rq[t] += rq[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double D = ldexp(1.0, N);
    out[0] = log2(rq[0] / D) / (1.0 - q);
    out[1] = 1.0 - r1[0] / D;
    scale[0] = 2.0 / ((1.0 - q) * rq[0] * log(2.0));
  }
}

// grad_s[y] = scale[s] * sum over blocks of G partials (fixed order); blockIdx.y = state s.
// A workgroup takes 64 consecutive y (one per lane, coalesced) x 16 groups of partials (one per
// wave): wave k sums partials k, k + 16, ... in turn, then wave 0 adds the 16 group sums in order.
static constexpr int RED_Y = 64, RED_G = 16;
template <typename T>
__global__ __launch_bounds__(RED_Y *RED_G) void k_grad_reduce(const vec2<T> *gpart, int nblk, int64_t n,
                                                              const double *scale, GradOuts outs) {
  __shared__ double sr[RED_G][RED_Y], si[RED_G][RED_Y];
  const uint32_t ly = threadIdx.x % RED_Y, g = threadIdx.x / RED_Y;
  const int64_t y = (int64_t)blockIdx.x * RED_Y + ly;
  gpart += (size_t)blockIdx.y * nblk * n;
  double gr = 0.0, gi = 0.0;
  if (y < n) {
    for (int b = (int)g; b < nblk; b += RED_G) {
      const vec2<T> v = gpart[(size_t)b * n + y];
      gr += (double)v.x;
      gi += (double)v.y;
    }
  }
  sr[g][ly] = gr;
  si[g][ly] = gi;
  __syncthreads();
  if (g == 0 && y < n) {
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int k = 0; k < RED_G; ++k) {
      tr += sr[k][ly];
      ti += si[k][ly];
    }
    const double sc = scale[blockIdx.y];
    vec2<T> o;
    o.x = (T)(sc * tr);
    o.y = (T)(sc * ti);
    ((vec2<T> *)outs.g[blockIdx.y])[y] = o;
  }
}

// ------------------------------------------------------------------------------------------------
static constexpr int GRAD_MAX_BLOCKS = 256;

static int grad_max_n(int dbl) { return dbl ? 12 : 13; }

// Workgroups per state: 256 for one to four states, then fewer so that a launch holds about 1024
// workgroups (each sums its own G partial, so fewer per state keeps the final reduction short).
static int grad_blocks(int N, int states) {
  int nb = GRAD_MAX_BLOCKS;
  while (nb > 4 && (int64_t)nb * states > 1024) nb >>= 1;
  const int64_t s = (int64_t)1 << N;
  return (int)(s < nb ? s : nb);
}

static int grad_chunk(int batch) { return batch < HM_BATCH_PTRS ? batch : HM_BATCH_PTRS; }

static size_t grad1_workspace(int N, int dbl, int states) {
  const size_t nb = (size_t)grad_blocks(N, states) * states;
  return align256(nb * ((size_t)1 << N) * (dbl ? 16 : 8)) + align256(nb * 2 * sizeof(double)) +
         align256((size_t)states * sizeof(double));
}

// Two-pass plan of the gradient: default split and tiles, sequential launches.
static int grad2_plan(const PlanOpts &o, int N, int dbl, SrePlan *p) {
  PlanOpts g{};
  g.force_path = 2;
  g.pipeline = 1;
  g.batch = o.batch;
  g.row_rb = 4;  // 2^4-value row tiles on the row side (forward, backward, fused accumulation)
  int e = sre_plan(N, dbl, g, p);
  if (e) return e;
  if (p->nf < 11 || p->nf > 19) return fail(E_UNSUPPORTED, "gradient: two-pass kernels cover n in [12, 20] (n = %d)", N);
  if (o.batch) return OK;
  if (p->nl <= 7) {
    // Rows of at most 2^7 (n <= 15): a batch of 2^nl shifts is a small launch, so take 256 MiB
    // (FP32) / 128 MiB (FP64) exchange batches through the separate backward-row and accumulation
    // kernels (n = 14: 1.5 against 3.4 ms; at n = 16 the fused 2^8-shift batches are 3 % faster).
    const int64_t want = ((int64_t)(dbl ? 128 : 256) << 20) / (((int64_t)1 << p->nf) * (dbl ? 16 : 8));
    const int64_t all = (int64_t)1 << N;
    g.batch = want < all ? want : all;
  } else {
    // Batches of at most 2^nl aligned shifts: every batch after the first then shares its top bit
    // and its bits above nl, which the fused backward-row + accumulation kernel needs.
    if (p->batch <= (1 << p->nl)) return OK;
    g.batch = (int64_t)1 << p->nl;
  }
  return sre_plan(N, dbl, g, p);
}

static bool grad_two_pass(const PlanOpts &o, int N, int dbl) { return N > grad_max_n(dbl) || (o.force_path == 2 && N >= 12); }

// Two-pass gradients of several states run on two streams (lanes) from n = 15 on.
static int grad_lanes(int N, int batch) { return (batch >= 2 && N >= 15) ? 2 : 1; }

int sre_grad_batched_workspace(const PlanOpts &o, int N, int dbl, int batch, size_t *bytes) {
  if (batch < 1) return fail(E_ARG, "gradient: batch = %d < 1", batch);
  if (!grad_two_pass(o, N, dbl)) {
    // full chunks of HM_BATCH_PTRS states and a shorter last one, which may take more workgroups
    const size_t full = grad1_workspace(N, dbl, grad_chunk(batch));
    const int rest = batch % HM_BATCH_PTRS;
    const size_t last = rest ? grad1_workspace(N, dbl, rest) : 0;
    *bytes = full > last ? full : last;
    return OK;
  }
  SrePlan p;
  int e = grad2_plan(o, N, dbl, &p);
  if (e) return e;
  const size_t one = dbl ? sre_grad2_workspace_f64(p) : sre_grad2_workspace_f32(p);
  *bytes = grad_lanes(N, batch) == 2 ? 2 * align256(one) : one;  // two lanes of states (sre_grad_batched_launch)
  return OK;
}

int sre_grad_workspace(const PlanOpts &o, int N, int dbl, size_t *bytes) {
  return sre_grad_batched_workspace(o, N, dbl, 1, bytes);
}

int grad_totals_launch(const double *shift_sums, int64_t n_shifts, int N, double q, double *out, double *scale,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_grad_totals, dim3(1), dim3(TOT_T), 0, st, shift_sums, (int)n_shifts, N, q, out, scale);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "gradient totals: %s", hipGetErrorString(hipGetLastError()));
}

template <typename T, int RB, int NL>
static void launch_grad_nl(const GradArgs &A, int nblk, int states, hipStream_t st) {
  constexpr int NT = (1 << (NL - RB)) < 64 ? 64 : (1 << (NL - RB));
  ProfScope prof("sre_grad_resident", st);
  const dim3 grid(nblk, states);
  if (A.q == 2.0) hipLaunchKernelGGL((k_sre_grad_resident<T, RB, NL, true>), grid, dim3(NT), 0, st, A);
  else hipLaunchKernelGGL((k_sre_grad_resident<T, RB, NL, false>), grid, dim3(NT), 0, st, A);
}

// Up to HM_BATCH_PTRS states of size N: psis[s] -> out[2 s .. 2 s + 1], grads[s].
template <typename T>
static int grad_t(int N, const void *const *psis, int states, double q, double *out, void *const *grads, void *ws,
                  hipStream_t st) {
  const int nblk = grad_blocks(N, states);
  const size_t nb = (size_t)nblk * states;
  char *w = (char *)ws;
  GradArgs A{};
  GradOuts G{};
  for (int s = 0; s < states; ++s) {
    A.psis[s] = psis[s];
    G.g[s] = grads[s];
  }
  A.nf = N - 1;
  A.n_shifts = (int64_t)1 << N;
  A.q = q;
  A.gpart = w;
  A.spart = (double *)(w + align256(nb * ((size_t)1 << N) * sizeof(vec2<T>)));
  double *scale = A.spart + align256(nb * 2 * sizeof(double)) / sizeof(double);
  const int NL = N - 1;
  constexpr int RBmax = sizeof(T) == 4 ? 4 : 3;  // R = 16 (FP32) or 8 (FP64) values per thread: no spills
#define HM_G(nl, rb) \
  case nl:           \
    launch_grad_nl<T, rb, nl>(A, nblk, states, st); \
    break;
  switch (NL) {
    HM_G(0, 0) HM_G(1, 1) HM_G(2, 2) HM_G(3, 3) HM_G(4, RBmax) HM_G(5, RBmax) HM_G(6, RBmax) HM_G(7, RBmax)
    HM_G(8, RBmax) HM_G(9, RBmax) HM_G(10, 3) HM_G(11, 3)
    case 12:
      if constexpr (sizeof(T) == 4) {
        launch_grad_nl<T, 3, 12>(A, nblk, states, st);
        break;
      }
      [[fallthrough]];
    default:
      return fail(E_SIZE, "gradient: n = %d above the workgroup-resident limit %d", N, grad_max_n(sizeof(T) == 8));
  }
#undef HM_G
  hipLaunchKernelGGL(k_grad_totals, dim3(states), dim3(TOT_T), 0, st, A.spart, nblk, N, q, out, scale);
  const int64_t n = (int64_t)1 << N;
  hipLaunchKernelGGL(k_grad_reduce<T>, dim3((unsigned)((n + RED_Y - 1) / RED_Y), states), dim3(RED_Y * RED_G), 0, st,
                     (const vec2<T> *)A.gpart, nblk, n, (const double *)scale, G);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "gradient launch: %s", hipGetErrorString(hipGetLastError()));
}

int sre_grad_batched_launch(const PlanOpts &o, int N, int dbl, const void *const *psis, int batch, double q,
                            double *out, void *const *grads, void *ws, size_t ws_bytes, hipStream_t st) {
  size_t need = 0;
  int e = sre_grad_batched_workspace(o, N, dbl, batch, &need);
  if (e) return e;
  if (ws_bytes < need) return fail(E_WORKSPACE, "gradient workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (grad_two_pass(o, N, dbl)) {
    // States alternate between the caller's stream and an internal one, each lane with its own half
    // of the workspace (stream order separates the states of a lane), so that one state's serial
    // parts (the first batch, the final reductions) overlap the other state's transforms.
    SrePlan p;
    if ((e = grad2_plan(o, N, dbl, &p))) return e;
    const size_t one = align256(dbl ? sre_grad2_workspace_f64(p) : sre_grad2_workspace_f32(p));
    // (measured on 64 circuit states: n = 16 969 ms against 1276 ms for one lane; n = 14 91 against
    // 85 ms, so one lane below n = 15)
    const int L = grad_lanes(N, batch);
    hipStream_t lst[2] = {st, st};
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    if (L == 2) {
      if ((e = side_stream(&lst[1]))) return e;
      if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess) {
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        return fail(E_HIP, "gradient: event creation failed");
      }
      if (hipEventRecord(ev_fork, st) != hipSuccess || hipStreamWaitEvent(lst[1], ev_fork, 0) != hipSuccess) {
        (void)hipEventDestroy(ev_fork);
        (void)hipEventDestroy(ev_join);
        return fail(E_HIP, "gradient: stream fork failed");
      }
    }
    for (int s = 0; s < batch && !e; ++s) {
      const int l = s % L;
      void *w = (char *)ws + (size_t)l * one;
      e = dbl ? sre_grad2_f64(p, psis[s], q, out + 2 * s, grads[s], w, lst[l])
              : sre_grad2_f32(p, psis[s], q, out + 2 * s, grads[s], w, lst[l]);
    }
    if (L == 2) {
      const bool ok = hipEventRecord(ev_join, lst[1]) == hipSuccess && hipStreamWaitEvent(st, ev_join, 0) == hipSuccess;
      (void)hipEventDestroy(ev_fork);
      (void)hipEventDestroy(ev_join);
      if (!ok && !e) e = fail(E_HIP, "gradient: stream join failed");
    }
    return e;
  }
  // resident: chunks of up to HM_BATCH_PTRS states, one launch each, sharing the workspace in order
  for (int s0 = 0; s0 < batch; s0 += HM_BATCH_PTRS) {
    const int cnt = grad_chunk(batch - s0);
    e = dbl ? grad_t<double>(N, psis + s0, cnt, q, out + 2 * s0, grads + s0, ws, st)
            : grad_t<float>(N, psis + s0, cnt, q, out + 2 * s0, grads + s0, ws, st);
    if (e) return e;
  }
  return OK;
}

int sre_grad_launch(const PlanOpts &o, int N, int dbl, const void *psi, double q, double *out, void *grad, void *ws,
                    size_t ws_bytes, hipStream_t st) {
  return sre_grad_batched_launch(o, N, dbl, &psi, 1, q, out, &grad, ws, ws_bytes, st);
}

}  // namespace hm
