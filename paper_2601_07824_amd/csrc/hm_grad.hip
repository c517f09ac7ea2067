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

struct GradArgs {
  const void *psi;
  int nf;              // N - 1
  int64_t n_shifts;    // 2^N
  double q;
  void *gpart;         // [gridDim][2^N] vec2<T>
  double *spart;       // [gridDim][2]: sum |chi|^2, sum |chi|^{2q}
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

  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
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
  vec2<T> *gp = (vec2<T> *)A.gpart + (size_t)blockIdx.x * GN;
  for (uint32_t i = tau; i < (uint32_t)GN; i += blockDim.x) gp[i] = gacc[i];
  // block sums of s1, sq (fixed order)
  constexpr int BT = NT < 64 ? 64 : NT;
  const double t1 = seg_sum<BT, BT>(s1, red, tau);
  const double tq = seg_sum<BT, BT>(sq, red + (BT / 64 + 1), tau);
  if (tau == 0) {
    A.spart[2 * blockIdx.x] = t1;
    A.spart[2 * blockIdx.x + 1] = tq;
  }
}

// totals over blocks -> out = {M_q, lost_norm}; scale = 2 / ((1 - q) S_q ln 2) for the gradient
__global__ __launch_bounds__(256) void k_grad_totals(const double *spart, int nblk, int N, double q, double *out,
                                                    double *scale) {
  __shared__ double r1[256], rq[256];
  const uint32_t t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < nblk; i += 256) {
    a += spart[2 * i];
    b += spart[2 * i + 1];
  }
  r1[t] = a;
  rq[t] = b;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
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

template <typename T>
__global__ void k_grad_reduce(const vec2<T> *gpart, int nblk, int64_t n, const double *scale, vec2<T> *grad) {
  const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= n) return;
  double gr = 0.0, gi = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const vec2<T> v = gpart[(size_t)b * n + y];
    gr += (double)v.x;
    gi += (double)v.y;
  }
  const double s = scale[0];
  vec2<T> o;
  o.x = (T)(s * gr);
  o.y = (T)(s * gi);
  grad[y] = o;
}

// ------------------------------------------------------------------------------------------------
static constexpr int GRAD_MAX_BLOCKS = 256;

static int grad_max_n(int dbl) { return dbl ? 12 : 13; }

static int grad_blocks(int N) {
  const int64_t s = (int64_t)1 << N;
  return (int)(s < GRAD_MAX_BLOCKS ? s : GRAD_MAX_BLOCKS);
}

static size_t grad1_workspace(int N, int dbl) {
  const size_t nb = (size_t)grad_blocks(N);
  return align256(nb * ((size_t)1 << N) * (dbl ? 16 : 8)) + align256(nb * 2 * sizeof(double)) + 256;
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
  // Batches of at most 2^nl aligned shifts: every batch after the first then shares its top bit and
  // its bits above nl, which the fused backward-row + accumulation kernel needs.
  if (!o.batch && p->batch > (1 << p->nl)) {
    g.batch = (int64_t)1 << p->nl;
    if ((e = sre_plan(N, dbl, g, p))) return e;
  }
  return OK;
}

static bool grad_two_pass(const PlanOpts &o, int N, int dbl) { return N > grad_max_n(dbl) || (o.force_path == 2 && N >= 12); }

int sre_grad_workspace(const PlanOpts &o, int N, int dbl, size_t *bytes) {
  if (!grad_two_pass(o, N, dbl)) {
    *bytes = grad1_workspace(N, dbl);
    return OK;
  }
  SrePlan p;
  int e = grad2_plan(o, N, dbl, &p);
  if (e) return e;
  *bytes = dbl ? sre_grad2_workspace_f64(p) : sre_grad2_workspace_f32(p);
  return OK;
}

int grad_totals_launch(const double *shift_sums, int64_t n_shifts, int N, double q, double *out, double *scale,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_grad_totals, dim3(1), dim3(256), 0, st, shift_sums, (int)n_shifts, N, q, out, scale);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "gradient totals: %s", hipGetErrorString(hipGetLastError()));
}

template <typename T, int RB, int NL>
static void launch_grad_nl(const GradArgs &A, int nblk, hipStream_t st) {
  constexpr int NT = (1 << (NL - RB)) < 64 ? 64 : (1 << (NL - RB));
  ProfScope prof("sre_grad_resident", st);
  if (A.q == 2.0) hipLaunchKernelGGL((k_sre_grad_resident<T, RB, NL, true>), dim3(nblk), dim3(NT), 0, st, A);
  else hipLaunchKernelGGL((k_sre_grad_resident<T, RB, NL, false>), dim3(nblk), dim3(NT), 0, st, A);
}

template <typename T>
static int grad_t(int N, const void *psi, double q, double *out, void *grad, void *ws, hipStream_t st) {
  const int nblk = grad_blocks(N);
  char *w = (char *)ws;
  GradArgs A{};
  A.psi = psi;
  A.nf = N - 1;
  A.n_shifts = (int64_t)1 << N;
  A.q = q;
  A.gpart = w;
  A.spart = (double *)(w + align256((size_t)nblk * ((size_t)1 << N) * sizeof(vec2<T>)));
  double *scale = A.spart + align256((size_t)nblk * 2 * sizeof(double)) / sizeof(double);
  const int NL = N - 1;
  constexpr int RBmax = sizeof(T) == 4 ? 4 : 3;  // R = 16 (FP32) or 8 (FP64) values per thread: no spills
#define HM_G(nl, rb) \
  case nl:           \
    launch_grad_nl<T, rb, nl>(A, nblk, st); \
    break;
  switch (NL) {
    HM_G(0, 0) HM_G(1, 1) HM_G(2, 2) HM_G(3, 3) HM_G(4, RBmax) HM_G(5, RBmax) HM_G(6, RBmax) HM_G(7, RBmax)
    HM_G(8, RBmax) HM_G(9, RBmax) HM_G(10, RBmax) HM_G(11, RBmax)
    case 12:
      if constexpr (sizeof(T) == 4) {
        launch_grad_nl<T, 4, 12>(A, nblk, st);
        break;
      }
      [[fallthrough]];
    default:
      return fail(E_SIZE, "gradient: n = %d above the workgroup-resident limit %d", N, grad_max_n(sizeof(T) == 8));
  }
#undef HM_G
  hipLaunchKernelGGL(k_grad_totals, dim3(1), dim3(256), 0, st, A.spart, nblk, N, q, out, scale);
  const int64_t n = (int64_t)1 << N;
  hipLaunchKernelGGL(k_grad_reduce<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const vec2<T> *)A.gpart,
                     nblk, n, (const double *)scale, (vec2<T> *)grad);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "gradient launch: %s", hipGetErrorString(hipGetLastError()));
}

int sre_grad_launch(const PlanOpts &o, int N, int dbl, const void *psi, double q, double *out, void *grad, void *ws,
                    size_t ws_bytes, hipStream_t st) {
  size_t need = 0;
  int e = sre_grad_workspace(o, N, dbl, &need);
  if (e) return e;
  if (ws_bytes < need) return fail(E_WORKSPACE, "gradient workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (grad_two_pass(o, N, dbl)) {
    SrePlan p;
    if ((e = grad2_plan(o, N, dbl, &p))) return e;
    return dbl ? sre_grad2_f64(p, psi, q, out, grad, ws, st) : sre_grad2_f32(p, psi, q, out, grad, ws, st);
  }
  return dbl ? grad_t<double>(N, psi, q, out, grad, ws, st) : grad_t<float>(N, psi, q, out, grad, ws, st);
}

}  // namespace hm
