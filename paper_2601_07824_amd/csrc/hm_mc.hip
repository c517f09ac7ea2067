// hm_mc.hip -- Monte Carlo estimate of M_2 by thermodynamic integration (the sampling algorithm for
// the SRE of "Computing quantum magic of state vectors", Sec. "Monte Carlo sampling algorithm for
// SRE", Eqs. feP, Boltz, f_expect_beta_reg, Ie, Var_I_eps, m2error and its Algorithm).
//
// L x R Metropolis chains over X-strings a (R independent chains at each of the L inverse
// temperatures beta_l = l / (L - 1)) advance in lock step.  One step of all chains is
//   1. the row sums S(a') = sum_b chi_b(a')^4 of every chain's proposal a' = a XOR m: one launch of
//      the SRE row kernels over the C = L R proposals (one Walsh-Hadamard transform per row);
//   2. k_mc_accept: f(a') = -ln(S'(a') + eps), acceptance with probability min(1, exp(-beta df)),
//      the chain's current energy appended to its trace, and the next proposal formed.
// The chains' randomness (initial strings, XOR masks, acceptance uniforms) is an input, so a chain
// is a deterministic function of it.  After the last step one workgroup per chain computes the mean,
// variance and integrated autocorrelation time of its trace past the thermalisation steps, and a
// final kernel forms <f>_beta per grid point, the Simpson integral I = ln Z_0 - ln Z_1 and
// M_2 = -log2(e^-I - eps + 2^-N [identity re-added]) with its error bar.
//
// S'(a) = S(a) for a != 0; with the identity string left out, S'(0) = sum_{b != 0} <Z_b>^4, computed
// once per call in FP64 from the Walsh-Hadamard transform of |psi_x|^2 (the a = 0 row, whose b = 0
// term <I> = |psi|^2 would swamp the rest in FP32).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/hmag.h"
#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

static constexpr double MC_WINDOW_C = 5.0;  // autocorrelation window: smallest W with W >= 5 tau(W)

// ---- S'(0) in FP64 ------------------------------------------------------------------------------
template <typename T>
__global__ void k_mc_prob(const vec2<T> *psi, uint64_t D, double *p) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= D) return;
  const vec2<T> v = psi[x];
  p[x] = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

__global__ void k_mc_wht_stage(double *v, uint64_t D, uint64_t h) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D / 2) return;
  const uint64_t lo = ((i / h) * 2 * h) + (i % h), hi = lo + h;
  const double u = v[lo], w = v[hi];
  v[lo] = u + w;
  v[hi] = u - w;
}

// Fixed-order sum of chi_b^4 over b in [1, D): per-block partials, then one block.
static constexpr int MC_RED_BLOCKS = 1024;
__global__ __launch_bounds__(256) void k_mc_sum4(const double *chi, uint64_t D, double *part) {
  __shared__ double red[256];
  double s = 0.0;
  for (uint64_t b = 1 + (uint64_t)blockIdx.x * 256 + threadIdx.x; b < D; b += (uint64_t)gridDim.x * 256) {
    const double c2 = chi[b] * chi[b];
    s = fma(c2, c2, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_mc_sum_parts(const double *part, int n, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---- chain steps --------------------------------------------------------------------------------
struct McChains {
  int C;             // chains = L * R
  int L, R;
  uint64_t mask;     // 2^N - 1
  double eps;
  int excl;          // identity string left out
  const double *s0;  // S'(0) (when excl)
  uint64_t *cur;     // current X-string per chain
  uint64_t *prop;    // proposal per chain
  double *fcur;      // current energy per chain
  int64_t *acc;      // accepted moves per chain
  const double *rs;  // row sums of the proposals [C][2] = {sum chi^2, sum chi^4}
};

__device__ __forceinline__ double mc_energy(const McChains &M, uint64_t a, double s4) {
  const double s = (M.excl && a == 0) ? *M.s0 : s4;
  const double v = s + M.eps;
  return v > 0.0 ? -log(v) : HUGE_VAL;
}

// Initial strings: the first row evaluation is of a_init (already in prop).
__global__ void k_mc_init(McChains M, const uint64_t *moves) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M.C) return;
  const uint64_t a = M.prop[c];
  M.cur[c] = a;
  M.fcur[c] = mc_energy(M, a, M.rs[2 * c + 1]);
  M.acc[c] = 0;
  M.prop[c] = (a ^ moves[c]) & M.mask;  // proposal of step 0
}

__global__ void k_mc_seed(McChains M, const uint64_t *a_init) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < M.C) M.prop[c] = a_init[c] & M.mask;
}

__global__ void k_mc_accept(McChains M, int64_t step, int64_t n_steps, const uint64_t *moves, const double *uniforms,
                            double *trace) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M.C) return;
  const int l = c / M.R;
  const double beta = (double)l / (double)(M.L - 1);
  const uint64_t ap = M.prop[c];
  const double fnew = mc_energy(M, ap, M.rs[2 * c + 1]);
  double f = M.fcur[c];
  uint64_t a = M.cur[c];
  bool take;
  if (beta == 0.0) {
    take = true;
  } else {
    const double d = fnew - f;
    take = (d <= 0.0) || (uniforms[step * M.C + c] < exp(-beta * d));
  }
  if (take) {
    a = ap;
    f = fnew;
    M.cur[c] = a;
    M.fcur[c] = f;
    M.acc[c] += 1;
  }
  trace[step * M.C + c] = f;
  if (step + 1 < n_steps) M.prop[c] = (a ^ moves[(step + 1) * M.C + c]) & M.mask;
}

// ---- statistics -------------------------------------------------------------------------------
// Fixed-order block sum (256 threads).
__device__ __forceinline__ double block_sum256(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// One workgroup per chain: mean, variance C(0) and integrated autocorrelation time of the trace
// samples [n_therm, n_steps).  stats[c] = {mean, C(0), tau}.
__global__ __launch_bounds__(256) void k_mc_chain_stats(const double *trace, int C, int64_t n_therm, int64_t n_steps,
                                                        double *stats) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int64_t m = n_steps - n_therm;
  const double *x = trace + n_therm * C + c;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += x[i * C];
  const double mean = block_sum256(s, red) / (double)m;
  s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double d = x[i * C] - mean;
    s = fma(d, d, s);
  }
  const double c0 = block_sum256(s, red) / (double)m;
  double tau = 0.5;
  if (c0 > 0.0) {
    for (int64_t t = 1; t <= m / 2; ++t) {
      s = 0.0;
      for (int64_t i = threadIdx.x; i + t < m; i += 256) s = fma(x[i * C] - mean, x[(i + t) * C] - mean, s);
      tau += block_sum256(s, red) / (double)m / c0;
      if ((double)t >= MC_WINDOW_C * tau) break;
    }
  }
  if (threadIdx.x == 0) {
    stats[3 * c + 0] = mean;
    stats[3 * c + 1] = c0;
    stats[3 * c + 2] = tau;
  }
}

// out = {M2_hat, dM2, I_hat, S2_hat} then, per grid point l: {<f>_l, variance of <f>_l, sigma_f^2
// (mean over its chains), tau_int (mean over its chains), acceptance rate}.
__global__ void k_mc_final(const double *stats, const int64_t *acc, int L, int R, int64_t n_therm, int64_t n_steps,
                           double eps, int excl, int N, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double m = (double)(n_steps - n_therm);
  const double h = 1.0 / (double)(L - 1);
  double I = 0.0, varI = 0.0;
  for (int l = 0; l < L; ++l) {
    double mu = 0.0, var = 0.0, s2 = 0.0, tau = 0.0, na = 0.0;
    for (int r = 0; r < R; ++r) {
      const int c = l * R + r;
      mu += stats[3 * c + 0];
      var += 2.0 * stats[3 * c + 2] * stats[3 * c + 1] / m;
      s2 += stats[3 * c + 1];
      tau += stats[3 * c + 2];
      na += (double)acc[c];
    }
    mu /= (double)R;
    var /= (double)R * (double)R;
    // composite Simpson weights h/3 {1, 4, 2, 4, ..., 2, 4, 1}
    const double w = h / 3.0 * ((l == 0 || l == L - 1) ? 1.0 : (l % 2 ? 4.0 : 2.0));
    I += w * mu;
    varI += w * w * var;
    double *o = out + 4 + 5 * l;
    o[0] = mu;
    o[1] = var;
    o[2] = s2 / (double)R;
    o[3] = tau / (double)R;
    o[4] = na / ((double)R * (double)n_steps);
  }
  const double eI = exp(-I);
  const double sD = eI - eps + (excl ? ldexp(1.0, -N) : 0.0);  // S_2 / 2^N
  out[0] = -log2(sD);
  out[1] = eI / sD * sqrt(varI) / log(2.0);
  out[2] = I;
  out[3] = sD * ldexp(1.0, N);
}

// ---- host side --------------------------------------------------------------------------------
struct McLayout {
  size_t s0_vec, s0_part, chains, rs, stats, rows, total;
};

static McLayout mc_layout(const SrePlan &p, int C, int excl) {
  McLayout Lo{};
  size_t o = 0;
  Lo.s0_vec = o;
  o += excl ? align256(((size_t)1 << p.N) * sizeof(double)) : 0;
  Lo.s0_part = o;
  o += align256((MC_RED_BLOCKS + 1) * sizeof(double));
  Lo.chains = o;  // cur, prop (u64), fcur (double), acc (i64)
  o += 4 * align256((size_t)C * 8);
  Lo.rs = o;
  o += align256((size_t)C * 2 * sizeof(double));
  Lo.stats = o;
  o += align256((size_t)C * 3 * sizeof(double));
  Lo.rows = o;
  o += sre_workspace(p, 1, 0);
  Lo.total = o;
  return Lo;
}

int mc_check(int n, const hm_mc_params *prm) {
  if (!prm) return fail(E_ARG, "mc: params is NULL");
  if (prm->n_beta < 3 || prm->n_beta % 2 == 0 || prm->n_beta > 1025)
    return fail(E_ARG, "mc: n_beta = %d must be odd and in [3, 1025] (composite Simpson rule)", prm->n_beta);
  if (prm->chains_per_beta < 1 || (int64_t)prm->chains_per_beta * prm->n_beta > (1 << 20))
    return fail(E_ARG, "mc: chains_per_beta = %d outside [1, 2^20 / n_beta]", prm->chains_per_beta);
  if (prm->n_steps < 2 || prm->n_therm < 0 || prm->n_therm > prm->n_steps - 2)
    return fail(E_ARG, "mc: need n_steps >= 2 and 0 <= n_therm <= n_steps - 2 (got %lld, %lld)",
                (long long)prm->n_steps, (long long)prm->n_therm);
  if ((double)prm->n_steps * prm->n_beta * prm->chains_per_beta > 1e10)
    return fail(E_ARG, "mc: n_steps x chains above 1e10");
  if (!(prm->epsilon >= 0.0) || !isfinite(prm->epsilon)) return fail(E_ARG, "mc: epsilon = %g must be >= 0", prm->epsilon);
  if (prm->exclude_identity != 0 && prm->exclude_identity != 1)
    return fail(E_ARG, "mc: exclude_identity = %d not 0 or 1", prm->exclude_identity);
  (void)n;
  return OK;
}

int mc_workspace(const SrePlan &p, const hm_mc_params *prm, size_t *bytes) {
  *bytes = mc_layout(p, prm->n_beta * prm->chains_per_beta, prm->exclude_identity).total;
  return OK;
}

int mc_run(const SrePlan &p, const void *psi, const hm_mc_params *prm, const uint64_t *a_init, const uint64_t *moves,
           const double *uniforms, double *out, double *trace, void *ws, hipStream_t st) {
  const int C = prm->n_beta * prm->chains_per_beta;
  const McLayout Lo = mc_layout(p, C, prm->exclude_identity);
  char *w = (char *)ws;
  McChains M{};
  M.C = C;
  M.L = prm->n_beta;
  M.R = prm->chains_per_beta;
  M.mask = (p.N >= 64) ? ~0ull : ((1ull << p.N) - 1ull);
  M.eps = prm->epsilon;
  M.excl = prm->exclude_identity;
  M.cur = (uint64_t *)(w + Lo.chains);
  M.prop = (uint64_t *)(w + Lo.chains + align256((size_t)C * 8));
  M.fcur = (double *)(w + Lo.chains + 2 * align256((size_t)C * 8));
  M.acc = (int64_t *)(w + Lo.chains + 3 * align256((size_t)C * 8));
  M.rs = (const double *)(w + Lo.rs);
  double *rs = (double *)(w + Lo.rs);
  double *part = (double *)(w + Lo.s0_part);
  M.s0 = part + MC_RED_BLOCKS;
  const unsigned thr = 256;
  if (M.excl) {
    const uint64_t D = 1ull << p.N;
    double *v = (double *)(w + Lo.s0_vec);
    if (p.dbl) hipLaunchKernelGGL(k_mc_prob<double>, dim3((unsigned)((D + thr - 1) / thr)), dim3(thr), 0, st, (const double2 *)psi, D, v);
    else hipLaunchKernelGGL(k_mc_prob<float>, dim3((unsigned)((D + thr - 1) / thr)), dim3(thr), 0, st, (const float2 *)psi, D, v);
    for (uint64_t h = 1; h < D; h <<= 1)
      hipLaunchKernelGGL(k_mc_wht_stage, dim3((unsigned)((D / 2 + thr - 1) / thr)), dim3(thr), 0, st, v, D, h);
    hipLaunchKernelGGL(k_mc_sum4, dim3(MC_RED_BLOCKS), dim3(256), 0, st, (const double *)v, D, part);
    hipLaunchKernelGGL(k_mc_sum_parts, dim3(1), dim3(256), 0, st, (const double *)part, MC_RED_BLOCKS, part + MC_RED_BLOCKS);
  }
  QArgs qa;
  memset(&qa, 0, sizeof(qa));
  qa.nq = 1;
  qa.q[0] = 2.0;
  const unsigned cb = (unsigned)((C + 255) / 256);
  char *rws = w + Lo.rows;
  hipLaunchKernelGGL(k_mc_seed, dim3(cb), dim3(256), 0, st, M, a_init);
  int e = sre_run(p, psi, qa, 0, M.prop, C, rs, nullptr, nullptr, rws, st);
  if (e) return e;
  hipLaunchKernelGGL(k_mc_init, dim3(cb), dim3(256), 0, st, M, moves);
  for (int64_t s = 0; s < prm->n_steps; ++s) {
    if ((e = sre_run(p, psi, qa, 0, M.prop, C, rs, nullptr, nullptr, rws, st))) return e;
    hipLaunchKernelGGL(k_mc_accept, dim3(cb), dim3(256), 0, st, M, s, prm->n_steps, moves, uniforms, trace);
  }
  double *stats = (double *)(w + Lo.stats);
  hipLaunchKernelGGL(k_mc_chain_stats, dim3(C), dim3(256), 0, st, (const double *)trace, C, prm->n_therm, prm->n_steps, stats);
  hipLaunchKernelGGL(k_mc_final, dim3(1), dim3(64), 0, st, (const double *)stats, (const int64_t *)M.acc, M.L, M.R,
                     prm->n_therm, prm->n_steps, M.eps, M.excl, p.N, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "mc launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace hm
