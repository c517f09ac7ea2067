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

#include <mutex>
#include <math.h>
#include <stdint.h>

#include "hm_tile.h"

namespace hm {

static inline int nacc_of(const QArgs &qa) { return qa.nq + 1; }

int sre_shift_sums_f32(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                       int64_t n_slots, double *shift_sums, char *w, hipStream_t st);
int sre_shift_sums_f64(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                       int64_t n_slots, double *shift_sums, char *w, hipStream_t st);
int sre_states_f32(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *shift_sums,
                   hipStream_t st);
int sre_states_f64(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *shift_sums,
                   hipStream_t st);

__device__ __forceinline__ void sre_finalize_into(const double *tot, int N, const QArgs &qa, double *out) {
  const double D = ldexp(1.0, N);
  for (int i = 0; i < qa.nq; ++i) {
    const double q = qa.q[i];
    out[i] = (q == 1.0) ? -tot[1 + i] / D : log2(tot[1 + i] / D) / (1.0 - q);
  }
  out[qa.nq] = 1.0 - tot[0] / D;
}

// One block per state: fixed-order sum of the state's 2^N per-shift sums, finalised (Eq. sre).
struct StateOuts {
  double *out[HM_BATCH_PTRS];
};
__global__ __launch_bounds__(256) void k_sre_state_totals(const double *shift_sums, int N, int nacc, QArgs qa,
                                                          StateOuts outs) {
  __shared__ double red[256];
  __shared__ double tot[HM_MAX_Q + 1];
  const uint32_t t = threadIdx.x;
  const int64_t ns = (int64_t)1 << N;
  const double *base = shift_sums + (int64_t)blockIdx.x * ns * nacc;
  for (int k = 0; k < nacc; ++k) {
    double s = 0.0;
    for (int64_t i = t; i < ns; i += 256) s += base[i * nacc + k];
    red[t] = s;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) tot[k] = red[0];
    __syncthreads();
  }
  if (t == 0) sre_finalize_into(tot, N, qa, outs.out[blockIdx.x]);
}

// Monte Carlo M_2 from sampled X-rows, with the a = 0 row (which holds the identity, <I>^4 = 1, a
// single heavy term that uniform sampling would almost always miss) taken exactly:
//   S_hat = (S(0) + (2^N - 1) mean_k S(a_k)) / 2^N,  M2_hat = -log2 S_hat,
// with mean and sample standard deviation over the sampled rows a_k != 0 (rows equal to 0 are
// skipped).  out = {M2_hat, its standard error, S_hat, std_k S(a_k)}.
__global__ __launch_bounds__(256) void k_sre_sampled_stats(const double *row_sums, const uint64_t *rows, int64_t n,
                                                           int nacc, const double *s0_sums, int N, double *out) {
  __shared__ double r1[256], r2[256];
  const uint32_t t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int64_t i = t; i < n; i += 256)
    if (rows[i] != 0) {
      s += row_sums[i * nacc + 1];
      c += 1.0;
    }
  r1[t] = s;
  r2[t] = c;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (t < w) {
      r1[t] += r1[t + w];
      r2[t] += r2[t + w];
    }
    __syncthreads();
  }
  const double cnt = r2[0];
  const double mean = r1[0] / cnt;
  __syncthreads();
  double v = 0.0;
  for (int64_t i = t; i < n; i += 256)
    if (rows[i] != 0) {
      const double d = row_sums[i * nacc + 1] - mean;
      v += d * d;
    }
  r2[t] = v;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (t < w) r2[t] += r2[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double D = ldexp(1.0, N);
    const double sd = cnt > 1.0 ? sqrt(r2[0] / (cnt - 1.0)) : __builtin_nan("");
    const double shat = (s0_sums[1] + (D - 1.0) * mean) / D;
    out[0] = -log2(shat);
    out[1] = (D - 1.0) / D * sd / (sqrt(cnt) * shat * log(2.0));
    out[2] = shat;
    out[3] = sd;
  }
}

// Fixed-order sum of rows [0, n) of nacc doubles by one workgroup: thread t adds the rows
// t, t + TOT_NT, ... (all nacc slots of a row at once), then a tree over the threads per slot.
// tot[k] (shared) receives the sums.
static constexpr int TOT_NT = 1024;
__device__ __forceinline__ void block_rows_sum(const double *rows_, int64_t n, int nacc, double *red, double *tot) {
  const uint32_t t = threadIdx.x;
  double s[HM_MAX_Q + 1];
#pragma unroll
  for (int k = 0; k <= HM_MAX_Q; ++k) s[k] = 0.0;
  for (int64_t i = t; i < n; i += TOT_NT) {
    const double *row = rows_ + i * nacc;
#pragma unroll
    for (int k = 0; k <= HM_MAX_Q; ++k)
      if (k < nacc) s[k] += row[k];
  }
#pragma unroll
  for (int k = 0; k <= HM_MAX_Q; ++k) {
    if (k < nacc) {  // uniform across the workgroup
      red[t] = s[k];
      __syncthreads();
      for (uint32_t w = TOT_NT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
      }
      if (t == 0) tot[k] = red[0];
      __syncthreads();
    }
  }
}

// First level for long shift lists: workgroup g sums the contiguous chunk of rows
// [g chunk, (g + 1) chunk) into part[g] (fixed order within and across workgroups).
__global__ __launch_bounds__(TOT_NT) void k_sre_total_part(const double *shift_sums, int64_t n_slots, int nacc,
                                                           int64_t chunk, double *part) {
  __shared__ double red[TOT_NT];
  __shared__ double tot[HM_MAX_Q + 1];
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t n = r0 >= n_slots ? 0 : (n_slots - r0 < chunk ? n_slots - r0 : chunk);
  block_rows_sum(shift_sums + r0 * nacc, n, nacc, red, tot);
  if (threadIdx.x == 0)
    for (int k = 0; k < nacc; ++k) part[blockIdx.x * nacc + k] = tot[k];
}

// Fixed-order sum over all per-shift sums (or first-level partials); optionally finalise (Eq. sre).
__global__ __launch_bounds__(TOT_NT) void k_sre_total(const double *shift_sums, int64_t n_slots, int nacc, QArgs qa,
                                                      int N, double *sums, double *out) {
  __shared__ double red[TOT_NT];
  __shared__ double tot[HM_MAX_Q + 1];
  block_rows_sum(shift_sums, n_slots, nacc, red, tot);
  if (threadIdx.x == 0) {
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

// ---- internal streams -----------------------------------------------------------------------------
int side_stream(hipStream_t *st) {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(E_HIP, "SRE: no current device");
  std::lock_guard<std::mutex> g(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    return fail(E_HIP, "SRE: internal stream creation failed");
  *st = streams[dev];
  return OK;
}

// ---- planning -------------------------------------------------------------------------------------
// Defaults (tuned on MI355X; see hm_autotune): FP32 register tiles of 2^5 values, FP64 of 2^4; the
// two-pass split puts ceil(nf / 2) index bits in the row pass.  Every choice can be overridden
// through PlanOpts (options of the handle) and is validated against the built kernels here.
// Pipelined launches (row pass of batch k with the column pass of batch k - 1) and split LDS staging
// (two-pass kernels) are used automatically when these are set.
static constexpr bool SRE_PIPE_DEFAULT = false, SRE_SPLIT_DEFAULT = true;
static constexpr int SRE_STREAMS_DEFAULT = 1;

int sre_plan(int N, int dbl, const PlanOpts &o, SrePlan *p) {
  if (N < 1 || N > 26) return fail(E_SIZE, "SRE: n = %d outside [1, 26]", N);
  SrePlan P{};
  P.N = N;
  P.nf = N - 1;
  P.dbl = dbl;
  const int RB = dbl ? 4 : 5;
  const int onepass_max = dbl ? 14 : 15;  // folded bits one workgroup tile can hold (VGPR-resident)
  const int twopass_min = 6 + RB;         // smallest column tile is 64 threads x 2^RB values
  int path = o.force_path;
  if (path == 0) path = (P.nf <= onepass_max) ? 1 : 2;
  if (path != 1 && path != 2) return fail(E_ARG, "SRE: path %d unknown", path);
  if (path == 1 && P.nf > onepass_max)
    return fail(E_UNSUPPORTED, "SRE: workgroup-resident path holds at most 2^%d folded values (n = %d)", onepass_max, N);
  if (path == 2 && P.nf < twopass_min)
    return fail(E_UNSUPPORTED, "SRE: two-pass path needs n >= %d", twopass_min + 1);
  P.path = path;
  // Resident tiles of 2^10..2^14 (FP32) / 2^13 (FP64) values: split LDS staging with a higher
  // occupancy register budget unless HM_OPT_LDS_SPLIT = 1 (measured 1.2-1.3x faster at n = 13, 14
  // on MI355X).
  if (path == 1)
    P.split = (o.lds_split == 2 || (o.lds_split == 0 && SRE_SPLIT_DEFAULT)) && P.nf >= 10 && P.nf <= (dbl ? 13 : 14);
  if (path == 2) {
    const int row_rb = o.row_rb ? o.row_rb : RB;
    const int col_rb = o.col_rb ? o.col_rb : RB;
    if (dbl ? (row_rb != 4 || col_rb != 4) : ((row_rb != 4 && row_rb != 5) || (col_rb != 4 && col_rb != 5)))
      return fail(E_UNSUPPORTED, "SRE: register tiles (%d, %d) not built for this dtype", row_rb, col_rb);
    const int col_tb = sre_default_col_tb(P.nf, dbl, col_rb);
    // rows of up to 2^13 values; FP32 row tiles of 2^14 (2^4 or 2^5 values per thread) and 2^15
    // (2^5 per thread) as well
    const int nl_max = dbl ? 13 : (row_rb == 5 ? 15 : 14), nl_min = 6;
    int nl = o.row_bits ? o.row_bits : sre_default_nl(P.nf, col_tb, col_rb);
    // From 2^21 folded values on, the default split leaves column tiles 2^1..2^3 columns wide, so a
    // column read uses 16-64 contiguous bytes per row; longer rows widen them at the cost of a
    // slower row pass.  Measured on MI355X (256 shifts): n = 22 best with 12-13 row bits, n = 24
    // with 13 (13.9 ms against 14.7 for 12 and 15.9 for 15); the rows grow by one bit per qubit
    // beyond that (2^15 at n = 26).  Pipelined kernels are built for the default split only.
    if (!o.row_bits && !dbl && row_rb == 5 && P.nf >= 21 && o.pipeline != 2 && o.lds_split != 1) {
      const int want = P.nf - 10 > 13 ? P.nf - 10 : 13;
      nl = want < nl_max ? want : nl_max;
    }
    int nh = P.nf - nl;
    if (nh < col_rb || nh > col_tb || nl < col_tb - nh || nl > nl_max || nl < nl_min)
      return fail(E_UNSUPPORTED, "SRE: no two-pass split for n = %d (row bits %d, column tile 2^%d)", N, nl, col_tb);
    P.nl = nl;
    P.nh = nh;
    P.col_tb = col_tb;
    P.row_rb = row_rb;
    P.col_rb = col_rb;
    // Pipelined launches keep two exchange buffers in flight (one written, one read).
    P.pipe = 0;
    if (o.pipeline == 2 && !sre_pipe_built(P))
      return fail(E_UNSUPPORTED, "SRE: no pipelined kernels for n = %d with these tiles", N);
    if (o.pipeline == 2 || (o.pipeline == 0 && SRE_PIPE_DEFAULT && sre_pipe_built(P))) P.pipe = 1;
    // Split LDS staging (half the LDS per workgroup) exists for the default column tiles and for
    // row tiles of 2^4 or 2^5 (FP32) / 2^4 (FP64) values.
    const bool split_ok = col_rb == RB && (row_rb == RB || row_rb == 4);
    if (o.lds_split == 2 && !split_ok)
      return fail(E_UNSUPPORTED, "SRE: split LDS staging needs the default column register tiles (2^%d)", RB);
    P.split = split_ok && (o.lds_split == 2 || (o.lds_split == 0 && !dbl && SRE_SPLIT_DEFAULT));
    if (nl == 15 && !P.split)
      return fail(E_UNSUPPORTED, "SRE: rows of 2^15 values need split LDS staging (HM_OPT_LDS_SPLIT 0 or 2)");
    if (o.streams == 2 && P.pipe) return fail(E_UNSUPPORTED, "SRE: two streams apply to sequential launches only");
    P.streams = (o.streams == 2 || (o.streams == 0 && SRE_STREAMS_DEFAULT == 2 && !P.pipe)) ? 2 : 1;
    // Untuned batch: 256 MiB of exchange per FP32 launch (measured best at n = 20 on MI355X: the
    // launch count matters more than staying inside the 256 MiB MALL), 128 MiB for FP64; pipelined
    // launches hold two buffers.
    const size_t per_shift = ((size_t)1 << P.nf) * (dbl ? 16 : 8);
    const size_t xb = P.pipe ? (64ull << 20) : dbl ? (128ull << 20) : (256ull << 20);
    int64_t b = o.batch > 0 ? o.batch : (int64_t)(xb / per_shift);
    if ((size_t)b * per_shift > (3ull << 30)) b = (int64_t)((3ull << 30) / per_shift);  // 32-bit offsets
    if (b < 1) b = 1;
    if (b > ((int64_t)1 << N)) b = (int64_t)1 << N;
    P.batch = (int)b;
  }
  *p = P;
  return OK;
}

// Workspace layout: [per-shift sums, unless the caller supplies them] [exchange] [column partials].

size_t sre_workspace(const SrePlan &p, int nq, int64_t n_internal_slots) {
  const size_t nacc = (size_t)nq + 1;
  size_t b = align256((size_t)n_internal_slots * nacc * sizeof(double));
  if (p.path == 2) {
    const size_t lane = sre_exch_bytes(p) + 2 * align256((size_t)p.batch * (size_t)sre_col_blocks(p) * nacc *
                                                         sizeof(double));  // double-buffered partials
    b += (p.streams == 2 ? 2 : 1) * lane;
  }
  return b < 256 ? 256 : b;
}

int sre_run(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows, int64_t n_slots,
            double *ext_shift_sums, double *sums, double *out, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  double *ss = ext_shift_sums;
  if (!ss) {
    ss = (double *)w;
    w += align256((size_t)n_slots * (size_t)nacc_of(qa) * sizeof(double));
  }
  int e = p.dbl ? sre_shift_sums_f64(p, psi, qa, a0, rows, n_slots, ss, w, st)
                : sre_shift_sums_f32(p, psi, qa, a0, rows, n_slots, ss, w, st);
  if (e) return e;
  if (sums || out) {
    // the two-pass path's exchange region is free again once the shift sums are written (stream
    // order) and holds the first-level partials of a long shift list
    const size_t spare = p.path == 2 ? sre_exch_bytes(p) : 0;
    return sre_reduce_shifts(ss, n_slots, qa, p.N, sums, out, st, (double *)w, spare);
  }
  return OK;
}

// Above 2^18 shifts the sum runs in two levels (TOT_PARTS workgroups over contiguous chunks, then
// one over their partials) where scratch for the partials is given; one workgroup otherwise.
static constexpr int64_t TOT_TWO_LEVEL = (int64_t)1 << 18;
static constexpr int TOT_PARTS = 512;

int sre_reduce_shifts(const double *shift_sums, int64_t n_slots, const QArgs &qa, int N, double *sums, double *out,
                      hipStream_t st, double *scratch, size_t scratch_bytes) {
  ProfScope prof("sre_total", st);
  const int nacc = nacc_of(qa);
  if (n_slots > TOT_TWO_LEVEL && scratch && scratch_bytes >= (size_t)TOT_PARTS * nacc * sizeof(double)) {
    const int64_t chunk = (n_slots + TOT_PARTS - 1) / TOT_PARTS;
    hipLaunchKernelGGL(k_sre_total_part, dim3(TOT_PARTS), dim3(TOT_NT), 0, st, shift_sums, n_slots, nacc, chunk, scratch);
    hipLaunchKernelGGL(k_sre_total, dim3(1), dim3(TOT_NT), 0, st, (const double *)scratch, (int64_t)TOT_PARTS, nacc, qa,
                       N, sums, out);
  } else {
    hipLaunchKernelGGL(k_sre_total, dim3(1), dim3(TOT_NT), 0, st, shift_sums, n_slots, nacc, qa, N, sums, out);
  }
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE reduce launch: %s", hipGetErrorString(hipGetLastError()));
}

size_t sre_states_workspace(const SrePlan &p, int nq, int n_states) {
  return align256(((size_t)n_states << p.N) * ((size_t)nq + 1) * sizeof(double));
}

int sre_run_states(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *const *outs,
                   void *ws, hipStream_t st) {
  if (p.path != 1) return fail(E_UNSUPPORTED, "batched launch needs the workgroup-resident path (n = %d)", p.N);
  if (n_states < 1 || n_states > HM_BATCH_PTRS) return fail(E_ARG, "batched launch of %d states", n_states);
  double *ss = (double *)ws;
  int e = p.dbl ? sre_states_f64(p, psis, n_states, qa, ss, st) : sre_states_f32(p, psis, n_states, qa, ss, st);
  if (e) return e;
  StateOuts o{};
  for (int i = 0; i < n_states; ++i) o.out[i] = outs[i];
  ProfScope prof("sre_state_totals", st);
  hipLaunchKernelGGL(k_sre_state_totals, dim3(n_states), dim3(256), 0, st, ss, p.N, nacc_of(qa), qa, o);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE batched totals: %s", hipGetErrorString(hipGetLastError()));
}

int sre_sampled_stats(const double *row_sums, const uint64_t *rows, int64_t n_rows, int nacc, const double *s0_sums,
                      int N, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sre_sampled_stats, dim3(1), dim3(256), 0, st, row_sums, rows, n_rows, nacc, s0_sums, N, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "SRE sampled stats: %s", hipGetErrorString(hipGetLastError()));
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
