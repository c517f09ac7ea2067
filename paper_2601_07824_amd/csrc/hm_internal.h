// hm_internal.h -- declarations shared by the C-ABI layer and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#ifndef HM_MAX_Q
#define HM_MAX_Q 8
#endif
// states per batched launch (their pointers travel in the kernel arguments)
#define HM_BATCH_PTRS 64

namespace hm {

struct QArgs;

// Status codes mirror hm_status in include/hmag.h.
enum Status {
  OK = 0, E_ARG = 1, E_DTYPE = 2, E_SIZE = 3, E_WORKSPACE = 4, E_UNSUPPORTED = 5, E_HIP = 6, E_ALIGN = 7,
  E_NOT_NORMALIZED = 8
};

// Records a formatted message for hm_last_error() and returns st.
int fail(int st, const char *fmt, ...);

// Kernel timing hooks (hm_profile_*): bracket a launch on stream st.
void *prof_begin(const char *name, hipStream_t st);
void prof_end(void *tok, hipStream_t st);
struct ProfScope {
  void *tok;
  hipStream_t st;
  ProfScope(const char *name, hipStream_t s) : tok(prof_begin(name, s)), st(s) {}
  ~ProfScope() { prof_end(tok, st); }
};

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---- SRE forward -----------------------------------------------------------------------------
// Plan for one qubit count and dtype.
struct SrePlan {
  int N;        // qubits
  int nf;       // folded bits = N - 1
  int dbl;      // 1: FP64 transforms
  int path;     // 1: workgroup-resident, 2: two-pass
  int nl, nh;   // two-pass split: row bits, column-pass (row-index) bits; nl + nh = nf
  int batch;    // shifts per two-pass launch pair
  int col_tb;   // column tile bits (log2 of values per column tile)
  int row_rb;   // register-tile bits of the two-pass row pass
  int col_rb;   // register-tile bits of the column pass
  int pipe;     // 1: row pass of batch k and column pass of batch k-1 share one launch
  int split;    // 1: pipelined tiles stage one component at a time through LDS (half the LDS)
  int streams;  // 2: sequential batches alternate between the caller's stream and an internal one
};

// Default two-pass split.  Column tiles hold 2^col_tb values; the row pass takes about half of the
// folded bits, at least enough for one column tile's width, at least 6 and at most 13.
constexpr int sre_default_col_tb(int nf, int dbl, int col_rb) {
  return dbl ? (nf >= 12 ? 12 : 10) : (nf >= 13 ? 13 : 11);
}
constexpr int sre_default_nl(int nf, int col_tb, int col_rb) {
  int nl = (nf + 1) / 2, nh = nf - nl;
  if (nh < col_rb) { nh = col_rb; nl = nf - nh; }
  if (nl < col_tb - nh) { nl = col_tb - nh; nh = nf - nl; }
  if (nl < 6 && nf - 6 >= col_rb) nl = 6;  // shortest row the row-pass kernels are built for
  if (nl > 13) nl = 13;
  return nl;
}
// Folded-bit range with pipelined kernels built (default split and register tiles only).
constexpr int SRE_PIPE_NF_MIN = 11, SRE_PIPE_NF_MAX = 25;
inline bool sre_pipe_built(const SrePlan &p) {
  const int rb = p.dbl ? 4 : 5;
  return p.path == 2 && p.nf >= SRE_PIPE_NF_MIN && p.nf <= (p.dbl ? SRE_PIPE_NF_MAX - 1 : SRE_PIPE_NF_MAX) &&
         p.row_rb == rb && p.col_rb == rb &&
         p.col_tb == sre_default_col_tb(p.nf, p.dbl, rb) && p.nl == sre_default_nl(p.nf, p.col_tb, rb);
}
// Internal stream of the current device (created on first use, default priority, non-blocking),
// used as the second stream of two-stream plans.
int side_stream(hipStream_t *st);
// Workspace pieces of the two-pass path: exchange buffer(s) and per-column-block partials.
inline size_t sre_exch_bytes(const SrePlan &p) {
  if (p.path != 2) return 0;
  const size_t one = align256((size_t)p.batch * ((size_t)1 << p.nf) * (p.dbl ? 16 : 8));
  return p.pipe ? 2 * one : one;
}
inline int64_t sre_col_blocks(const SrePlan &p) { return (int64_t)1 << (p.nl - (p.col_tb - p.nh)); }

// Planner overrides (0 = automatic), set through hm_set_option.
struct PlanOpts {
  int force_path = 0;
  int64_t batch = 0;
  int row_rb = 0;
  int col_rb = 0;
  int row_bits = 0;
  int pipeline = 0;  // 0 automatic, 1 off, 2 on
  int lds_split = 0; // 0 automatic, 1 off, 2 on
  int streams = 0;   // 0 automatic, 1 or 2
  int batch_launch = 0;  // hm_sre_batched: 0 automatic, 1 one persistent launch, 2 one launch per size class
};

// Plan options chosen by the autotuner for one (qubit count, dtype).
struct TunedPlan {
  int n;
  int dbl;
  PlanOpts opts;
  double ms_per_shift;
};
// Mana plan chosen by the autotuner for one (qutrit count, dtype): X-shifts per two-pass launch pair
// and streams.
struct TunedMana {
  int n, dbl;
  int64_t batch;
  int streams;
  double ms_per_shift;
};
// Gradient path chosen by the autotuner for one (qubit count, dtype): 1 resident, 2 two-pass.
struct TunedGrad {
  int n, dbl;
  int path;
  double ms;
};

}  // namespace hm

// The handle: options set by the caller and the autotuner's table.
struct hm_context {
  hm::PlanOpts opts;
  std::vector<hm::TunedPlan> tuned;
  std::vector<hm::TunedMana> tuned_mana;
  std::vector<hm::TunedGrad> tuned_grad;
  int tuned_batch_launch = 0;  // launch form of hm_sre_batched picked by hm_autotune_batched
  int check_norm = 0;          // HM_OPT_CHECK_NORM
};

namespace hm {

// Autotuner: times the candidate plans for (n, dbl) on psi over the first `sample` X-shifts
// (16384 if <= 0, at most 2^n) and records the fastest in h->tuned.  Blocks until done.
int sre_autotune(hm_context *h, const void *psi, int n, int dbl, int64_t sample, void *ws, size_t ws_bytes,
                 hipStream_t st, TunedPlan *best);
size_t sre_autotune_workspace(const hm_context *h, int n, int dbl, int64_t sample);

// Options for planning (n, dbl) on handle h: every field the caller left automatic (0) is taken
// from the autotuner's entry for (n, dbl), if there is one.
PlanOpts plan_opts(const hm_context *h, int n, int dbl);
// The same for mana (X-shifts per launch pair, streams) and the gradient (path).
void mana_opts(const hm_context *h, int n, int dbl, int64_t *batch, int *streams);
PlanOpts grad_opts(const hm_context *h, int n, int dbl);

// Fills a plan; returns OK or E_UNSUPPORTED/E_SIZE with a message.
int sre_plan(int N, int dbl, const PlanOpts &o, SrePlan *p);
// Workspace bytes for a forward run whose per-shift sums live in the workspace for
// n_internal_slots shifts (0 when the caller supplies the per-shift output buffer).
size_t sre_workspace(const SrePlan &p, int nq, int64_t n_internal_slots);
// Per-shift sums for shifts a0 + s (rows == nullptr) or rows[s], s in [0, n_slots), in the unfolded
// convention; written to ext_shift_sums if given (else into ws).  If sums / out are given, also the
// fixed-order totals / the finalised {M_q..., lost_norm} for N qubits.  Enqueued on stream.
int sre_run(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows, int64_t n_slots,
            double *ext_shift_sums, double *sums, double *out, void *ws, hipStream_t stream);
int sre_reduce_shifts(const double *shift_sums, int64_t n_slots, const QArgs &qa, int N, double *sums, double *out,
                      hipStream_t stream, double *scratch = nullptr, size_t scratch_bytes = 0);
// Many states of one size n on the workgroup-resident path: per-shift sums of all shifts of the
// n_states states (pointers psis) in one launch, then one fixed-order total per state into
// outs[s][0..nq] = {M_q..., lost_norm}.
int sre_run_states(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *const *outs,
                   void *ws, hipStream_t stream);
size_t sre_states_workspace(const SrePlan &p, int nq, int n_states);
// Many states of uneven size in one persistent launch (hm_batch.hip): states whose folded vector
// fits one workgroup tile (batch_resident_ok), all shifts of all of them.  out[s (nq+1) ...] for
// each selected s.
bool batch_resident_ok(int N, int dbl);
size_t batch_persistent_workspace(const int *ns, const int *sel, int cnt, int nq, int dbl);
int batch_persistent_run(int dbl, const void *const *psis, const int *ns, const int *sel, int cnt, const QArgs &qa,
                         double *out, void *ws, hipStream_t stream);
// Monte Carlo M_2 from the row sums of sampled rows (rows equal to 0 skipped) and the exact row
// sums of a = 0: out = {M2_hat, standard error, S_hat, std of the sampled S(a)}.
int sre_sampled_stats(const double *row_sums, const uint64_t *rows, int64_t n_rows, int nacc, const double *s0_sums,
                      int N, double *out, hipStream_t stream);
int sre_finalize_launch(int N, const QArgs &qa, const double *sums, double *out, hipStream_t stream);

// Per-dtype drivers of the SRE kernels (one translation unit each).
int sre_shift_sums_f32(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                       int64_t n_slots, double *shift_sums, char *w, hipStream_t st);
int sre_shift_sums_f64(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                       int64_t n_slots, double *shift_sums, char *w, hipStream_t st);
int sre_pipe_f32(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                 int64_t n_slots, double *shift_sums, char *w, hipStream_t st);
int sre_pipe_f64(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                 int64_t n_slots, double *shift_sums, char *w, hipStream_t st);

// Row values <P_{a,b}> of one X-row (unfolded FWHT of one row).
int sre_row_values_launch(int N, int dbl, const void *psi, uint64_t a, double *out, void *ws, hipStream_t stream);
size_t sre_row_values_workspace(int N, int dbl);

// ---- input checks ----------------------------------------------------------------------------
// Squared norm of a state of D amplitudes on the device; synchronises `stream`; E_NOT_NORMALIZED
// when it is off 1 by more than 1e-5 (FP32) / 1e-12 (FP64).
int check_norm(const void *psi, uint64_t D, int dbl, hipStream_t stream);

// ---- SRE gradient ----------------------------------------------------------------------------
// Workgroup-resident kernel up to n = 13 (FP32) / 12 (FP64), two-pass kernels (default split)
// for n in [12, 20]; opts.force_path = 2 selects the two-pass kernels where both exist.
int sre_grad_launch(const PlanOpts &opts, int N, int dbl, const void *psi, double q, double *out, void *grad,
                    void *ws, size_t ws_bytes, hipStream_t stream);
int sre_grad_workspace(const PlanOpts &opts, int N, int dbl, size_t *bytes);
// batch states of one size: psis[s] -> out[2 s .. 2 s + 1], grads[s]; one resident launch per
// HM_BATCH_PTRS states, or the two-pass kernels state after state on one workspace.
int sre_grad_batched_launch(const PlanOpts &opts, int N, int dbl, const void *const *psis, int batch, double q,
                            double *out, void *const *grads, void *ws, size_t ws_bytes, hipStream_t stream);
int sre_grad_batched_workspace(const PlanOpts &opts, int N, int dbl, int batch, size_t *bytes);
int grad_totals_launch(const double *shift_sums, int64_t n_shifts, int N, double q, double *out, double *scale,
                       hipStream_t stream);
int sre_grad2_f32(const SrePlan &p, const void *psi, double q, double *out, void *grad, void *ws, hipStream_t st);
int sre_grad2_f64(const SrePlan &p, const void *psi, double q, double *out, void *grad, void *ws, hipStream_t st);
size_t sre_grad2_workspace_f32(const SrePlan &p);
size_t sre_grad2_workspace_f64(const SrePlan &p);

// ---- Mana ------------------------------------------------------------------------------------
// batch: X-shifts per two-pass launch pair (0 = automatic; HM_OPT_BATCH_SHIFTS of the handle).
// streams: two-pass batches alternate over 1 or 2 streams (0 = automatic, HM_OPT_STREAMS).
int mana_launch(int N, int dbl, int64_t batch, int streams, const void *psi, uint64_t a0, uint64_t a1, double *sums,
                double *out, void *ws, size_t ws_bytes, hipStream_t stream);
// Pure-state mana of qudits of odd prime dimension d in {3, 5, 7} (hm_qudit.hip): out = {mana, sum W,
// d^N sum W^2}; the d^N-value transform of a shift pair lives in one workgroup's LDS.
int qudit_nmax_of(int d, int dbl);
int qudit_workspace(int N, int d, int dbl, size_t *bytes);
int qudit_launch(int N, int d, int dbl, const void *psi, double *out, void *ws, hipStream_t st);
// Mixed-state mana (hm_mixed.hip): rho row-major 3^N x 3^N; out = {mana, Tr rho, Tr rho^2}.
int mixed_workspace(int N, int dbl, size_t *bytes);
int mixed_launch(int N, int dbl, const void *rho, double *out, void *ws, hipStream_t st);
int reduced_density_launch(int N, int NA, int dbl, const void *psi, void *rho, hipStream_t st);

// Workspace bytes of a mana call (E_SIZE when n has no plan).
int mana_workspace(int N, int dbl, int64_t batch, int streams, size_t *bytes);

}  // namespace hm
