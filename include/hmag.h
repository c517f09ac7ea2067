/*
 * hmag.h -- C-ABI of libhmag: numerically exact magic of pure state vectors on AMD MI355X (gfx950).
 *
 * Computes, for a state vector psi of N qudits:
 *   - qubits (d = 2): the stabilizer Renyi entropies M_q (Eq. sre of "Computing quantum magic of
 *     state vectors", Sec. 2) by Algorithm 2: for every X-string a, the vector
 *     v_x = conj(psi_{x XOR a}) psi_x is Walsh-Hadamard transformed (Eqs. Z_FT_qubits, Z_ovN) to give
 *     chi_b(a) = <psi|X_a Z_b|psi> for all Z-strings b, and S_q = sum_{a,b} |chi_b(a)|^{2q};
 *   - qutrits (d = 3): the pure-state mana (Eq. mana2) by Algorithm 4: for every shift a in Z_3^N,
 *     v_x = conj(alpha_x) alpha_{-x} with alpha = X_a psi is transformed by F_3^{(x)N},
 *     (F_3)_{jk} = omega^{2jk} (Eqs. mana_FT, F3_unnorm_def), and m = sum_{a,b} |chi_b(a)|.
 *
 * Conventions shared by every entry point
 *   - State layout: psi[x] for basis index x = sum_k x_k d^k (qudit k is digit k, little-endian),
 *     interleaved (re, im): HM_C64 = 2 x float per amplitude, HM_C128 = 2 x double.
 *   - Pointers named psi, out, sums, rows, row_sums, grad, ws are DEVICE pointers (HIP global
 *     memory of the current device), owned by the caller; the library never frees or retains them.
 *     psi must be 8-byte (C64) or 16-byte (C128) aligned; ws must be 256-byte aligned.
 *   - q (Renyi indices) is a HOST array of n_q doubles, 1 <= n_q <= HM_MAX_Q, each q > 0 and finite.
 *     q == 1 means the Shannon limit M_1 = -2^{-N} sum_P <P>^2 log2 <P>^2.
 *   - Work is enqueued on `stream` (NULL = the default stream) and is stream-ordered: buffers must
 *     stay alive until the stream has consumed them.  Results are written to device memory; no call
 *     synchronises the host unless its description says so.
 *   - Every argument is validated on the host before anything is enqueued; on error nothing is
 *     launched and the outputs are untouched.  The detailed message of the last error on the calling
 *     thread is available from hm_last_error().
 *   - The state is not renormalised (S_q scales as |psi|^{4q}); lost_norm reports 1 - sum_P <P>^2/2^N.
 *   - Results are bitwise reproducible for a fixed (entry point, n, dtype, q list, launch plan,
 *     library build): every reduction runs in a fixed order.  The plan is the handle's options or
 *     its autotuned choice; another plan (e.g. other row bits) changes the FP32 rounding of the
 *     transforms, and with it the last bits of the result.
 *   - Floating point: HM_C128 runs the transforms and sums in FP64.  HM_C64 runs the transforms in
 *     FP32 and accumulates every sum over Pauli strings / phase-space points in FP64 (each thread
 *     sums at most 64 FP32 terms before widening).
 */
#ifndef HMAG_H
#define HMAG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HM_MAX_Q 8

typedef enum {
  HM_OK = 0,
  HM_E_ARG = 1,         /* null/invalid pointer or argument (message says which)              */
  HM_E_DTYPE = 2,       /* dtype not HM_C64 / HM_C128                                          */
  HM_E_SIZE = 3,        /* n outside the supported range for this entry point                  */
  HM_E_WORKSPACE = 4,   /* ws_bytes smaller than the size the matching *_workspace call gives   */
  HM_E_UNSUPPORTED = 5, /* valid request the library does not implement (message says what)   */
  HM_E_HIP = 6,         /* a HIP runtime call failed (message carries hipGetErrorString)       */
  HM_E_ALIGN = 7,       /* a pointer violates the alignment stated above                      */
  HM_E_NOT_NORMALIZED = 8 /* HM_OPT_CHECK_NORM set and sum |psi|^2 off 1 (see HM_OPT_CHECK_NORM) */
} hm_status;

typedef enum { HM_C64 = 0, HM_C128 = 1 } hm_dtype;

/* Library context: holds per-device launch plans and options; owns no device memory. */
typedef struct hm_context *hm_handle;

hm_status hm_create(hm_handle *h);
hm_status hm_destroy(hm_handle h);
const char *hm_status_string(hm_status s);
/* Message describing the most recent failure on the calling thread ("" if none). */
const char *hm_last_error(void);
/* Version string of the library (names the target, gfx950). */
const char *hm_version(void);

/* Options (testing and tuning); 0 always means "automatic".
 *   HM_OPT_FORCE_PATH: SRE kernel family, 1 = workgroup-resident (one workgroup holds a whole
 *     folded shift vector), 2 = two-pass (row pass, exchange through device memory, column pass).
 *   HM_OPT_BATCH_SHIFTS: X-shifts covered by one two-pass launch pair (qubit SRE and qutrit mana).
 *   HM_OPT_ROW_RB / HM_OPT_COL_RB: log2 of the values each thread holds in registers in the
 *     two-pass row / column kernels (4 or 5 for HM_C64, 4 for HM_C128).
 *   HM_OPT_ROW_BITS: index bits handled by the two-pass row pass (6..13; 14 and 15 for HM_C64); the
 *     column pass takes the remaining n - 1 - row_bits.  Unset, the row pass takes about half the
 *     bits, and from n = 22 on (HM_C64, sequential launches) 13, 14 at n = 25 and 15 at n = 26, so
 *     that the column tiles keep reading several contiguous values of each row.
 *   HM_OPT_PIPELINE: two-pass launches, 1 = one row pass then one column pass per batch of
 *     shifts, 2 = pipelined (each launch runs the row pass of batch k beside the column pass of
 *     batch k - 1, with two exchange buffers; default tiles and split only).
 *   HM_OPT_LDS_SPLIT: 1 = stage complex values through LDS, 2 = stage real and imaginary parts one
 *     after the other (half the LDS per workgroup, so more workgroups per CU): two-pass kernels
 *     with the default column register tiles, and workgroup-resident tiles of 2^10..2^14 (HM_C64)
 *     or 2^10..2^13 (HM_C128) values, which then also keep to a register budget of three or four
 *     waves per SIMD; the default for the resident tiles and for HM_C64 two-pass kernels.
 *   HM_OPT_STREAMS: sequential two-pass launches on 1 stream (the caller's) or 2 (batches alternate
 *     between the caller's stream and an internal stream of the library, forked from and joined
 *     back into the caller's stream with events, so results stay stream-ordered; twice the
 *     exchange workspace).  Applies to SRE and mana (default 1 for both).  The FP64 partial
 *     sums of two-stream mana are grouped per stream, so its last bits differ from the
 *     one-stream result (each is deterministic).
 *   HM_OPT_CHECK_NORM (0 or 1, default 0): every entry point that takes a state first computes
 *     sum_x |psi_x|^2 in FP64 on the device, synchronises `stream` (so not usable under stream
 *     capture) and returns HM_E_NOT_NORMALIZED, with nothing else enqueued, when it is off 1 by
 *     more than 1e-5 (HM_C64) or 1e-12 (HM_C128).  The results assume a unit state (the paper's
 *     problem statement; S_q scales as |psi|^{4q}); without the check the state is used as given
 *     and lost_norm reports the deviation.  The check's two scalars (one device, one pinned host
 *     double per device) are allocated by the library on first use and kept until the process
 *     ends.
 *   HM_OPT_BATCH_LAUNCH: how hm_sre_batched runs its workgroup-resident states: 1 (default) = one
 *     persistent launch for all of them, as many workgroups as fit the device taking work units from
 *     a device counter; 2 = one launch per size class of up to 64 states, each with the kernel
 *     specialised for that size.
 * A combination outside the built kernels makes the SRE calls return HM_E_UNSUPPORTED. */
typedef enum {
  HM_OPT_FORCE_PATH = 1,
  HM_OPT_BATCH_SHIFTS = 2,
  HM_OPT_ROW_RB = 3,
  HM_OPT_COL_RB = 4,
  HM_OPT_ROW_BITS = 5,
  HM_OPT_PIPELINE = 6,
  HM_OPT_LDS_SPLIT = 7,
  HM_OPT_STREAMS = 8,
  HM_OPT_CHECK_NORM = 9,
  HM_OPT_BATCH_LAUNCH = 10
} hm_option;
hm_status hm_set_option(hm_handle h, hm_option opt, int64_t value);

/* Autotuner.  Times every candidate SRE plan for (n, dtype) on the state psi (device) over the
 * first sample_shifts X-shifts (16384 if <= 0, at most 2^n): the workgroup-resident kernel where it
 * applies, and two-pass plans over exchange batches of 64/128/256 MiB, both LDS stagings,
 * sequential launches (one or two streams) with the default, 11, 12 or 13 row bits (and 14, 15 for
 * HM_C64 from n = 20 on), and pipelined
 * launches.  Options already set on the handle are kept fixed.  The fastest plan is stored in the handle; later calls
 * on the handle for the same (n, dtype) fill every option left automatic from it.  Candidates
 * whose workspace exceeds ws_bytes are skipped (hm_autotune_workspace gives the size that admits
 * all of them).  Blocks until the timings are done (it synchronises on events on `stream`).
 * Results of the sampled shifts are discarded. */
hm_status hm_autotune_workspace(hm_handle h, int n, hm_dtype dtype, int64_t sample_shifts, size_t *bytes);
hm_status hm_autotune(hm_handle h, const void *psi, int n, hm_dtype dtype, int64_t sample_shifts, void *ws,
                      size_t ws_bytes, hipStream_t stream);
/* Autotuners of the other plans; each times its candidates on the caller's data (a warm-up and one
 * timed run each, hipEvents on `stream`, blocking until done), keeps the fastest in the handle and
 * is used from then on for options left automatic.  Results of the timed runs are discarded.
 *   hm_autotune_mana: exchange of 128 / 192 / 256 MiB per two-pass launch pair on one or two
 *     streams, over the first sample_shifts shifts (4096 if <= 0); HM_OPT_BATCH_SHIFTS and
 *     HM_OPT_STREAMS set on the handle are kept.
 *   hm_autotune_grad: workgroup-resident or two-pass gradient kernels (where both exist for n), one
 *     full fused forward + adjoint each; out and grad as hm_sre_grad.
 *   hm_autotune_batched: hm_sre_batched's launch form (HM_OPT_BATCH_LAUNCH 1 or 2) on the given
 *     batch, M_2 only; out as hm_sre_batched with n_q = 1; workspace: the larger of the two forms'
 *     hm_sre_batched_workspace.  HM_E_ARG if HM_OPT_BATCH_LAUNCH is set on the handle. */
hm_status hm_autotune_mana_workspace(hm_handle h, int n, hm_dtype dtype, size_t *bytes);
hm_status hm_autotune_mana(hm_handle h, const void *psi, int n, hm_dtype dtype, int64_t sample_shifts, void *ws,
                           size_t ws_bytes, hipStream_t stream);
hm_status hm_autotune_grad_workspace(hm_handle h, int n, hm_dtype dtype, size_t *bytes);
hm_status hm_autotune_grad(hm_handle h, const void *psi, int n, hm_dtype dtype, double q, double *out, void *grad,
                           void *ws, size_t ws_bytes, hipStream_t stream);
hm_status hm_autotune_batched(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype,
                              double *out, void *ws, size_t ws_bytes, hipStream_t stream);
/* The stored plan for (n, dtype): opts[0..7] = {HM_OPT_FORCE_PATH, HM_OPT_BATCH_SHIFTS,
 * HM_OPT_ROW_RB, HM_OPT_COL_RB, HM_OPT_ROW_BITS, HM_OPT_PIPELINE, HM_OPT_LDS_SPLIT, HM_OPT_STREAMS}
 * values (host array of 8), and its measured milliseconds per X-shift.  HM_E_ARG if none is
 * stored. */
hm_status hm_tune_query(hm_handle h, int n, hm_dtype dtype, int64_t *opts, double *ms_per_shift);
/* Forgets every stored plan of the handle (SRE, mana, gradient and batched). */
hm_status hm_tune_clear(hm_handle h);

/* ------------------------------------------------------------------------------------------ */
/* Workspace sizes.  Each entry point needs a device workspace of at least the returned size.   */
/* ------------------------------------------------------------------------------------------ */
typedef enum {
  HM_OP_SRE = 0,        /* hm_sre and hm_sre_partial (count ignored)                         */
  HM_OP_SRE_ROWS = 1,   /* hm_sre_rows; count = n_rows                                       */
  HM_OP_ROW_VALUES = 2, /* hm_sre_row_values (count ignored)                                 */
  HM_OP_SRE_GRAD = 3,   /* hm_sre_grad (count ignored)                                       */
  HM_OP_MANA = 4,       /* hm_mana and hm_mana_partial (count ignored)                       */
  HM_OP_SRE_SAMPLED = 5, /* hm_sre_sampled; count = n_rows                                   */
  HM_OP_SRE_GRAD_BATCHED = 6, /* hm_sre_grad_batched; count = batch                         */
  HM_OP_MANA_MIXED = 7,  /* hm_mana_mixed (count ignored)                                     */
  HM_OP_MANA_QUDIT = 8   /* hm_mana_qudit; count = d (3, 5 or 7)                              */
} hm_op;
hm_status hm_workspace_size(hm_handle h, hm_op op, int n, hm_dtype dtype, int n_q, int64_t count,
                            size_t *bytes);

/* ------------------------------------------------------------------------------------------ */
/* Qubits: stabilizer Renyi entropy (Eq. sre, Algorithm 2)                                     */
/* ------------------------------------------------------------------------------------------ */
/* out[0..n_q-1] = M_{q_i}(psi); out[n_q] = lost_norm = 1 - sum_P <P>^2 / 2^n.
 * 1 <= n <= 26 (HM_C64) or 25 (HM_C128).  out: device, n_q + 1 doubles. */
hm_status hm_sre(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q, int n_q,
                 double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Raw sums over the X-shifts a in [a0, a1): the X-string loop of Algorithm 2 cut into chunks
 * (Sec. "Calculation of SRE for qubits": the loop over X-strings of Algorithm 2 splits into chunks
 * evaluated independently), for sharding over devices and checkpoint/resume:
 *   sums[0] = sum_{a,b} |chi_b(a)|^2,
 *   sums[1+i] = sum_{a,b} |chi_b(a)|^{2 q_i}   (q_i == 1: sum |chi|^2 log2 |chi|^2).
 * Sums over disjoint ranges add up to the sums over their union.  0 <= a0 <= a1 <= 2^n.
 * sums: device, n_q + 1 doubles (overwritten). */
hm_status hm_sre_partial(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q,
                         int n_q, uint64_t a0, uint64_t a1, double *sums, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* Turns raw sums (layout of hm_sre_partial, over all 2^n shifts) into out = {M_q..., lost_norm}
 * (Eq. sre; the q -> 1 limit for q == 1).  sums, out: device. */
hm_status hm_sre_finalize(int n, const double *q, int n_q, const double *sums, double *out,
                          hipStream_t stream);

/* Per-row sums for an explicit list of X-strings (the row evaluation of the sampling algorithm,
 * Eq. feP, and of uniform-row Monte Carlo):
 *   row_sums[r*(n_q+1) + 0] = sum_b |chi_b(rows[r])|^2,  row_sums[r*(n_q+1) + 1+i] = sum_b |chi_b|^{2 q_i}.
 * rows: device array of n_rows uint64 values, each < 2^n (checked on the device: rows out of range
 * give NaN row sums).  row_sums: device, n_rows * (n_q + 1) doubles. */
hm_status hm_sre_rows(hm_handle h, const void *psi, int n, hm_dtype dtype, const uint64_t *rows,
                      int64_t n_rows, const double *q, int n_q, double *row_sums, void *ws,
                      size_t ws_bytes, hipStream_t stream);

/* Signed real Pauli expectations of one X-row: out[b] = <psi|P_{a,b}|psi> for b in [0, 2^n), with
 * P_{a,b} the Hermitian Pauli string whose qubit k carries I, X, Z, Y for (a_k, b_k) = (0,0), (1,0),
 * (0,1), (1,1); i.e. out[b] = i^{popcount(a & b)} chi_b(a).  out: device, 2^n doubles.  n <= 26. */
hm_status hm_sre_row_values(hm_handle h, const void *psi, int n, hm_dtype dtype, uint64_t a,
                            double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Fused forward + adjoint of M_q (q != 1): out = {M_q, lost_norm} (device, 2 doubles);
 * grad = dM_q/dRe(psi) + i dM_q/dIm(psi) (torch's convention), same dtype and length as psi
 * (device).  The adjoint differentiates chi_b(a) through Algorithm 2: with
 * w_b(a) = |chi_b(a)|^{2q-2} chi_b(a), dS_q/dpsi*_y = 2q sum_a psi_{y XOR a} [H^{(x)n} w(a)]_y.
 * 1 <= n <= 20: one workgroup per X-shift up to n = 13 (HM_C64) / 12 (HM_C128), two-pass kernels
 * above (and for n >= 12 when HM_OPT_FORCE_PATH is 2).  The transforms of each shift are recomputed
 * (nothing is stored across shifts).  Precision of the accumulation over shifts: the scalar sums
 * are FP64; the gradient is summed in the state's precision within a workgroup (the resident
 * kernels hold one copy of it per workgroup in LDS, i.e. FP32 for HM_C64, over the shifts that
 * workgroup takes) and in FP64 across workgroups; the two-pass kernels add every batch of shifts
 * into FP64 partials. */
hm_status hm_sre_grad(hm_handle h, const void *psi, int n, hm_dtype dtype, double q, double *out,
                      void *grad, void *ws, size_t ws_bytes, hipStream_t stream);

/* hm_sre_grad for `batch` states of one size n (the same adjoint): psis[s] and grads[s] are host
 * arrays of device pointers (the arrays are read during the call and not kept); out (device,
 * 2 * batch doubles) receives {M_q, lost_norm} of state s at out[2 s].  Up to n = 13 (HM_C64) /
 * 12 (HM_C128) each launch covers up to 64 states, one workgroup row per state; above, the
 * two-pass kernels take the states one after another, from n = 15 on in turn on two streams (the
 * caller's and an internal one, default priority), each with half of the workspace; the call
 * returns with all work ordered before later work on `stream`.  Results equal
 * hm_sre_grad's up to the order of the FP64 partial sums.  Workspace:
 * hm_workspace_size(HM_OP_SRE_GRAD_BATCHED, count = batch).  batch >= 1. */
hm_status hm_sre_grad_batched(hm_handle h, const void *const *psis, int n, int batch, hm_dtype dtype,
                              double q, double *out, void *const *grads, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* hm_sre_grad for `batch` states of uneven n (one q): psis, grads: HOST arrays of `batch` DEVICE
 * pointers, ns: HOST array of their n (1..20).  Consecutive states of equal n form one batched
 * gradient (hm_sre_grad_batched) each, so a batch ordered by n is taken in the fewest runs; the
 * runs share the workspace in stream order.  out (device, 2 * batch doubles) receives {M_q, lost_norm}
 * of state s at out[2 s]; grads[s] as hm_sre_grad's grad (same dtype and length as psis[s]).
 * Workspace: hm_sre_batched_grad_workspace (the largest run's).  This is the gradient of the batched
 * form of Algorithm 2 (the X-string loop of every state in independent chunks, Sec. "Calculation of
 * SRE for qubits"), differentiated as for hm_sre_grad. */
hm_status hm_sre_batched_grad_workspace(hm_handle h, const int *ns, int batch, hm_dtype dtype, size_t *bytes);
hm_status hm_sre_batched_grad(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype,
                              double q, double *out, void *const *grads, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* Many states, each of its own qubit count, in one call (all of one dtype and one q list): the
 * batched form of Algorithm 2 (every X-shift of every state is an independent transform; the
 * chunks of the X-string loop that Sec. "Calculation of SRE for qubits" evaluates separately).
 * psis: HOST array of `batch` DEVICE pointers (one state each); ns: HOST array of their n.
 * out: device, batch * (n_q + 1) doubles; out[s*(n_q+1) + i] = M_{q_i}(psi_s), out[s*(n_q+1) + n_q]
 * = lost_norm of state s (as hm_sre).  The states whose folded vector fits one workgroup tile
 * (6 <= n <= 16 for HM_C64, 5 <= n <= 15 for HM_C128) run in ONE persistent launch: their work
 * units (tiles of the workgroup-resident row pass: one shift at the largest n, several whole shifts
 * of smaller states) are numbered largest state first and taken from a device counter by a grid of
 * as many workgroups as fit the device; the state table reaches the device through kernel arguments
 * (no host-to-device copy).  One workgroup per state then sums its per-shift sums in a fixed order,
 * so results are deterministic and equal hm_sre's up to the order of the FP64 sums and the FP32
 * tile shape.  Smaller states run by size class (up to 64 per launch) and two-pass sizes one after
 * another, after the persistent launch, on the same workspace.  HM_OPT_BATCH_LAUNCH = 2 runs every
 * resident size class in a launch of its own instead.  Workspace: hm_sre_batched_workspace. */
hm_status hm_sre_batched_workspace(hm_handle h, const int *ns, int batch, hm_dtype dtype, int n_q,
                                   size_t *bytes);
hm_status hm_sre_batched(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype,
                         const double *q, int n_q, double *out, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* Monte Carlo estimate of M_2 from sampled X-rows (Sec. "Monte Carlo sampling algorithm for SRE":
 * a row is one transform, Eq. feP; here with uniform rows instead of the Metropolis chain of
 * hm_sre_mc).  S(a) = sum_b |chi_b(a)|^4 and M_2 = -log2(mean over all a of S(a)).  The
 * row a = 0 holds the identity, whose single term <I>^4 = 1 is about a quarter of the sum for
 * Haar-like states and would almost never be drawn, so that row is always evaluated exactly and the sampled rows
 * (caller-drawn, e.g. i.i.d. uniform in [1, 2^n); entries equal to 0 are skipped) estimate the
 * mean over a != 0:
 *   S_hat = (S(0) + (2^n - 1) mean_k S(a_k)) / 2^n,  M2_hat = -log2 S_hat.
 * out (device, 4 doubles) = {M2_hat, its standard error (2^n - 1) std_k S / (2^n sqrt(K) S_hat ln 2)
 * with K the number of nonzero rows, S_hat, std_k S(a_k)}.  n_rows >= 2; K < 2 gives NaN errors.
 * Workspace: hm_workspace_size(HM_OP_SRE_SAMPLED, count = n_rows). */
hm_status hm_sre_sampled(hm_handle h, const void *psi, int n, hm_dtype dtype, const uint64_t *rows,
                         int64_t n_rows, double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Monte Carlo estimate of M_2 by thermodynamic integration (sampling algorithm for the SRE,
 * Sec. "Monte Carlo sampling algorithm for SRE": Eqs. feP, Boltz, f_expect_beta_reg, Ie, Var_I_eps,
 * m2error).  L = n_beta inverse temperatures beta_l = l / (L - 1) (L odd: composite Simpson rule),
 * R = chains_per_beta independent Metropolis chains at each, C = L R chains in all (chain
 * c = l R + r).  Each chain walks over X-strings a with the energy f(a) = -ln(S'(a) + epsilon),
 * S(a) = sum_b chi_b(a)^4 evaluated by one Walsh-Hadamard transform per proposal (Eq. feP with the
 * natural log, which the Boltzmann and integration identities require), proposal a' = a XOR m and
 * acceptance min(1, exp(-beta_l (f(a') - f(a)))), always at beta = 0.  With exclude_identity = 1
 * the identity string (a = 0, b = 0) is left out of the sampled energy, S'(0) = S(0) - <I>^4,
 * and added back exactly.  <f>_beta_l is the mean of the chains' energies after n_therm steps,
 * I = sum_l w_l <f>_beta_l (Simpson weights) estimates ln Z_0 - ln Z_1 (Eq. f_expect_beta_reg
 * integrated; the paper's Eq. TI_logZ_reg carries the opposite sign), and
 *   M2_hat = -log2(e^-I - epsilon + exclude_identity 2^-n),
 *   dM2 = e^-I / (e^-I - epsilon + ...) sqrt(sum_l w_l^2 var_l) / ln 2,
 *   var_l = sum_r 2 tau_r sigma_r^2 / ((n_steps - n_therm) R^2), tau_r the integrated
 *   autocorrelation time of chain r (window: smallest W >= 5 tau(W)).
 * The randomness is the caller's (device arrays, e.g. drawn from a seeded generator):
 *   a_init: C initial X-strings; moves: n_steps x C XOR masks (step-major); uniforms: n_steps x C
 *   numbers in [0, 1) for the acceptance tests.  Bits at or above n are ignored.
 * Outputs (device): trace: n_steps x C doubles, the energy of each chain after each step;
 *   out: 4 + 5 L doubles = {M2_hat, dM2, I, S2_hat = 2^n (e^-I - epsilon + ...)}, then per beta_l:
 *   {<f>_l, variance of <f>_l, sigma_f^2 (mean over its chains), tau_int (mean), acceptance rate}.
 * A zero row sum with epsilon = 0 gives f = +inf (never entered at beta > 0; the beta = 0 chains
 * then make the result infinite or NaN): use epsilon > 0 for states with vanishing sectors.
 * Per step: one row launch over the C proposals (hm_sre_rows' kernels) and one small kernel; n_steps
 * steps are enqueued without host synchronisation.  1 <= n <= 26 (HM_C64) / 25 (HM_C128).
 * Workspace: hm_sre_mc_workspace (2^n doubles for S'(0) when exclude_identity, plus the row
 * kernels' workspace and O(C) chain state). */
typedef struct {
  int n_beta;           /* L: odd, 3 <= L <= 1025                                   */
  int chains_per_beta;  /* R >= 1, L R <= 2^20                                      */
  int64_t n_steps;      /* Metropolis steps per chain, >= 2                         */
  int64_t n_therm;      /* leading steps left out of the averages, <= n_steps - 2   */
  double epsilon;       /* regulariser of Eq. feP, >= 0                             */
  int exclude_identity; /* 0 or 1                                                   */
} hm_mc_params;
hm_status hm_sre_mc_workspace(hm_handle h, int n, hm_dtype dtype, const hm_mc_params *params, size_t *bytes);
hm_status hm_sre_mc(hm_handle h, const void *psi, int n, hm_dtype dtype, const hm_mc_params *params,
                    const uint64_t *a_init, const uint64_t *moves, const double *uniforms, double *out,
                    double *trace, void *ws, size_t ws_bytes, hipStream_t stream);

/* hm_sre without any device allocation, for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): same arguments and results
 * as hm_sre minus the workspace, bitwise equal to hm_sre's on the same handle options.  The per-shift
 * sums live in a scratch array inside the library, one per GPU, of HM_SRE_NOALLOC_MAX_BYTES (it
 * holds 2^16 shifts x (HM_MAX_Q + 1) doubles and stays allocated until the process ends).
 * Covers the workgroup-resident sizes: 1 <= n <= 16 (HM_C64) or 15 (HM_C128); larger n, or handle
 * options that select the two-pass kernels, return HM_E_SIZE.  HM_OPT_CHECK_NORM returns
 * HM_E_UNSUPPORTED (its scalars are allocated on first use).  Every call on a GPU uses that GPU's one
 * scratch array: calls that overlap on one GPU (other streams, other threads, other handles) race
 * and must be serialised by the caller; calls on one stream are ordered and safe.  Each call
 * overwrites every slot it reads, so nothing needs clearing between calls. */
#define HM_SRE_NOALLOC_MAX_BYTES ((size_t)4718592)
hm_status hm_sre_noalloc(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q, int n_q,
                         double *out, hipStream_t stream);

/* ------------------------------------------------------------------------------------------ */
/* Qutrits: pure-state mana (Eq. mana2, Algorithm 4)                                            */
/* ------------------------------------------------------------------------------------------ */
/* out[0] = mana = log2(sum_u |<psi|A_u|psi>| / 3^n); out[1] = sum_u W(u) (= 1);
 * out[2] = 3^n sum_u W(u)^2 (= 1 for a normalised pure state).  1 <= n <= 16.
 * out: device, 3 doubles.
 * Error of HM_C64 (FP32 transforms): every value chi_b(a) carries rounding noise of order 1e-7 of
 * the largest |chi|; where chi is exactly zero, |.| turns that noise into a one-sided excess of
 * sum |chi|, so the FP32 mana lies ABOVE the exact one by up to about 1.5e-5 at n = 10 and 4.5e-5
 * at n = 12 for states whose phase-space spectrum is mostly exact zeros (stabilizer states,
 * measured on MI355X), growing by about sqrt(3) per qutrit (about 4e-4 at n = 16).  States with
 * few exact zeros (Haar-like states) are within 1e-5 of the exact mana for n <= 12.  HM_C128 agrees
 * with the FP64 definition to about 1e-12 relative. */
hm_status hm_mana(hm_handle h, const void *psi, int n, hm_dtype dtype, double *out, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/* Raw sums over shifts a in [a0, a1) (a = sum_k a_k 3^k), the shift loop of Algorithm 4 cut into
 * chunks as the X-string loop of Algorithm 2 is (Sec. "Calculation of SRE for qubits"):
 * sums = {sum |chi|, sum chi, sum chi^2}.
 * sums: device, 3 doubles (overwritten).  0 <= a0 <= a1 <= 3^n. */
hm_status hm_mana_partial(hm_handle h, const void *psi, int n, hm_dtype dtype, uint64_t a0,
                          uint64_t a1, double *sums, void *ws, size_t ws_bytes, hipStream_t stream);


/* Pure-state mana of n qudits of odd prime dimension d in {3, 5, 7}: the construction of Sec. "Mana
 * for qutrits", which its footnote extends to every odd prime d (clock and shift operators with
 * omega = exp(2 pi i / d), T_ab = omega^{-2^{-1} a b} Z^a X^b, phase-space point operators A_u,
 * W(u) = <psi|A_u|psi> / d^n), computed by Algorithm 4 with radix-d transforms: for every shift a,
 * v_x = conj(alpha_x) alpha_{-x} with alpha = X_a psi, chi(a) = F_d^{(x)n} v, (F_d)_{jk} = omega^{2jk}.
 * psi: device, d^n amplitudes (qudit k = base-d digit k of the index), not renormalised.
 * out: device, 3 doubles = {mana = log2(sum_u |<psi|A_u|psi>| / d^n), sum_u W(u), d^n sum_u W(u)^2}
 * (1 and 1 for a normalised pure state).  The d^n values of a shift pair are transformed inside one
 * workgroup's LDS, which bounds n: 1 <= n <= 9 / 6 / 5 for d = 3 / 5 / 7 (HM_C64) and 8 / 5 / 4
 * (HM_C128); HM_E_SIZE above.  For d = 3, hm_mana is the fast path (to n = 16); this entry point
 * computes the same value through the generic kernel.  Precision as hm_mana (FP32 transforms and
 * FP64 sums for HM_C64).  Workspace: hm_workspace_size(HM_OP_MANA_QUDIT, count = d); HM_E_ARG for
 * d not in {3, 5, 7}. */
hm_status hm_mana_qudit(hm_handle h, const void *psi, int n, int d, hm_dtype dtype, double *out, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* Mana of a mixed state (Sec. "Mana of mixed states via a fast tensor-product transform", Eq.
 * MN_factor_mana and its Algorithm): all 9^n values w_u = Tr(rho A_u) as the tensor power of a 9 x 9
 * single-qutrit matrix applied to the reordered density matrix, several qutrits per HBM-streaming
 * pass (qutrits 0..2 in the pass that reorders rho, then two per pass, the last pass summing instead
 * of writing).
 * rho: device, 3^n x 3^n row-major (rho[r 3^n + c] = <r|rho|c>, qutrit k = base-3 digit k of r and c),
 * Hermitian (not checked; the imaginary parts of w are dropped).  out: device, 3 doubles
 * = {mana = log2(sum_u |w_u| / 3^n), sum_u W(u) = Tr rho, 3^n sum_u W(u)^2 = Tr rho^2} with
 * W = w / 3^n.  1 <= n <= 10.  Workspace: hm_workspace_size(HM_OP_MANA_MIXED): the reordered
 * 9^n-value copy of rho (HM_C128 at n = 10: 56 GB) plus 48 KB of partial sums. */
hm_status hm_mana_mixed(hm_handle h, const void *rho, int n, hm_dtype dtype, double *out, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* Reduced density matrix of a pure state on its first n_a qutrits (base-3 digits 0..n_a-1 of the
 * index; the others traced out): rho[i 3^n_a + j] = sum_b psi[i + 3^n_a b] conj(psi[j + 3^n_a b]),
 * summed in FP64, stored in the state's dtype, row-major 3^n_a x 3^n_a (device).  The subsystem
 * mana of the paper's examples is hm_mana_mixed of this matrix.  1 <= n_a <= min(n, 10), n <= 16.
 * No workspace. */
hm_status hm_reduced_density(hm_handle h, const void *psi, int n, int n_a, hm_dtype dtype, void *rho,
                             hipStream_t stream);

/* ------------------------------------------------------------------------------------------ */
/* Kernel timing (diagnostics)                                                                 */
/* ------------------------------------------------------------------------------------------ */
/* every > 0: every every-th launch of each kernel family (the first, the every+1-th, ...) is
 * bracketed by hipEvents recorded on its stream; 0 turns timing off (the default).  Sampling keeps
 * the event overhead of long launch sequences small.  Process-wide. */
hm_status hm_profile_enable(int every);
/* Drops the accumulated timings. */
hm_status hm_profile_reset(void);
/* Kernel family `index` (0-based, in order of first launch since the last reset): its name
 * (NUL-terminated, truncated to name_len), the number of its launches, the number of those that
 * were timed and their summed device milliseconds.  Synchronises with the recorded events.  Any
 * output pointer may be NULL.  HM_E_ARG once index passes the last family. */
hm_status hm_profile_query(int index, char *name, size_t name_len, int64_t *launches, int64_t *timed,
                           double *ms);

#ifdef __cplusplus
}
#endif
#endif /* HMAG_H */
