// hm_internal.h -- declarations shared by the C-ABI layer and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#ifndef HM_MAX_Q
#define HM_MAX_Q 8
#endif

namespace hm {

struct QArgs;

// Status codes mirror hm_status in include/hmag.h.
enum Status { OK = 0, E_ARG = 1, E_DTYPE = 2, E_SIZE = 3, E_WORKSPACE = 4, E_UNSUPPORTED = 5, E_HIP = 6, E_ALIGN = 7 };

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
};

// Fills a plan; returns OK or E_UNSUPPORTED/E_SIZE with a message.
int sre_plan(int N, int dbl, int force_path, int64_t batch_opt, SrePlan *p);
// Workspace bytes for a forward run whose per-shift sums live in the workspace for
// n_internal_slots shifts (0 when the caller supplies the per-shift output buffer).
size_t sre_workspace(const SrePlan &p, int nq, int64_t n_internal_slots);
// Per-shift sums for shifts a0 + s (rows == nullptr) or rows[s], s in [0, n_slots), in the unfolded
// convention; written to ext_shift_sums if given (else into ws).  If sums / out are given, also the
// fixed-order totals / the finalised {M_q..., lost_norm} for N qubits.  Enqueued on stream.
int sre_run(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows, int64_t n_slots,
            double *ext_shift_sums, double *sums, double *out, void *ws, hipStream_t stream);
int sre_reduce_shifts(const double *shift_sums, int64_t n_slots, const QArgs &qa, int N, double *sums, double *out,
                      hipStream_t stream);
int sre_finalize_launch(int N, const QArgs &qa, const double *sums, double *out, hipStream_t stream);

// Row values <P_{a,b}> of one X-row (unfolded FWHT of one row).
int sre_row_values_launch(int N, int dbl, const void *psi, uint64_t a, double *out, void *ws, hipStream_t stream);
size_t sre_row_values_workspace(int N, int dbl);

// ---- SRE gradient ----------------------------------------------------------------------------
int sre_grad_launch(int N, int dbl, const void *psi, double q, double *out, void *grad, void *ws, size_t ws_bytes,
                    hipStream_t stream);
size_t sre_grad_workspace(int N, int dbl);

// ---- Mana ------------------------------------------------------------------------------------
int mana_launch(int N, int dbl, const void *psi, uint64_t a0, uint64_t a1, double *sums, double *out, void *ws,
                size_t ws_bytes, hipStream_t stream);
size_t mana_workspace(int N, int dbl, uint64_t n_shifts);

}  // namespace hm
