// hm_api.hip -- the C-ABI of libhmag (include/hmag.h): argument validation, planning, workspace
// sizing and dispatch to the gfx950 kernels.  Every check runs on the host before anything is
// enqueued, so a failing call launches nothing and leaves its outputs untouched.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <utility>
#include <vector>

#include "../../include/hmag.h"
#include "hm_internal.h"
#include "hm_tile.h"

#define HM_VERSION_STRING "hmag 0.1.0 (gfx950)"


namespace hm {

static thread_local char g_err[1024];

int fail(int st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

static int check_dtype(hm_dtype dt) {
  if (dt != HM_C64 && dt != HM_C128) return fail(E_DTYPE, "dtype %d is neither HM_C64 nor HM_C128", (int)dt);
  return OK;
}

static int check_ptr(const void *p, size_t align, const char *name) {
  if (!p) return fail(E_ARG, "%s is NULL", name);
  if ((uintptr_t)p % align) return fail(E_ALIGN, "%s = %p is not %zu-byte aligned", name, p, align);
  return OK;
}

static int check_q(const double *q, int n_q, QArgs *qa) {
  if (!q) return fail(E_ARG, "q is NULL");
  if (n_q < 1 || n_q > HM_MAX_Q) return fail(E_ARG, "n_q = %d outside [1, %d]", n_q, HM_MAX_Q);
  memset(qa, 0, sizeof(*qa));
  qa->nq = n_q;
  for (int i = 0; i < n_q; ++i) {
    if (!(q[i] > 0.0) || !isfinite(q[i])) return fail(E_ARG, "q[%d] = %g must be positive and finite", i, q[i]);
    qa->q[i] = q[i];
  }
  return OK;
}

static int check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (ws_bytes < need) return fail(E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, need);
  if (need > 0) {
    if (!ws) return fail(E_ARG, "ws is NULL but %zu bytes are needed", need);
    if ((uintptr_t)ws % 256) return fail(E_ALIGN, "ws = %p is not 256-byte aligned", ws);
  }
  return OK;
}

// HM_OPT_CHECK_NORM: the state's squared norm, checked on the device before anything is launched.
static int norm_ok(hm_handle h, const void *psi, int d, int n, hm_dtype dtype, hipStream_t stream) {
  if (!h->check_norm) return OK;
  uint64_t D = 1;
  for (int i = 0; i < n; ++i) D *= (uint64_t)d;
  return check_norm(psi, D, dtype == HM_C128, stream);
}

static size_t psi_align(hm_dtype dt) { return dt == HM_C128 ? 16 : 8; }

__global__ void k_fill(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static int fill_dev(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return OK;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "fill launch: %s", hipGetErrorString(hipGetLastError()));
}

// Times fn() once after a warm-up call, on stream st (milliseconds).
template <typename F>
static int time_once_api(hipStream_t st, F fn, float *ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(E_HIP, "autotune: hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(E_HIP, "autotune: hipEventCreate failed");
  }
  int err = fn();
  if (!err && hipEventRecord(e0, st) != hipSuccess) err = fail(E_HIP, "autotune: hipEventRecord failed");
  if (!err) err = fn();
  if (!err && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    err = fail(E_HIP, "autotune: %s", hipGetErrorString(hipGetLastError()));
  if (!err) (void)hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return err;
}

// Autotuners of the mana, gradient plans (hm_tune.hip).
size_t mana_autotune_workspace(const hm_context *h, int n, int dbl);
int mana_autotune(hm_context *h, const void *psi, int n, int dbl, int64_t sample, void *ws, size_t ws_bytes,
                  hipStream_t st);
size_t grad_autotune_workspace(const hm_context *h, int n, int dbl);
int grad_autotune(hm_context *h, const void *psi, int n, int dbl, double q, void *out, void *grad, void *ws,
                  size_t ws_bytes, hipStream_t st);

// Monte Carlo by thermodynamic integration (hm_mc.hip).
int mc_check(int n, const hm_mc_params *prm);
int mc_workspace(const SrePlan &p, const hm_mc_params *prm, size_t *bytes);
int mc_run(const SrePlan &p, const void *psi, const hm_mc_params *prm, const uint64_t *a_init, const uint64_t *moves,
           const double *uniforms, double *out, double *trace, void *ws, hipStream_t st);

}  // namespace hm

using namespace hm;

#define HM_TRY(x)                          \
  do {                                     \
    int _s = (x);                          \
    if (_s != OK) return (hm_status)_s;    \
  } while (0)

extern "C" {

hm_status hm_create(hm_handle *h) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  *h = new (std::nothrow) hm_context();
  if (!*h) return (hm_status)fail(E_ARG, "out of host memory");
  return HM_OK;
}

hm_status hm_destroy(hm_handle h) {
  delete h;
  return HM_OK;
}

const char *hm_status_string(hm_status s) {
  switch (s) {
    case HM_OK: return "HM_OK";
    case HM_E_ARG: return "HM_E_ARG: invalid argument";
    case HM_E_DTYPE: return "HM_E_DTYPE: unsupported dtype";
    case HM_E_SIZE: return "HM_E_SIZE: n outside the supported range";
    case HM_E_WORKSPACE: return "HM_E_WORKSPACE: workspace too small";
    case HM_E_UNSUPPORTED: return "HM_E_UNSUPPORTED: not implemented for these arguments";
    case HM_E_HIP: return "HM_E_HIP: HIP runtime error";
    case HM_E_ALIGN: return "HM_E_ALIGN: misaligned pointer";
    case HM_E_NOT_NORMALIZED: return "HM_E_NOT_NORMALIZED: state norm off 1 (HM_OPT_CHECK_NORM)";
  }
  return "unknown hm_status";
}

const char *hm_last_error(void) { return g_err; }
const char *hm_version(void) { return HM_VERSION_STRING; }

hm_status hm_set_option(hm_handle h, hm_option opt, int64_t value) {
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  switch (opt) {
    case HM_OPT_FORCE_PATH:
      if (value < 0 || value > 2) return (hm_status)fail(E_ARG, "HM_OPT_FORCE_PATH %lld not in {0,1,2}", (long long)value);
      h->opts.force_path = (int)value;
      return HM_OK;
    case HM_OPT_BATCH_SHIFTS:
      if (value < 0 || value > (1ll << 30)) return (hm_status)fail(E_ARG, "HM_OPT_BATCH_SHIFTS %lld out of range", (long long)value);
      h->opts.batch = value;
      return HM_OK;
    case HM_OPT_ROW_RB:
      if (value != 0 && value != 4 && value != 5) return (hm_status)fail(E_ARG, "HM_OPT_ROW_RB %lld not in {0,4,5}", (long long)value);
      h->opts.row_rb = (int)value;
      return HM_OK;
    case HM_OPT_COL_RB:
      if (value != 0 && value != 4 && value != 5) return (hm_status)fail(E_ARG, "HM_OPT_COL_RB %lld not in {0,4,5}", (long long)value);
      h->opts.col_rb = (int)value;
      return HM_OK;
    case HM_OPT_ROW_BITS:
      if (value != 0 && (value < 6 || value > 15)) return (hm_status)fail(E_ARG, "HM_OPT_ROW_BITS %lld not in {0, 6..15}", (long long)value);
      h->opts.row_bits = (int)value;
      return HM_OK;
    case HM_OPT_PIPELINE:
      if (value < 0 || value > 2) return (hm_status)fail(E_ARG, "HM_OPT_PIPELINE %lld not in {0,1,2}", (long long)value);
      h->opts.pipeline = (int)value;
      return HM_OK;
    case HM_OPT_LDS_SPLIT:
      if (value < 0 || value > 2) return (hm_status)fail(E_ARG, "HM_OPT_LDS_SPLIT %lld not in {0,1,2}", (long long)value);
      h->opts.lds_split = (int)value;
      return HM_OK;
    case HM_OPT_STREAMS:
      if (value < 0 || value > 2) return (hm_status)fail(E_ARG, "HM_OPT_STREAMS %lld not in {0,1,2}", (long long)value);
      h->opts.streams = (int)value;
      return HM_OK;
    case HM_OPT_BATCH_LAUNCH:
      if (value < 0 || value > 2) return (hm_status)fail(E_ARG, "HM_OPT_BATCH_LAUNCH %lld not in {0,1,2}", (long long)value);
      h->opts.batch_launch = (int)value;
      return HM_OK;
    case HM_OPT_CHECK_NORM:
      if (value < 0 || value > 1) return (hm_status)fail(E_ARG, "HM_OPT_CHECK_NORM %lld not in {0,1}", (long long)value);
      h->check_norm = (int)value;
      return HM_OK;
  }
  return (hm_status)fail(E_ARG, "unknown option %d", (int)opt);
}

hm_status hm_workspace_size(hm_handle h, hm_op op, int n, hm_dtype dtype, int n_q, int64_t count, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  const int dbl = dtype == HM_C128;
  switch (op) {
    case HM_OP_SRE: {
      if (n_q < 1 || n_q > HM_MAX_Q) return (hm_status)fail(E_ARG, "n_q = %d outside [1, %d]", n_q, HM_MAX_Q);
      SrePlan p;
      HM_TRY(sre_plan(n, dbl, plan_opts(h, n, dbl), &p));
      *bytes = sre_workspace(p, n_q, (int64_t)1 << n);
      return HM_OK;
    }
    case HM_OP_SRE_ROWS: {
      if (n_q < 1 || n_q > HM_MAX_Q) return (hm_status)fail(E_ARG, "n_q = %d outside [1, %d]", n_q, HM_MAX_Q);
      if (count < 0) return (hm_status)fail(E_ARG, "count = %lld < 0", (long long)count);
      SrePlan p;
      HM_TRY(sre_plan(n, dbl, plan_opts(h, n, dbl), &p));
      *bytes = sre_workspace(p, n_q, 0);
      return HM_OK;
    }
    case HM_OP_ROW_VALUES:
      if (n < 1 || n > 26) return (hm_status)fail(E_SIZE, "row values: n = %d outside [1, 26]", n);
      *bytes = sre_row_values_workspace(n, dbl);
      return HM_OK;
    case HM_OP_SRE_GRAD:
      if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
      HM_TRY(sre_grad_workspace(grad_opts(h, n, dbl), n, dbl, bytes));
      return HM_OK;
    case HM_OP_SRE_GRAD_BATCHED:
      if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
      if (count < 1 || count > INT32_MAX) return (hm_status)fail(E_ARG, "gradient: count = %lld outside [1, 2^31)", (long long)count);
      HM_TRY(sre_grad_batched_workspace(grad_opts(h, n, dbl), n, dbl, (int)count, bytes));
      return HM_OK;
    case HM_OP_SRE_SAMPLED: {
      if (count < 2) return (hm_status)fail(E_ARG, "sampled: count = %lld < 2", (long long)count);
      SrePlan p;
      HM_TRY(sre_plan(n, dbl, plan_opts(h, n, dbl), &p));
      *bytes = align256((size_t)(count + 1) * 2 * sizeof(double)) + sre_workspace(p, 1, 0);
      return HM_OK;
    }
    case HM_OP_MANA_MIXED:
      HM_TRY(mixed_workspace(n, dbl, bytes));
      return HM_OK;
    case HM_OP_MANA_QUDIT:
      if (count != 3 && count != 5 && count != 7)
        return (hm_status)fail(E_ARG, "qudit mana: count (d) = %lld is not 3, 5 or 7", (long long)count);
      HM_TRY(qudit_workspace(n, (int)count, dbl, bytes));
      return HM_OK;
    case HM_OP_MANA: {
      if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "mana: n = %d outside [1, 16]", n);
      int64_t mb;
      int ms;
      mana_opts(h, n, dbl, &mb, &ms);
      HM_TRY(mana_workspace(n, dbl, mb, ms, bytes));
      return HM_OK;
    }
  }
  return (hm_status)fail(E_ARG, "unknown op %d", (int)op);
}

hm_status hm_sre(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q, int n_q, double *out, void *ws,
                 size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(out, 8, "out"));
  QArgs qa;
  HM_TRY(check_q(q, n_q, &qa));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  const int64_t n_shifts = (int64_t)1 << n;
  HM_TRY(check_ws(ws, ws_bytes, sre_workspace(p, n_q, n_shifts)));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  return (hm_status)sre_run(p, psi, qa, 0, nullptr, n_shifts, nullptr, nullptr, out, ws, stream);
}

hm_status hm_sre_partial(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q, int n_q, uint64_t a0,
                         uint64_t a1, double *sums, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(sums, 8, "sums"));
  QArgs qa;
  HM_TRY(check_q(q, n_q, &qa));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  const uint64_t D = 1ull << n;
  if (a0 > a1 || a1 > D) return (hm_status)fail(E_ARG, "shift range [%llu, %llu) not inside [0, 2^%d]", (unsigned long long)a0, (unsigned long long)a1, n);
  const int64_t n_slots = (int64_t)(a1 - a0);
  HM_TRY(check_ws(ws, ws_bytes, sre_workspace(p, n_q, n_slots)));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  if (n_slots == 0) return (hm_status)fill_dev(sums, n_q + 1, 0.0, stream);
  return (hm_status)sre_run(p, psi, qa, a0, nullptr, n_slots, nullptr, sums, nullptr, ws, stream);
}

hm_status hm_sre_finalize(int n, const double *q, int n_q, const double *sums, double *out, hipStream_t stream) {
  g_err[0] = 0;
  if (n < 1 || n > 62) return (hm_status)fail(E_SIZE, "n = %d outside [1, 62]", n);
  HM_TRY(check_ptr(sums, 8, "sums"));
  HM_TRY(check_ptr(out, 8, "out"));
  QArgs qa;
  HM_TRY(check_q(q, n_q, &qa));
  return (hm_status)sre_finalize_launch(n, qa, sums, out, stream);
}

hm_status hm_sre_rows(hm_handle h, const void *psi, int n, hm_dtype dtype, const uint64_t *rows, int64_t n_rows,
                      const double *q, int n_q, double *row_sums, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  if (n_rows < 0) return (hm_status)fail(E_ARG, "n_rows = %lld < 0", (long long)n_rows);
  QArgs qa;
  HM_TRY(check_q(q, n_q, &qa));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  if (n_rows == 0) return HM_OK;
  HM_TRY(check_ptr(rows, 8, "rows"));
  HM_TRY(check_ptr(row_sums, 8, "row_sums"));
  HM_TRY(check_ws(ws, ws_bytes, sre_workspace(p, n_q, 0)));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  return (hm_status)sre_run(p, psi, qa, 0, rows, n_rows, row_sums, nullptr, nullptr, ws, stream);
}

hm_status hm_sre_row_values(hm_handle h, const void *psi, int n, hm_dtype dtype, uint64_t a, double *out, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 26) return (hm_status)fail(E_SIZE, "row values: n = %d outside [1, 26]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(out, 8, "out"));
  if (a >> n) return (hm_status)fail(E_ARG, "a = %llu is not an %d-bit X-string", (unsigned long long)a, n);
  HM_TRY(check_ws(ws, ws_bytes, sre_row_values_workspace(n, dtype == HM_C128)));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  return (hm_status)sre_row_values_launch(n, dtype == HM_C128, psi, a, out, ws, stream);
}

hm_status hm_sre_grad(hm_handle h, const void *psi, int n, hm_dtype dtype, double q, double *out, void *grad, void *ws,
                      size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(grad, psi_align(dtype), "grad"));
  HM_TRY(check_ptr(out, 8, "out"));
  if (!(q > 0.0) || !isfinite(q) || q == 1.0) return (hm_status)fail(E_ARG, "gradient: q = %g must be positive, finite and != 1", q);
  const PlanOpts o = grad_opts(h, n, dtype == HM_C128);
  size_t need = 0;
  HM_TRY(sre_grad_workspace(o, n, dtype == HM_C128, &need));
  HM_TRY(check_ws(ws, ws_bytes, need));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  return (hm_status)sre_grad_launch(o, n, dtype == HM_C128, psi, q, out, grad, ws, ws_bytes, stream);
}

hm_status hm_sre_grad_batched(hm_handle h, const void *const *psis, int n, int batch, hm_dtype dtype, double q,
                              double *out, void *const *grads, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
  if (batch < 1) return (hm_status)fail(E_ARG, "gradient: batch = %d < 1", batch);
  if (!psis || !grads) return (hm_status)fail(E_ARG, "psis or grads is NULL");
  for (int s = 0; s < batch; ++s) {
    HM_TRY(check_ptr(psis[s], psi_align(dtype), "psis[s]"));
    HM_TRY(check_ptr(grads[s], psi_align(dtype), "grads[s]"));
  }
  HM_TRY(check_ptr(out, 8, "out"));
  if (!(q > 0.0) || !isfinite(q) || q == 1.0) return (hm_status)fail(E_ARG, "gradient: q = %g must be positive, finite and != 1", q);
  const PlanOpts o = grad_opts(h, n, dtype == HM_C128);
  size_t need = 0;
  HM_TRY(sre_grad_batched_workspace(o, n, dtype == HM_C128, batch, &need));
  HM_TRY(check_ws(ws, ws_bytes, need));
  for (int s = 0; s < batch; ++s) HM_TRY(norm_ok(h, psis[s], 2, n, dtype, stream));
  return (hm_status)sre_grad_batched_launch(o, n, dtype == HM_C128, psis, batch, q, out, grads, ws, ws_bytes, stream);
}

// Runs [i0, i1) of consecutive states with equal n (batches of uneven n: one batched gradient per run).
static void equal_n_runs(const int *ns, int batch, std::vector<std::pair<int, int>> *runs) {
  for (int i0 = 0; i0 < batch;) {
    int i1 = i0 + 1;
    while (i1 < batch && ns[i1] == ns[i0]) ++i1;
    runs->push_back({i0, i1});
    i0 = i1;
  }
}

hm_status hm_sre_batched_grad_workspace(hm_handle h, const int *ns, int batch, hm_dtype dtype, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !ns || !bytes) return (hm_status)fail(E_ARG, "h, ns or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  if (batch < 1) return (hm_status)fail(E_ARG, "gradient: batch = %d < 1", batch);
  std::vector<std::pair<int, int>> runs;
  equal_n_runs(ns, batch, &runs);
  size_t need = 256;
  for (const auto &r : runs) {
    const int n = ns[r.first];
    if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d (state %d) outside [1, 20]", n, r.first);
    size_t b = 0;
    HM_TRY(sre_grad_batched_workspace(grad_opts(h, n, dtype == HM_C128), n, dtype == HM_C128, r.second - r.first, &b));
    if (b > need) need = b;
  }
  *bytes = need;
  return HM_OK;
}

hm_status hm_sre_batched_grad(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype, double q,
                              double *out, void *const *grads, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  if (!psis || !ns || !grads) return (hm_status)fail(E_ARG, "psis, ns or grads is NULL");
  size_t need = 0;
  HM_TRY(hm_sre_batched_grad_workspace(h, ns, batch, dtype, &need));
  for (int s = 0; s < batch; ++s) {
    HM_TRY(check_ptr(psis[s], psi_align(dtype), "psis[s]"));
    HM_TRY(check_ptr(grads[s], psi_align(dtype), "grads[s]"));
  }
  HM_TRY(check_ptr(out, 8, "out"));
  if (!(q > 0.0) || !isfinite(q) || q == 1.0) return (hm_status)fail(E_ARG, "gradient: q = %g must be positive, finite and != 1", q);
  HM_TRY(check_ws(ws, ws_bytes, need));
  for (int s = 0; s < batch; ++s) HM_TRY(norm_ok(h, psis[s], 2, ns[s], dtype, stream));
  std::vector<std::pair<int, int>> runs;
  equal_n_runs(ns, batch, &runs);
  for (const auto &r : runs) {  // the runs share the workspace in stream order
    const int n = ns[r.first];
    HM_TRY(sre_grad_batched_launch(grad_opts(h, n, dtype == HM_C128), n, dtype == HM_C128, psis + r.first,
                                   r.second - r.first, q, out + 2 * (size_t)r.first, grads + r.first, ws, ws_bytes,
                                   stream));
  }
  return HM_OK;
}

// Default launch form of the batched forward (HM_OPT_BATCH_LAUNCH).
static constexpr int BATCH_LAUNCH_DEFAULT = 1;

// Batched calls: states of workgroup-resident size (path 1 under the handle's options, at least
// 2^RB folded values) go to one persistent launch; the rest (tiny states, two-pass sizes) run by
// size class / one after another on the same workspace after it.
static void batched_split(hm_handle h, const int *ns, int batch, int dbl, std::vector<int> *pers,
                          std::vector<int> *rest) {
  const int mode = h->opts.batch_launch ? h->opts.batch_launch
                   : h->tuned_batch_launch ? h->tuned_batch_launch : BATCH_LAUNCH_DEFAULT;
  for (int i = 0; i < batch; ++i) {
    if (mode == 2) {
      rest->push_back(i);
      continue;
    }
    SrePlan p;
    const bool res = sre_plan(ns[i], dbl, plan_opts(h, ns[i], dbl), &p) == OK && p.path == 1;
    (res && batch_resident_ok(ns[i], dbl) ? pers : rest)->push_back(i);
  }
}

static int batched_ws(hm_handle h, const int *ns, int batch, int dbl, int n_q, size_t *bytes) {
  if (!ns || batch < 1) return fail(E_ARG, "batched: ns is NULL or batch = %d < 1", batch);
  size_t need = 256;
  for (int i = 0; i < batch; ++i) {
    SrePlan p;
    int st = sre_plan(ns[i], dbl, plan_opts(h, ns[i], dbl), &p);
    if (st) return st;
  }
  std::vector<int> pers, rest;
  batched_split(h, ns, batch, dbl, &pers, &rest);
  if (!pers.empty()) need = batch_persistent_workspace(ns, pers.data(), (int)pers.size(), n_q, dbl);
  for (int i : rest) {
    SrePlan p;
    sre_plan(ns[i], dbl, plan_opts(h, ns[i], dbl), &p);
    size_t b;
    if (p.path == 1) {
      int cnt = 0;
      for (int j : rest) cnt += ns[j] == ns[i];
      b = sre_states_workspace(p, n_q, cnt < HM_BATCH_PTRS ? cnt : HM_BATCH_PTRS);
    } else {
      b = sre_workspace(p, n_q, (int64_t)1 << ns[i]);
    }
    if (b > need) need = b;
  }
  *bytes = need;
  return OK;
}

hm_status hm_sre_batched_workspace(hm_handle h, const int *ns, int batch, hm_dtype dtype, int n_q, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  if (n_q < 1 || n_q > HM_MAX_Q) return (hm_status)fail(E_ARG, "n_q = %d outside [1, %d]", n_q, HM_MAX_Q);
  return (hm_status)batched_ws(h, ns, batch, dtype == HM_C128, n_q, bytes);
}

hm_status hm_sre_batched(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype,
                         const double *q, int n_q, double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (!psis) return (hm_status)fail(E_ARG, "psis is NULL");
  HM_TRY(check_ptr(out, 8, "out"));
  QArgs qa;
  HM_TRY(check_q(q, n_q, &qa));
  const int dbl = dtype == HM_C128;
  size_t need;
  HM_TRY(batched_ws(h, ns, batch, dbl, n_q, &need));
  for (int i = 0; i < batch; ++i) HM_TRY(check_ptr(psis[i], psi_align(dtype), "psis[i]"));
  HM_TRY(check_ws(ws, ws_bytes, need));
  for (int i = 0; i < batch; ++i) HM_TRY(norm_ok(h, psis[i], 2, ns[i], dtype, stream));
  std::vector<int> pers, rest;
  batched_split(h, ns, batch, dbl, &pers, &rest);
  HM_TRY(batch_persistent_run(dbl, psis, ns, pers.data(), (int)pers.size(), qa, out, ws, stream));
  // the rest: resident size classes up to HM_BATCH_PTRS states per launch, two-pass states one by one
  std::vector<char> done(batch, 0);
  for (int i : rest) {
    if (done[i]) continue;
    SrePlan p;
    HM_TRY(sre_plan(ns[i], dbl, plan_opts(h, ns[i], dbl), &p));
    if (p.path != 1) {
      done[i] = 1;
      HM_TRY(sre_run(p, psis[i], qa, 0, nullptr, (int64_t)1 << ns[i], nullptr, nullptr, out + (size_t)i * (n_q + 1), ws,
                     stream));
      continue;
    }
    std::vector<const void *> ptrs;
    std::vector<double *> outs;
    for (int j : rest) {
      if (done[j] || ns[j] != ns[i]) continue;
      done[j] = 1;
      ptrs.push_back(psis[j]);
      outs.push_back(out + (size_t)j * (n_q + 1));
      if ((int)ptrs.size() == HM_BATCH_PTRS) {
        HM_TRY(sre_run_states(p, ptrs.data(), (int)ptrs.size(), qa, outs.data(), ws, stream));
        ptrs.clear();
        outs.clear();
      }
    }
    if (!ptrs.empty()) HM_TRY(sre_run_states(p, ptrs.data(), (int)ptrs.size(), qa, outs.data(), ws, stream));
  }
  return HM_OK;
}

hm_status hm_sre_sampled(hm_handle h, const void *psi, int n, hm_dtype dtype, const uint64_t *rows, int64_t n_rows,
                         double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(rows, 8, "rows"));
  HM_TRY(check_ptr(out, 8, "out"));
  if (n_rows < 2) return (hm_status)fail(E_ARG, "sampled: n_rows = %lld < 2", (long long)n_rows);
  QArgs qa;
  const double q2 = 2.0;
  HM_TRY(check_q(&q2, 1, &qa));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  const size_t rs_bytes = align256((size_t)(n_rows + 1) * 2 * sizeof(double));
  HM_TRY(check_ws(ws, ws_bytes, rs_bytes + sre_workspace(p, 1, 0)));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  double *rs = (double *)ws;
  double *s0 = rs + 2 * n_rows;  // exact row a = 0
  HM_TRY(sre_run(p, psi, qa, 0, nullptr, 1, s0, nullptr, nullptr, (char *)ws + rs_bytes, stream));
  HM_TRY(sre_run(p, psi, qa, 0, rows, n_rows, rs, nullptr, nullptr, (char *)ws + rs_bytes, stream));
  return (hm_status)sre_sampled_stats(rs, rows, n_rows, 2, s0, n, out, stream);
}

hm_status hm_sre_mc_workspace(hm_handle h, int n, hm_dtype dtype, const hm_mc_params *params, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(mc_check(n, params));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  return (hm_status)mc_workspace(p, params, bytes);
}

hm_status hm_sre_mc(hm_handle h, const void *psi, int n, hm_dtype dtype, const hm_mc_params *params,
                    const uint64_t *a_init, const uint64_t *moves, const double *uniforms, double *out, double *trace,
                    void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(mc_check(n, params));
  HM_TRY(check_ptr(a_init, 8, "a_init"));
  HM_TRY(check_ptr(moves, 8, "moves"));
  HM_TRY(check_ptr(uniforms, 8, "uniforms"));
  HM_TRY(check_ptr(out, 8, "out"));
  HM_TRY(check_ptr(trace, 8, "trace"));
  SrePlan p;
  HM_TRY(sre_plan(n, dtype == HM_C128, plan_opts(h, n, dtype == HM_C128), &p));
  size_t need = 0;
  HM_TRY(mc_workspace(p, params, &need));
  HM_TRY(check_ws(ws, ws_bytes, need));
  HM_TRY(norm_ok(h, psi, 2, n, dtype, stream));
  return (hm_status)mc_run(p, psi, params, a_init, moves, uniforms, out, trace, ws, stream);
}

hm_status hm_autotune_workspace(hm_handle h, int n, hm_dtype dtype, int64_t sample_shifts, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 26) return (hm_status)fail(E_SIZE, "autotune: n = %d outside [1, 26]", n);
  *bytes = sre_autotune_workspace(h, n, dtype == HM_C128, sample_shifts);
  return HM_OK;
}

hm_status hm_autotune(hm_handle h, const void *psi, int n, hm_dtype dtype, int64_t sample_shifts, void *ws,
                      size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 26) return (hm_status)fail(E_SIZE, "autotune: n = %d outside [1, 26]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ws(ws, ws_bytes, 256));
  return (hm_status)sre_autotune(h, psi, n, dtype == HM_C128, sample_shifts, ws, ws_bytes, stream, nullptr);
}

hm_status hm_autotune_mana_workspace(hm_handle h, int n, hm_dtype dtype, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "mana: n = %d outside [1, 16]", n);
  *bytes = mana_autotune_workspace(h, n, dtype == HM_C128);
  return HM_OK;
}

hm_status hm_autotune_mana(hm_handle h, const void *psi, int n, hm_dtype dtype, int64_t sample_shifts, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "mana: n = %d outside [1, 16]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ws(ws, ws_bytes, 256));
  return (hm_status)mana_autotune(h, psi, n, dtype == HM_C128, sample_shifts, ws, ws_bytes, stream);
}

hm_status hm_autotune_grad_workspace(hm_handle h, int n, hm_dtype dtype, size_t *bytes) {
  g_err[0] = 0;
  if (!h || !bytes) return (hm_status)fail(E_ARG, "h or bytes is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
  *bytes = grad_autotune_workspace(h, n, dtype == HM_C128);
  return HM_OK;
}

hm_status hm_autotune_grad(hm_handle h, const void *psi, int n, hm_dtype dtype, double q, double *out, void *grad,
                           void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 20) return (hm_status)fail(E_SIZE, "gradient: n = %d outside [1, 20]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(grad, psi_align(dtype), "grad"));
  HM_TRY(check_ptr(out, 8, "out"));
  if (!(q > 0.0) || !isfinite(q) || q == 1.0) return (hm_status)fail(E_ARG, "gradient: q = %g must be positive, finite and != 1", q);
  HM_TRY(check_ws(ws, ws_bytes, 256));
  return (hm_status)grad_autotune(h, psi, n, dtype == HM_C128, q, out, grad, ws, ws_bytes, stream);
}

hm_status hm_autotune_batched(hm_handle h, const void *const *psis, const int *ns, int batch, hm_dtype dtype,
                              double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (h->opts.batch_launch) return (hm_status)fail(E_ARG, "batched autotune: HM_OPT_BATCH_LAUNCH is fixed on the handle");
  const double q2 = 2.0;
  float best = -1.f;
  int pick = 0;
  for (int mode : {1, 2}) {
    h->opts.batch_launch = mode;
    size_t need = 0;
    hm_status st = hm_sre_batched_workspace(h, ns, batch, dtype, 1, &need);
    if (st == HM_OK && need > ws_bytes) st = HM_E_WORKSPACE;
    float ms = 0.f;
    int err = st;
    if (!err)
      err = time_once_api(stream, [&]() { return (int)hm_sre_batched(h, psis, ns, batch, dtype, &q2, 1, out, ws, ws_bytes, stream); }, &ms);
    h->opts.batch_launch = 0;
    if (err == E_WORKSPACE) continue;
    if (err) return (hm_status)err;
    if (best < 0.f || ms < best) {
      best = ms;
      pick = mode;
    }
  }
  if (!pick) return (hm_status)fail(E_WORKSPACE, "batched autotune: no launch form fits a workspace of %zu bytes", ws_bytes);
  h->tuned_batch_launch = pick;
  return HM_OK;
}

hm_status hm_tune_query(hm_handle h, int n, hm_dtype dtype, int64_t *opts, double *ms_per_shift) {
  g_err[0] = 0;
  if (!h || !opts) return (hm_status)fail(E_ARG, "h or opts is NULL");
  HM_TRY(check_dtype(dtype));
  for (const auto &t : h->tuned)
    if (t.n == n && t.dbl == (dtype == HM_C128)) {
      const PlanOpts &o = t.opts;
      const int64_t v[8] = {o.force_path, o.batch, o.row_rb, o.col_rb, o.row_bits, o.pipeline, o.lds_split, o.streams};
      for (int i = 0; i < 8; ++i) opts[i] = v[i];
      if (ms_per_shift) *ms_per_shift = t.ms_per_shift;
      return HM_OK;
    }
  return (hm_status)fail(E_ARG, "no autotuned plan for n = %d on this handle", n);
}

hm_status hm_tune_clear(hm_handle h) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  h->tuned.clear();
  h->tuned_mana.clear();
  h->tuned_grad.clear();
  h->tuned_batch_launch = 0;
  return HM_OK;
}

hm_status hm_mana(hm_handle h, const void *psi, int n, hm_dtype dtype, double *out, void *ws, size_t ws_bytes,
                  hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "mana: n = %d outside [1, 16]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(out, 8, "out"));
  uint64_t D = 1;
  for (int i = 0; i < n; ++i) D *= 3;
  size_t need = 0;
  int64_t mb;
  int ms;
  mana_opts(h, n, dtype == HM_C128, &mb, &ms);
  HM_TRY(mana_workspace(n, dtype == HM_C128, mb, ms, &need));
  HM_TRY(check_ws(ws, ws_bytes, need));
  HM_TRY(norm_ok(h, psi, 3, n, dtype, stream));
  return (hm_status)mana_launch(n, dtype == HM_C128, mb, ms, psi, 0, D, nullptr, out, ws, ws_bytes, stream);
}

hm_status hm_mana_mixed(hm_handle h, const void *rho, int n, hm_dtype dtype, double *out, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  size_t need = 0;
  HM_TRY(mixed_workspace(n, dtype == HM_C128, &need));
  HM_TRY(check_ptr(rho, psi_align(dtype), "rho"));
  HM_TRY(check_ptr(out, 8, "out"));
  HM_TRY(check_ws(ws, ws_bytes, need));
  return (hm_status)mixed_launch(n, dtype == HM_C128, rho, out, ws, stream);
}

hm_status hm_mana_qudit(hm_handle h, const void *psi, int n, int d, hm_dtype dtype, double *out, void *ws,
                        size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  size_t need = 0;
  HM_TRY(qudit_workspace(n, d, dtype == HM_C128, &need));
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(out, 8, "out"));
  HM_TRY(check_ws(ws, ws_bytes, need));
  return (hm_status)qudit_launch(n, d, dtype == HM_C128, psi, out, ws, stream);
}

hm_status hm_reduced_density(hm_handle h, const void *psi, int n, int n_a, hm_dtype dtype, void *rho,
                             hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "reduced density: n = %d outside [1, 16]", n);
  if (n_a < 1 || n_a > n || n_a > 10) return (hm_status)fail(E_SIZE, "reduced density: n_a = %d outside [1, min(n, 10)]", n_a);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(rho, psi_align(dtype), "rho"));
  return (hm_status)reduced_density_launch(n, n_a, dtype == HM_C128, psi, rho, stream);
}

hm_status hm_mana_partial(hm_handle h, const void *psi, int n, hm_dtype dtype, uint64_t a0, uint64_t a1, double *sums,
                          void *ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  HM_TRY(check_dtype(dtype));
  if (n < 1 || n > 16) return (hm_status)fail(E_SIZE, "mana: n = %d outside [1, 16]", n);
  HM_TRY(check_ptr(psi, psi_align(dtype), "psi"));
  HM_TRY(check_ptr(sums, 8, "sums"));
  uint64_t D = 1;
  for (int i = 0; i < n; ++i) D *= 3;
  if (a0 > a1 || a1 > D) return (hm_status)fail(E_ARG, "shift range [%llu, %llu) not inside [0, 3^%d]", (unsigned long long)a0, (unsigned long long)a1, n);
  size_t need = 0;
  int64_t mb;
  int ms;
  mana_opts(h, n, dtype == HM_C128, &mb, &ms);
  HM_TRY(mana_workspace(n, dtype == HM_C128, mb, ms, &need));
  HM_TRY(check_ws(ws, ws_bytes, need));
  HM_TRY(norm_ok(h, psi, 3, n, dtype, stream));
  if (a1 == a0) return (hm_status)fill_dev(sums, 3, 0.0, stream);
  return (hm_status)mana_launch(n, dtype == HM_C128, mb, ms, psi, a0, a1, sums, nullptr, ws, ws_bytes, stream);
}

}  // extern "C"
