// hm_tune.hip -- on-device autotuner for the launch plans.
//
// The two-pass kernels have several free choices (X-shifts per launch, LDS staging, sequential or
// pipelined launches, the row/column split of the folded index bits), and which one is fastest
// depends on n, the dtype and the memory level the exchange lands in.  The tuner times each
// candidate plan on the caller's state over a prefix of the X-shifts (hipEvents on the caller's
// stream), keeps the fastest in the handle, and planning on that handle then fills every option
// the caller left automatic from that entry.  The same is done for the mana plan (X-shifts per
// launch pair, one or two streams), the gradient (workgroup-resident or two-pass kernels where
// both exist) and the batched forward (one persistent launch or one launch per size class).
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

PlanOpts plan_opts(const hm_context *h, int n, int dbl) {
  PlanOpts o = h->opts;
  for (const auto &t : h->tuned) {
    if (t.n != n || t.dbl != dbl) continue;
    if (!o.force_path) o.force_path = t.opts.force_path;
    if (!o.batch) o.batch = t.opts.batch;
    if (!o.row_rb) o.row_rb = t.opts.row_rb;
    if (!o.col_rb) o.col_rb = t.opts.col_rb;
    if (!o.row_bits) o.row_bits = t.opts.row_bits;
    if (!o.pipeline) o.pipeline = t.opts.pipeline;
    if (!o.lds_split) o.lds_split = t.opts.lds_split;
    if (!o.streams) o.streams = t.opts.streams;
    break;
  }
  return o;
}

void mana_opts(const hm_context *h, int n, int dbl, int64_t *batch, int *streams) {
  *batch = h->opts.batch;
  *streams = h->opts.streams;
  for (const auto &t : h->tuned_mana)
    if (t.n == n && t.dbl == dbl) {
      if (!*batch) *batch = t.batch;
      if (!*streams) *streams = t.streams;
      break;
    }
}

PlanOpts grad_opts(const hm_context *h, int n, int dbl) {
  PlanOpts o = h->opts;
  if (!o.force_path)
    for (const auto &t : h->tuned_grad)
      if (t.n == n && t.dbl == dbl) {
        o.force_path = t.path;
        break;
      }
  return o;
}

// Times fn() once after a warm-up call, on stream st (milliseconds).
template <typename F>
static int time_once(hipStream_t st, F fn, float *ms) {
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

// ---- mana ----------------------------------------------------------------------------------------
// Candidates: exchange of 128, 192 or 256 MiB per launch pair on one or two streams (one plan for
// the workgroup-resident sizes).  Options fixed on the handle are kept.
static std::vector<std::pair<int64_t, int>> mana_candidates(const hm_context *h, int n, int dbl) {
  std::vector<std::pair<int64_t, int>> c;
  uint64_t D = 1;
  for (int i = 0; i < n; ++i) D *= 3;
  const size_t per_pair = (size_t)D * (dbl ? 16 : 8);
  for (int mib : {128, 192, 256})
    for (int streams : {1, 2}) {
      int64_t b = h->opts.batch ? h->opts.batch : 2 * (int64_t)(((size_t)mib << 20) / per_pair);
      if (b < 2) b = 2;
      const int sm = h->opts.streams ? h->opts.streams : streams;
      bool dup = false;
      for (auto &e : c) dup |= e.first == b && e.second == sm;
      size_t bytes;
      if (!dup && mana_workspace(n, dbl, b, sm, &bytes) == OK) c.push_back({b, sm});
    }
  return c;
}

size_t mana_autotune_workspace(const hm_context *h, int n, int dbl) {
  size_t need = 256, b;
  for (auto &c : mana_candidates(h, n, dbl))
    if (mana_workspace(n, dbl, c.first, c.second, &b) == OK && b > need) need = b;
  return need;
}

int mana_autotune(hm_context *h, const void *psi, int n, int dbl, int64_t sample, void *ws, size_t ws_bytes,
                  hipStream_t st) {
  uint64_t D = 1;
  for (int i = 0; i < n; ++i) D *= 3;
  uint64_t k = sample > 0 ? (uint64_t)sample : 4096;
  if (k > D) k = D;
  TunedMana best{};
  best.ms_per_shift = -1.0;
  int tried = 0;
  for (auto &c : mana_candidates(h, n, dbl)) {
    size_t b;
    if (mana_workspace(n, dbl, c.first, c.second, &b) != OK || b > ws_bytes) continue;
    float ms = 0.f;
    int err = time_once(st, [&]() { return mana_launch(n, dbl, c.first, c.second, psi, 0, k, nullptr, nullptr, ws, ws_bytes, st); }, &ms);
    if (err) return err;
    ++tried;
    const double per = (double)ms / (double)k;
    if (best.ms_per_shift < 0 || per < best.ms_per_shift) best = TunedMana{n, dbl, c.first, c.second, per};
  }
  if (!tried) return fail(E_WORKSPACE, "mana autotune: no candidate plan fits a workspace of %zu bytes", ws_bytes);
  for (auto it = h->tuned_mana.begin(); it != h->tuned_mana.end(); ++it)
    if (it->n == n && it->dbl == dbl) {
      h->tuned_mana.erase(it);
      break;
    }
  h->tuned_mana.push_back(best);
  return OK;
}

// ---- gradient -------------------------------------------------------------------------------------
size_t grad_autotune_workspace(const hm_context *h, int n, int dbl) {
  size_t need = 256;
  for (int path : {1, 2}) {
    PlanOpts o = h->opts;
    if (!o.force_path) o.force_path = path;
    size_t b;
    if (sre_grad_workspace(o, n, dbl, &b) == OK && b > need) need = b;
  }
  return need;
}

int grad_autotune(hm_context *h, const void *psi, int n, int dbl, double q, void *out, void *grad, void *ws,
                  size_t ws_bytes, hipStream_t st) {
  TunedGrad best{n, dbl, 0, -1.0};
  int tried = 0;
  for (int path : {1, 2}) {
    PlanOpts o = h->opts;
    if (o.force_path && o.force_path != path) continue;
    o.force_path = path;
    size_t b;
    if (sre_grad_workspace(o, n, dbl, &b) != OK || b > ws_bytes) continue;
    float ms = 0.f;
    int err = time_once(st, [&]() { return sre_grad_launch(o, n, dbl, psi, q, (double *)out, grad, ws, ws_bytes, st); }, &ms);
    if (err == E_UNSUPPORTED || err == E_SIZE) continue;  // no kernels of this path for n
    if (err) return err;
    ++tried;
    if (best.ms < 0 || ms < best.ms) best = TunedGrad{n, dbl, path, ms};
  }
  if (!tried) return fail(E_WORKSPACE, "gradient autotune: no path fits a workspace of %zu bytes", ws_bytes);
  for (auto it = h->tuned_grad.begin(); it != h->tuned_grad.end(); ++it)
    if (it->n == n && it->dbl == dbl) {
      h->tuned_grad.erase(it);
      break;
    }
  h->tuned_grad.push_back(best);
  return OK;
}

// Candidate plans for (n, dbl): the workgroup-resident kernel when it applies, and two-pass plans
// over exchange batches of 64/128/256 MiB x LDS staging x {sequential with the default split or
// 11, 12 or 13 row bits, pipelined}.  Options the caller fixed on the handle are kept.
static std::vector<PlanOpts> candidates(const hm_context *h, int n, int dbl) {
  std::vector<PlanOpts> c;
  auto add = [&](PlanOpts o) {
    // the caller's explicit choices win
    const PlanOpts &u = h->opts;
    if (u.force_path) o.force_path = u.force_path;
    if (u.batch) o.batch = u.batch;
    if (u.row_rb) o.row_rb = u.row_rb;
    if (u.col_rb) o.col_rb = u.col_rb;
    if (u.row_bits) o.row_bits = u.row_bits;
    if (u.pipeline) o.pipeline = u.pipeline;
    if (u.lds_split) o.lds_split = u.lds_split;
    if (u.streams) o.streams = u.streams;
    SrePlan p;
    if (sre_plan(n, dbl, o, &p) != OK) return;
    for (const auto &e : c)
      if (!memcmp(&e, &o, sizeof(o))) return;
    c.push_back(o);
  };
  PlanOpts r{};
  r.force_path = 1;
  r.lds_split = 2;  // resident tiles with split staging and a higher occupancy budget
  add(r);
  r.lds_split = 1;
  add(r);
  const int nf = n - 1;
  const size_t per_shift = ((size_t)1 << nf) * (dbl ? 16 : 8);
  int64_t last_b = -1;
  for (int mib : {64, 128, 256}) {
    int64_t b = (int64_t)(((size_t)mib << 20) / per_shift);
    if (b < 1) b = 1;
    if (b > ((int64_t)1 << n)) b = (int64_t)1 << n;
    if (b == last_b) continue;
    last_b = b;
    for (int split : {1, 2})
      for (int v = 0; v < 7; ++v) {
        if (v >= 5 && (dbl || nf < 19)) continue;  // long FP32 rows only where the rows are long
        PlanOpts o{};
        o.force_path = 2;
        o.batch = b;
        o.lds_split = split;
        o.pipeline = v == 4 ? 2 : 1;
        o.row_bits = v == 1 ? 12 : v == 2 ? 11 : v == 3 ? 13 : v == 5 ? 14 : v == 6 ? 15 : 0;
        o.streams = 1;
        add(o);
        if (v != 4) {  // the same on two streams
          o.streams = 2;
          add(o);
        }
      }
  }
  return c;
}

static int64_t tune_shifts(int n, int64_t sample) {
  const int64_t all = (int64_t)1 << n;
  if (sample <= 0) sample = 16384;
  return sample < all ? sample : all;
}

size_t sre_autotune_workspace(const hm_context *h, int n, int dbl, int64_t sample) {
  const int64_t k = tune_shifts(n, sample);
  size_t need = 256;
  for (const auto &o : candidates(h, n, dbl)) {
    SrePlan p;
    if (sre_plan(n, dbl, o, &p) != OK) continue;
    const size_t b = sre_workspace(p, 1, k);
    if (b > need) need = b;
  }
  return need;
}

int sre_autotune(hm_context *h, const void *psi, int n, int dbl, int64_t sample, void *ws, size_t ws_bytes,
                 hipStream_t st, TunedPlan *best_out) {
  const int64_t k = tune_shifts(n, sample);
  QArgs qa{};
  qa.nq = 1;
  qa.q[0] = 2.0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(E_HIP, "autotune: hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(E_HIP, "autotune: hipEventCreate failed");
  }
  TunedPlan best{};
  best.ms_per_shift = -1.0;
  int err = OK, tried = 0;
  for (const auto &o : candidates(h, n, dbl)) {
    SrePlan p;
    if (sre_plan(n, dbl, o, &p) != OK) continue;
    if (sre_workspace(p, 1, k) > ws_bytes) continue;
    // warm-up run, then one timed run over the same k shifts
    if ((err = sre_run(p, psi, qa, 0, nullptr, k, nullptr, nullptr, nullptr, ws, st)) != OK) break;
    if (hipEventRecord(e0, st) != hipSuccess) { err = fail(E_HIP, "autotune: hipEventRecord failed"); break; }
    if ((err = sre_run(p, psi, qa, 0, nullptr, k, nullptr, nullptr, nullptr, ws, st)) != OK) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      err = fail(E_HIP, "autotune: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = (double)ms / (double)k;
    ++tried;
    if (best.ms_per_shift < 0 || per < best.ms_per_shift) {
      best.n = n;
      best.dbl = dbl;
      best.opts = o;
      best.ms_per_shift = per;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err) return err;
  if (!tried) return fail(E_WORKSPACE, "autotune: no candidate plan fits a workspace of %zu bytes", ws_bytes);
  for (auto it = h->tuned.begin(); it != h->tuned.end(); ++it)
    if (it->n == n && it->dbl == dbl) {
      h->tuned.erase(it);
      break;
    }
  h->tuned.push_back(best);
  if (best_out) *best_out = best;
  return OK;
}

}  // namespace hm
