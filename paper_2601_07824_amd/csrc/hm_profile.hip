// hm_profile.hip -- optional per-kernel-family timing with HIP events on the launch stream.
//
// When enabled (hm_profile_enable(k), k > 0), every k-th kernel launch of each kernel family is
// bracketed by two hipEventRecord calls on the stream it is enqueued on; hm_profile_query()
// synchronises on the recorded events and reports, per family, the number of timed launches and
// their summed event-to-event device time.  Disabled by default; costs nothing when disabled.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/hmag.h"
#include "hm_internal.h"

namespace hm {

struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};

static std::mutex g_mu;
static bool g_on = false;
static int64_t g_every = 1;
struct ProfSeen {
  std::string name;
  int64_t seen;
};
static std::vector<ProfSeen> g_seen;  // launches seen per family since the last reset
static std::vector<ProfRec> g_open;  // recorded, not yet harvested
struct ProfTot {
  std::string name;
  int64_t count;
  double ms;
};
static std::vector<ProfTot> g_tot;

bool prof_on() { return g_on; }

void *prof_begin(const char *name, hipStream_t st) {
  if (!g_on) return nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    ProfSeen *f = nullptr;
    for (auto &s : g_seen)
      if (s.name == name) f = &s;
    if (!f) {
      g_seen.push_back(ProfSeen{name, 0});
      f = &g_seen.back();
    }
    if (f->seen++ % g_every != 0) return nullptr;
  }
  ProfRec *r = new ProfRec{name, nullptr, nullptr};
  if (hipEventCreate(&r->a) != hipSuccess || hipEventCreate(&r->b) != hipSuccess) {
    delete r;
    return nullptr;
  }
  (void)hipEventRecord(r->a, st);
  return r;
}

void prof_end(void *tok, hipStream_t st) {
  if (!tok) return;
  ProfRec *r = (ProfRec *)tok;
  (void)hipEventRecord(r->b, st);
  std::lock_guard<std::mutex> g(g_mu);
  g_open.push_back(*r);
  delete r;
}

static void harvest() {
  for (auto &r : g_open) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.b);
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
    bool found = false;
    for (auto &t : g_tot)
      if (t.name == r.name) {
        t.count++;
        t.ms += ms;
        found = true;
        break;
      }
    if (!found) g_tot.push_back(ProfTot{r.name, 1, (double)ms});
  }
  g_open.clear();
}

}  // namespace hm

extern "C" {

hm_status hm_profile_enable(int every) {
  std::lock_guard<std::mutex> g(hm::g_mu);
  if (every < 0) return (hm_status)hm::fail(hm::E_ARG, "profile sampling interval %d < 0", every);
  hm::g_on = every > 0;
  hm::g_every = every > 0 ? every : 1;
  return HM_OK;
}

hm_status hm_profile_reset(void) {
  std::lock_guard<std::mutex> g(hm::g_mu);
  hm::harvest();
  hm::g_tot.clear();
  hm::g_seen.clear();
  return HM_OK;
}

hm_status hm_profile_query(int index, char *name, size_t name_len, int64_t *launches, int64_t *timed, double *ms) {
  std::lock_guard<std::mutex> g(hm::g_mu);
  hm::harvest();
  if (index < 0 || index >= (int)hm::g_seen.size())
    return (hm_status)hm::fail(hm::E_ARG, "profile index %d out of range", index);
  const auto &f = hm::g_seen[index];
  int64_t c = 0;
  double t = 0.0;
  for (const auto &r : hm::g_tot)
    if (r.name == f.name) {
      c = r.count;
      t = r.ms;
    }
  if (name && name_len) {
    strncpy(name, f.name.c_str(), name_len - 1);
    name[name_len - 1] = 0;
  }
  if (launches) *launches = f.seen;
  if (timed) *timed = c;
  if (ms) *ms = t;
  return HM_OK;
}

}  // extern "C"
