// hm_noalloc.hip -- hm_sre_noalloc: the exact SRE of hm_sre for callers that cannot allocate device
// memory (code under stream capture, tight serving loops).  The per-shift sums that hm_sre keeps in
// the caller's workspace live here in one file-scope device array per GPU instead, so the call
// allocates nothing; it runs the same kernels (workgroup-resident path, one workgroup per X-shift)
// and the same fixed-order reduction, so its results equal hm_sre's bit for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/hmag.h"
#include "hm_internal.h"
#include "hm_tile.h"

// Per-shift sums of up to 2^16 X-shifts with HM_MAX_Q + 1 slots each: HM_SRE_NOALLOC_MAX_BYTES
// (4.5 MiB) per GPU, held until the process ends.
static __device__ __align__(256) double scratch[HM_SRE_NOALLOC_MAX_BYTES / sizeof(double)];
static_assert(HM_SRE_NOALLOC_MAX_BYTES == ((size_t)1 << 16) * (HM_MAX_Q + 1) * sizeof(double), "scratch size");

namespace hm {

static constexpr int NOALLOC_MAX_DEV = 64;

// Device address of `scratch` on the current device.  The array's name in host code is only a
// host-side handle; the address comes from hipGetSymbolAddress, once per device, with the device
// current.
static int scratch_ptr(void **ptr) {
  static std::mutex mu;
  static void *addr[NOALLOC_MAX_DEV] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEV)
    return fail(E_HIP, "sre_noalloc: no current device (or device index >= %d)", NOALLOC_MAX_DEV);
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(E_HIP, "sre_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return OK;
}

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_sre_noalloc(hm_handle h, const void *psi, int n, hm_dtype dtype, const double *q, int n_q,
                                    double *out, hipStream_t stream) {
  if (!h) return (hm_status)fail(E_ARG, "h is NULL");
  if (dtype != HM_C64 && dtype != HM_C128)
    return (hm_status)fail(E_DTYPE, "dtype %d is neither HM_C64 nor HM_C128", (int)dtype);
  const size_t align = dtype == HM_C128 ? 16 : 8;
  if (!psi) return (hm_status)fail(E_ARG, "psi is NULL");
  if ((uintptr_t)psi % align) return (hm_status)fail(E_ALIGN, "psi = %p is not %zu-byte aligned", psi, align);
  if (!out) return (hm_status)fail(E_ARG, "out is NULL");
  if ((uintptr_t)out % 8) return (hm_status)fail(E_ALIGN, "out = %p is not 8-byte aligned", (const void *)out);
  if (!q) return (hm_status)fail(E_ARG, "q is NULL");
  if (n_q < 1 || n_q > HM_MAX_Q) return (hm_status)fail(E_ARG, "n_q = %d outside [1, %d]", n_q, HM_MAX_Q);
  QArgs qa;
  memset(&qa, 0, sizeof(qa));
  qa.nq = n_q;
  for (int i = 0; i < n_q; ++i) {
    if (!(q[i] > 0.0) || !isfinite(q[i])) return (hm_status)fail(E_ARG, "q[%d] = %g must be positive and finite", i, q[i]);
    qa.q[i] = q[i];
  }
  if (h->check_norm)
    return (hm_status)fail(E_UNSUPPORTED, "sre_noalloc: HM_OPT_CHECK_NORM allocates its scalars; unset it for this call");
  const int dbl = dtype == HM_C128;
  SrePlan p;
  int st = sre_plan(n, dbl, plan_opts(h, n, dbl), &p);
  if (st) return (hm_status)st;
  if (p.path != 1)
    return (hm_status)fail(E_SIZE, "sre_noalloc: n = %d needs the two-pass kernels and their exchange buffer; "
                                   "the no-allocation call covers the workgroup-resident sizes (n <= %d for "
                                   "HM_C64, %d for HM_C128)", n, 16, 15);
  const int64_t n_shifts = (int64_t)1 << n;
  const size_t need = sre_workspace(p, n_q, n_shifts);
  if (need > sizeof(scratch))
    return (hm_status)fail(E_SIZE, "sre_noalloc: %zu bytes of per-shift sums exceed the %zu-byte scratch", need,
                           sizeof(scratch));
  void *ws = nullptr;
  if ((st = scratch_ptr(&ws))) return (hm_status)st;
  return (hm_status)sre_run(p, psi, qa, 0, nullptr, n_shifts, nullptr, nullptr, out, ws, stream);
}
