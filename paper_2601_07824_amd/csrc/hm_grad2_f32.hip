// hm_grad2_f32.hip -- float instantiation of the two-pass SRE gradient (see hm_grad2_kern.h).
#include "hm_grad2_kern.h"

namespace hm {

int sre_grad2_f32(const SrePlan &p, const void *psi, double q, double *out, void *grad, void *ws, hipStream_t st) {
  return grad2_t<float>(p, psi, q, out, grad, (char *)ws, st);
}

size_t sre_grad2_workspace_f32(const SrePlan &p) { return grad2_workspace(p); }

}  // namespace hm
