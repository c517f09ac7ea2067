// hm_sre_f32.hip -- float instantiation of the qubit SRE kernels (see hm_sre_kern.h).
#include "hm_sre_kern.h"

namespace hm {

int sre_shift_sums_f32(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                       int64_t n_slots, double *shift_sums, char *w, hipStream_t st) {
  return shift_sums_t<float>(p, psi, qa, a0, rows, n_slots, shift_sums, w, st);
}

int sre_states_f32(const SrePlan &p, const void *const *psis, int n_states, const QArgs &qa, double *shift_sums,
                   hipStream_t st) {
  return states_t<float>(p, psis, n_states, qa, shift_sums, st);
}

}  // namespace hm
