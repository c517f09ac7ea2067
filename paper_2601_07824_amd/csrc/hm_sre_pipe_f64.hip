// hm_sre_pipe_f64.hip -- double instantiation of the pipelined two-pass SRE kernels (see hm_sre_kern.h).
#include "hm_sre_kern.h"

namespace hm {

int sre_pipe_f64(const SrePlan &p, const void *psi, const QArgs &qa, uint64_t a0, const uint64_t *rows,
                 int64_t n_slots, double *shift_sums, char *w, hipStream_t st) {
  return pipe_shift_sums_t<double>(p, psi, qa, a0, rows, n_slots, shift_sums, w, st);
}

}  // namespace hm
