// hm_stubs.hip -- entry points whose kernels are not in this build yet.
#include <hip/hip_runtime.h>

#include "hm_internal.h"

namespace hm {

size_t sre_grad_workspace(int, int) { return 256; }
int sre_grad_launch(int, int, const void *, double, double *, void *, void *, size_t, hipStream_t) {
  return fail(E_UNSUPPORTED, "hm_sre_grad is not implemented in this build");
}
size_t mana_workspace(int, int, uint64_t) { return 256; }
int mana_launch(int, int, const void *, uint64_t, uint64_t, double *, double *, void *, size_t, hipStream_t) {
  return fail(E_UNSUPPORTED, "hm_mana is not implemented in this build");
}

}  // namespace hm
