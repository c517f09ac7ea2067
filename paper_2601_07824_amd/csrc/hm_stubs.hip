// hm_stubs.hip -- entry points whose kernels are not in this build yet.
#include <hip/hip_runtime.h>

#include "hm_internal.h"

namespace hm {


}  // namespace hm
