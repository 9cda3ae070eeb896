// swe_batch_llf_cmp.hip - batched stage kernels of every tile variant with
// local Lax-Friedrichs splitting and the compensated level (see SWE_BK_L in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_LLFCMP(TX, TY, R, W) SWE_BK_L(TX, TY, R, W, false, true, true)
const BatchKernels g_bk_llf_cmp[] = {SWE_TILE_LIST(SWE_BK_LLFCMP)};

}  // namespace swe
