// swe_batch_cmp.hip - batched stage kernels of every tile variant with
// the compensated level (see SWE_BK_M in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_CMP(TX, TY, R, W) SWE_BK_M(TX, TY, R, W, false, true)
const BatchKernels g_bk_cmp[] = {SWE_TILE_LIST(SWE_BK_CMP)};

}  // namespace swe
