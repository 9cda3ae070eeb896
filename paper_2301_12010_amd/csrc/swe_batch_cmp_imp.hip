// swe_batch_cmp_imp.hip - batched stage kernels of every tile variant with
// the compensated level and point-implicit friction (see SWE_BK_M in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_CMPIMP(TX, TY, R, W) SWE_BK_M(TX, TY, R, W, true, true)
const BatchKernels g_bk_cmp_imp[] = {SWE_TILE_LIST(SWE_BK_CMPIMP)};

}  // namespace swe
