// swe_batch_llf_cmp_imp.hip - batched stage kernels of every tile variant with
// local Lax-Friedrichs splitting, the compensated level and
// point-implicit friction (see SWE_BK_L in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_LLFCMPIMP(TX, TY, R, W) SWE_BK_L(TX, TY, R, W, true, true, true)
const BatchKernels g_bk_llf_cmp_imp[] = {SWE_TILE_LIST(SWE_BK_LLFCMPIMP)};

}  // namespace swe
