// swe_batch_llf.hip - batched stage kernels of every tile variant with
// local Lax-Friedrichs splitting (see SWE_BK_L in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_LLF(TX, TY, R, W) SWE_BK_L(TX, TY, R, W, false, false, true)
const BatchKernels g_bk_llf[] = {SWE_TILE_LIST(SWE_BK_LLF)};

}  // namespace swe
