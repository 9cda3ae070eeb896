// swe_batch_imp.hip - batched stage kernels of every tile variant with
// point-implicit friction (see SWE_BK in swe_batch_kernels.hpp).
#include <hip/hip_runtime.h>

#include "swe_batch_kernels.hpp"

namespace swe {

#define SWE_BK_IMPLICIT(TX, TY, R, W) SWE_BK(TX, TY, R, W, true)
const BatchKernels g_bk_imp[] = {SWE_TILE_LIST(SWE_BK_IMPLICIT)};

}  // namespace swe
