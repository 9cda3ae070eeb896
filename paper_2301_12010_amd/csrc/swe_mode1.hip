// swe_mode1.hip - stage kernels of every tile variant with the compensated level
// (mode 1 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE1_SET(TX, TY, R, W) SWE_STAGE_SET(TX, TY, R, W, true, false)
const StageSet g_stage_mode1[] = {SWE_TILE_LIST(SWE_MODE1_SET)};

}  // namespace swe
