// swe_mode7.hip - stage kernels of every tile variant with local Lax-Friedrichs splitting, point-implicit friction and the compensated level
// (mode 7 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE7_SET(TX, TY, R, W) SWE_STAGE_SET_L(TX, TY, R, W, true, true, true)
const StageSet g_stage_mode7[] = {SWE_TILE_LIST(SWE_MODE7_SET)};

}  // namespace swe
