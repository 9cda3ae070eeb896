// swe_mode5.hip - stage kernels of every tile variant with local Lax-Friedrichs splitting and the compensated level
// (mode 5 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE5_SET(TX, TY, R, W) SWE_STAGE_SET_L(TX, TY, R, W, true, false, true)
const StageSet g_stage_mode5[] = {SWE_TILE_LIST(SWE_MODE5_SET)};

}  // namespace swe
