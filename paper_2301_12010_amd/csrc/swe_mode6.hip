// swe_mode6.hip - stage kernels of every tile variant with local Lax-Friedrichs splitting and point-implicit friction
// (mode 6 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE6_SET(TX, TY, R, W) SWE_STAGE_SET_L(TX, TY, R, W, false, true, true)
const StageSet g_stage_mode6[] = {SWE_TILE_LIST(SWE_MODE6_SET)};

}  // namespace swe
