// swe_mode4.hip - stage kernels of every tile variant with local Lax-Friedrichs splitting
// (mode 4 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE4_SET(TX, TY, R, W) SWE_STAGE_SET_L(TX, TY, R, W, false, false, true)
const StageSet g_stage_mode4[] = {SWE_TILE_LIST(SWE_MODE4_SET)};

}  // namespace swe
