// swe_mode2.hip - stage kernels of every tile variant with point-implicit friction
// (mode 2 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE2_SET(TX, TY, R, W) SWE_STAGE_SET(TX, TY, R, W, false, true)
const StageSet g_stage_mode2[] = {SWE_TILE_LIST(SWE_MODE2_SET)};

}  // namespace swe
