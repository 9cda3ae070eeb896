// swe_mode3.hip - stage kernels of every tile variant with the compensated level and point-implicit friction
// (mode 3 of a context; see StageSet in swe_internal.hpp).
#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

#define SWE_MODE3_SET(TX, TY, R, W) SWE_STAGE_SET(TX, TY, R, W, true, true)
const StageSet g_stage_mode3[] = {SWE_TILE_LIST(SWE_MODE3_SET)};

}  // namespace swe
