// Mixed-precision M2L (FP32 below the root levels) -- not built yet.
#include "fmm_device.h"

namespace fmm {

bool mixed_supported(int) { return false; }

void launch_m2l_mixed(Ctx&) { throw hip_error{hipErrorNotSupported, "mixed-precision M2L"}; }

}  // namespace fmm
