// Fused first stage of the dense H_eff (placeholder until the fused kernel lands).
#include "kernels.h"

namespace itn {
bool heff_fused_supported(int, int, int) { return false; }
hipError_t heff_stage1_fused(int, const HeffFusedArgs&, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace itn
