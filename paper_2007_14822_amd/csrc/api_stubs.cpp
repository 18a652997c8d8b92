// Entry points not yet implemented in this build.
#include "handle.h"

using namespace itn;

extern "C" {

itn_status itn_qn_heff_plan(itn_handle* h, const itn_tensor*, const itn_tensor*, const itn_tensor*,
                            const itn_tensor*, const itn_tensor*, int32_t, itn_prec, itn_plan** p) {
  if (p) *p = nullptr;
  return fail(h, ITN_E_UNSUPPORTED, "QN H_eff is not built yet");
}
itn_status itn_plan_destroy(itn_plan*) { return ITN_OK; }
itn_status itn_plan_query(const itn_plan*, itn_plan_info*) { return ITN_E_UNSUPPORTED; }
itn_status itn_plan_out_blocks(const itn_plan*, int32_t*, int64_t*) { return ITN_E_UNSUPPORTED; }
itn_status itn_qn_heff_apply(itn_handle* h, itn_plan*, const itn_tensor*, const itn_tensor*,
                             const itn_tensor*, itn_tensor*, void*) {
  return fail(h, ITN_E_UNSUPPORTED, "QN H_eff is not built yet");
}
}  // extern "C"
