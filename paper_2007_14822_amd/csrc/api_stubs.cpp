// Entry points not yet implemented in this build.
#include "handle.h"

using namespace itn;

extern "C" {

void itn_release_solver(itn_handle*) {}

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
itn_status itn_mpo_create(itn_handle* h, int32_t, int32_t, int32_t, const double*, itn_mpo** m) {
  if (m) *m = nullptr;
  return fail(h, ITN_E_UNSUPPORTED, "sweeps are not built yet");
}
itn_status itn_mpo_destroy(itn_mpo*) { return ITN_OK; }
itn_status itn_mps_create(itn_handle* h, int32_t, int32_t, const int32_t*, const double*, itn_mps** m) {
  if (m) *m = nullptr;
  return fail(h, ITN_E_UNSUPPORTED, "sweeps are not built yet");
}
itn_status itn_mps_destroy(itn_mps*) { return ITN_OK; }
itn_status itn_mps_bonds(const itn_mps*, int32_t*) { return ITN_E_UNSUPPORTED; }
itn_status itn_mps_get_site(itn_handle*, const itn_mps*, int32_t, double*) { return ITN_E_UNSUPPORTED; }
itn_status itn_dmrg_sweep(itn_handle* h, itn_mps*, const itn_mpo*, const itn_sweep_params*,
                          itn_sweep_result*) {
  return fail(h, ITN_E_UNSUPPORTED, "sweeps are not built yet");
}

}  // extern "C"
