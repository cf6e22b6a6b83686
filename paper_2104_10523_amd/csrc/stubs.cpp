// Entry points whose implementation is not built yet.
#include "common.hpp"

using namespace tn;

extern "C" {
tn_status tn_mps_create(int32_t, int32_t, void*, tn_mps**) { set_last_error("MPS not built"); return TN_ERR_UNSUPPORTED; }
tn_status tn_mps_destroy(tn_mps*) { return TN_OK; }
tn_status tn_mps_apply_gate1(tn_mps*, int32_t, const double*, void*) { return TN_ERR_UNSUPPORTED; }
tn_status tn_mps_apply_gate(tn_mps*, int32_t, const double*, int32_t, double, double*, void*) { return TN_ERR_UNSUPPORTED; }
tn_status tn_mps_bond_dims(const tn_mps*, int32_t*) { return TN_ERR_UNSUPPORTED; }
tn_status tn_mps_expect_z(tn_mps*, double*, void*) { return TN_ERR_UNSUPPORTED; }
tn_status tn_mps_amplitudes(tn_mps*, const int8_t*, int64_t, double*, void*) { return TN_ERR_UNSUPPORTED; }
tn_status tn_run_trajectories(const tn_circuit* const*, int32_t, int32_t, const double*, int64_t, double*, tn_report*, void*) { return TN_ERR_UNSUPPORTED; }
}
