// Learned warm start (placeholder until the MLP kernels land).
#include "operator.h"

extern "C" {
isvd_status isvd_ws_features(isvd_operator*, float*, void*) { return ISVD_E_UNSUPPORTED; }
isvd_status isvd_ws_create(int, uint64_t, isvd_warmstart**) { return ISVD_E_UNSUPPORTED; }
void isvd_ws_destroy(isvd_warmstart*) {}
int64_t isvd_ws_num_params(const isvd_warmstart*) { return 0; }
isvd_status isvd_ws_get_params(const isvd_warmstart*, float*) { return ISVD_E_UNSUPPORTED; }
isvd_status isvd_ws_set_params(isvd_warmstart*, const float*) { return ISVD_E_UNSUPPORTED; }
isvd_status isvd_ws_forward(isvd_warmstart*, int64_t, const float*, float*, int64_t, void*) { return ISVD_E_UNSUPPORTED; }
isvd_status isvd_ws_train_step(isvd_warmstart*, int64_t, const float*, const float*, int64_t, double, double*, float*, void*) { return ISVD_E_UNSUPPORTED; }
isvd_status isvd_ws_omega(isvd_warmstart*, isvd_operator*, const float*, int, uint64_t, void*, int64_t, int*, void*) { return ISVD_E_UNSUPPORTED; }
}
