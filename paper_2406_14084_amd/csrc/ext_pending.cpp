// ext_pending.cpp -- entry points declared in qs.h whose kernels are not in
// this build yet: they fail cleanly with QS_EUNSUPPORTED.
#include "qs_internal.h"

extern "C" {
qs_status qs_costmodel_create(uint64_t, void *, qs_costmodel **) { qs::set_error("cost model: not built"); return QS_EUNSUPPORTED; }
qs_status qs_costmodel_free(qs_costmodel *) { return QS_OK; }
qs_status qs_costmodel_get_params(const qs_costmodel *, float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_set_params(qs_costmodel *, const float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_train_step(qs_costmodel *, const float *, const float *, int, float, float *) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_predict(const qs_costmodel *, const float *, float *, int) { return QS_EUNSUPPORTED; }
qs_status qs_costmodel_get_grads(const qs_costmodel *, float *) { return QS_EUNSUPPORTED; }
qs_status qs_plan_block_features(const qs_plan *, float *, int, int *) { return QS_EUNSUPPORTED; }
}
