// placeholder, replaced by the batched kernels
#include "../../include/dg.h"
extern "C" {
int dg_batch_create(int, dg_problem1d*, int, const dg_options*, int64_t*, dg_batch** out)
{
    if (out) *out = nullptr;
    return DG_ERR_UNSUPPORTED;
}
int dg_batch_destroy(dg_batch*) { return DG_ERR_UNSUPPORTED; }
int dg_batch_buffer_sizes(const dg_batch*, size_t*, size_t*) { return DG_ERR_UNSUPPORTED; }
int dg_batch_bind(dg_batch*, void*, void*, void*, void*) { return DG_ERR_UNSUPPORTED; }
int dg_batch_set_state(dg_batch*, const double*) { return DG_ERR_UNSUPPORTED; }
int dg_batch_get_state(dg_batch*, double*) { return DG_ERR_UNSUPPORTED; }
int dg_batch_run(dg_batch*, const double*, int64_t, dg_report*) { return DG_ERR_UNSUPPORTED; }
}
