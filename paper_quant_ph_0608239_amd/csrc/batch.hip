// Batched persistent launch (placeholder until the batch kernel lands).
#include "qsim_internal.h"

extern "C" {
int qsim_batch_create(int, const int *, const int64_t *, const qsim_gate *, int, void *, qsim_batch **out)
{
    if (out) *out = nullptr;
    return qsim::set_error(QSIM_EUNSUPPORTED, "batch: not built yet");
}
int qsim_batch_run(qsim_batch *, qsim_batch_stats *) { return qsim::set_error(QSIM_EUNSUPPORTED, "batch: not built yet"); }
int qsim_batch_latencies(qsim_batch *, double *) { return qsim::set_error(QSIM_EUNSUPPORTED, "batch: not built yet"); }
int qsim_batch_download(qsim_batch *, int, void *, size_t) { return qsim::set_error(QSIM_EUNSUPPORTED, "batch: not built yet"); }
int qsim_batch_free(qsim_batch *) { return QSIM_OK; }
}
