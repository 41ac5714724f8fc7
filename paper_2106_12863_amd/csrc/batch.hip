// Batched form (placeholder until the persistent work-queue kernel lands).
#include <hip/hip_runtime.h>

#include "sinet_internal.h"

using namespace sinet;

extern "C" {

sinet_status sinet_autotune(const sinet_stream*, uint32_t, const char*, hipStream_t, sinet_tune*) {
    return fail(SINET_ERR_UNSUPPORTED, "batching not built yet");
}
sinet_status sinet_batch_plan_create(const sinet_stream*, uint32_t, const sinet_tune*, hipStream_t,
                                     sinet_batch_plan** out) {
    if (out) *out = nullptr;
    return fail(SINET_ERR_UNSUPPORTED, "batching not built yet");
}
sinet_status sinet_batch_run(sinet_batch_plan*, hipStream_t) {
    return fail(SINET_ERR_UNSUPPORTED, "batching not built yet");
}
sinet_status sinet_batch_plan_destroy(sinet_batch_plan*) {
    return fail(SINET_ERR_UNSUPPORTED, "batching not built yet");
}

}  // extern "C"
