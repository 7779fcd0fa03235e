// Batched execution of independent plans (placeholder until the batched launch lands).
#include <hip/hip_runtime.h>

#include "../../include/sharp.h"

extern "C" int sharp_batch_create(sharp_batch* out, int, const sharp_plan*) {
    if (out) *out = nullptr;
    return SHARP_ERR_INVALID_ARG;
}
extern "C" void sharp_batch_destroy(sharp_batch) {}
extern "C" size_t sharp_batch_workspace_bytes(sharp_batch) { return 0; }
extern "C" int sharp_batch_set_workspace(sharp_batch, void*, size_t) { return SHARP_ERR_INVALID_ARG; }
extern "C" int sharp_batch_set_stream(sharp_batch, void*) { return SHARP_ERR_INVALID_ARG; }
extern "C" int sharp_batch_raar_iterate(sharp_batch, int, float) { return SHARP_ERR_INVALID_ARG; }
