// sharp_apply_noalloc: sharp_apply for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).  The operators' scratch (see apply_scratch) lives in
// one file-scope device array instead of the plan's workspace; the caller
// still passes the input and output.  Each device holds its own copy of the
// array from the first call on it until the process ends, and every call on
// a device shares it: calls that overlap on one device (concurrent streams,
// other host threads) race on it.  Every scratch element an operator reads
// is written earlier in the same call, so nothing needs clearing between
// calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sharp.h"
#include "plan_impl.hpp"

namespace {

constexpr size_t kScratchBytes = SHARP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Host code must not use this name as an address: it is a host-side stand-in.
// The device address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_on_current_device(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SHARP_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SHARP_ERR_HIP;
        g_scratch[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch[dev]);
    return SHARP_OK;
}

}  // namespace

extern "C" int sharp_apply_noalloc(sharp_plan p, int op, const void* d_in, void* d_out) {
    if (!p || op < SHARP_OP_F || op > SHARP_OP_OBJECT) return SHARP_ERR_INVALID_ARG;
    if (sharp::apply_scratch(*p, op).total > kScratchBytes) return SHARP_ERR_SCRATCH_LIMIT;
    const int chk = sharp::apply_check(*p, op, d_in, d_out);  // host-side checks before any device call
    if (chk != SHARP_OK) return chk;
    char* ptr = nullptr;
    const int st = scratch_on_current_device(&ptr);
    if (st != SHARP_OK) return st;
    return sharp::apply_into(*p, op, d_in, d_out, ptr);
}
