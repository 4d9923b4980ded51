// The keys-only sort for callers that cannot allocate device memory
// (mms_sort_u32_noalloc in include/mms.h): the sort's workspace (its
// ping-pong buffer and partition table) is a fixed array of device memory
// in the library's code object, one copy per GPU, instead of a buffer the
// caller passes in.  The sort itself is mms_sort_u32's, kernels and all.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mms.h"
#include "mms_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MMS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// In host code this name is a host-side stand-in, not a device address:
// every use below goes through the per-device address of the symbol.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch` on each GPU

// Address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and kept for the process.
int scratch_on_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mms::host::hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return mms::host::fail(MMS_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return mms::host::hip_fail(e, "scratch symbol address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MMS_OK;
}

}  // namespace

extern "C" int mms_sort_u32_noalloc(const uint32_t* d_in, uint32_t* d_out, uint64_t n, uint32_t flags,
                                    void* stream) {
    if (flags & ~MMS_KEY_I32) return mms::host::fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (n == 0) return MMS_OK;
    if (n >= (1ull << 32)) return mms::host::fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    const size_t need = mms_workspace_bytes(n, flags);
    if (need > kScratchBytes)
        return mms::host::fail(MMS_EINVAL, "n = %llu needs %zu bytes of workspace; the fixed scratch holds %zu",
                               (unsigned long long)n, need, kScratchBytes);
    void* ws = nullptr;
    if (need) {
        const int rc = scratch_on_current_device(&ws);
        if (rc) return rc;
    }
    return mms_sort_u32(d_in, d_out, n, ws, need ? kScratchBytes : 0, flags, stream);
}
