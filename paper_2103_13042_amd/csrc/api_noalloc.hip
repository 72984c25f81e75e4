// The whole hot path for callers that cannot allocate (spamm_multiply_noalloc,
// include/spamm_noalloc.h): spamm_multiply with its workspace in a static
// device array instead of caller or library allocations.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"
#include "spamm.h"
#include "spamm_noalloc.h"

// One copy per device, held until the process ends.  In host code the name is
// only a handle: kernels get the device address that hipGetSymbolAddress
// returns for the current device, kept per device in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[SPAMM_NOALLOC_SCRATCH_BYTES];

namespace spamm_host {
namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

spamm_status scratch_of_current_device(void** out) {
    int dev = 0;
    spamm_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != SPAMM_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return fail(SPAMM_EUNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        if ((st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) !=
            SPAMM_OK)
            return st;
        if (!p) return fail(SPAMM_EDEVICE, "hipGetSymbolAddress(scratch) gave a null address on device %d", dev);
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return SPAMM_OK;
}

}  // namespace
}  // namespace spamm_host

using namespace spamm_host;

extern "C" spamm_status spamm_multiply_noalloc(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                               float* c, int64_t* pairs, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_grid(g);
    if (st != SPAMM_OK) return st;
    const size_t need = make_layout(g).total;
    if (need > size_t(SPAMM_NOALLOC_SCRATCH_BYTES))
        return fail(SPAMM_ENOSPACE, "n=%lld leaf=%d needs %zu bytes of workspace, above the %zu-byte static scratch",
                    (long long)n, leaf, need, size_t(SPAMM_NOALLOC_SCRATCH_BYTES));
    void* ws = nullptr;
    if ((st = scratch_of_current_device(&ws)) != SPAMM_OK) return st;
    return spamm_multiply(a, b, n, tau, leaf, c, pairs, ws, size_t(SPAMM_NOALLOC_SCRATCH_BYTES), stream);
}
