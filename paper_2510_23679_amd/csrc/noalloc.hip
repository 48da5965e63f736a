// Best hits of one genome pair without a caller workspace and without device allocation.
//
// pdp_bh takes its scratch (the plan's device tables, the shared-k-mer records of the
// join, the tiles' record ranges and row slabs, counters and scan partials) from a
// workspace the caller allocates.  Callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, hosts that forbid allocation) call
// pdp_bh_noalloc instead: the same kernels, with the scratch in a fixed device array of
// this library.  The array exists once per device, from the library's load to the end of
// the process; its address on a device is looked up once, on the first call made with
// that device current.  Calls share the array: every call's kernels clear or overwrite
// what they read (the launch's first kernel resets its counters and status, the plan's
// tables are copied in before the kernels), so a call never depends on what an earlier
// one left, but two calls that overlap on one device race on it.
#include <mutex>

#include "internal.hpp"

using namespace pdp;

// The scratch of pdp_bh_noalloc.  In host code this name is a stand-in, not a device
// address: only the address from hipGetSymbolAddress is ever used.
static __device__ __align__(256) uint8_t scratch[PDP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // the array's device address, per device (null: not looked up yet)

// The array's address on the current device, looked up on the first call with it current.
int32_t scratch_on_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return api_fail(PDP_E_HIP, "pdp_bh_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return api_fail(PDP_E_LIMIT, "pdp_bh_noalloc: device %d past the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return api_fail(PDP_E_HIP, "pdp_bh_noalloc: hipGetSymbolAddress of the scratch on device %d: %s", dev,
                            hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PDP_OK;
}

}  // namespace

extern "C" int32_t pdp_bh_noalloc(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, pdp_bh_out *out,
                                  pdp_status *status, void *stream) {
    if (!q || !t || !out || !status) return api_fail(PDP_E_INVAL, "pdp_bh_noalloc: null pointer");
    uint64_t need = 0;
    int32_t rc = pdp_bh_ws_size(q, t, params, &need);
    if (rc) return rc;
    if (need > PDP_NOALLOC_SCRATCH_BYTES)
        return api_fail(PDP_E_WORKSPACE,
                        "pdp_bh_noalloc: this genome pair needs %llu bytes of scratch, the fixed scratch holds %llu; "
                        "call pdp_bh with a workspace of pdp_bh_ws_size bytes",
                        static_cast<unsigned long long>(need), static_cast<unsigned long long>(PDP_NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    return pdp_bh(q, t, params, out, status, ws, PDP_NOALLOC_SCRATCH_BYTES, stream);
}
