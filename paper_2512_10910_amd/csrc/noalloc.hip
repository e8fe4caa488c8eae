// pne_contract_batch_noalloc: pne_contract_batch without device allocation.
//
// Every table and buffer of the batch (instance tables, site records,
// messages, slices, weights, results) is placed in `scratch`, a fixed device
// array of kNoAllocScratchBytes that each GPU the library runs on holds until
// the process ends.  Results are copied back to pageable host memory and the
// call ends with a synchronisation of the context stream; no hipMalloc,
// hipFree, pinned allocation or event creation happens here.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pne.h"
#include "runtime.h"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// Scratch of the allocation-free entry point.  In host code this name is a
// host-side stand-in, not a device address: only the per-device pointer that
// hipGetSymbolAddress returns is ever passed to the device.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up once per device.
hipError_t scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" pne_status pne_contract_batch_noalloc(pne_ctx *ctx, pne_network *const *nets, int32_t n,
                                                 const pne_options *opt, pne_result *results) {
    if (!ctx || !nets || n <= 0 || !opt || !results)
        return pne::ctx_fail(ctx, PNE_ERR_INVALID_ARG, "bad arguments");
    const int dev = pne::ctx_device(ctx);
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return pne::ctx_fail(ctx, PNE_ERR_DEVICE, "no current device");
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return pne::ctx_fail(ctx, PNE_ERR_DEVICE, "cannot select device");
    void *base = nullptr;
    const hipError_t e = scratch_address(dev, &base);
    pne_status st = PNE_OK;
    if (e != hipSuccess) {
        st = pne::ctx_fail(ctx, PNE_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    } else {
        pne::StaticArena arena;
        arena.base = static_cast<char *>(base);
        arena.cap = kNoAllocScratchBytes;
        pne_batch *b = nullptr;
        st = pne::batch_create_on(ctx, nets, n, opt, pne::ctx_stream(ctx), &b, &arena);
        if (st == PNE_OK) {
            st = pne_batch_run(b, results);
            pne_batch_destroy(b);
        }
    }
    if (prev != dev) (void)hipSetDevice(prev);
    return st;
}
