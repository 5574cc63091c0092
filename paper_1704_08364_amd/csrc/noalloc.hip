// noalloc.hip -- bst_backproject_noalloc: the backprojection with its
// workspace in a static device array instead of a caller buffer, for callers
// that cannot allocate device memory.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, of kScratchBytes, from the library's load until the process
// ends. In host code its name is only a host-side stand-in, so the kernels
// never receive it: on the first call on a device (with that device current)
// hipGetSymbolAddress yields the device address, which is cached per device
// and passed as the workspace. Nothing needs clearing between calls (every
// workspace word the kernels read is written by an earlier kernel of the same
// call), and calls that overlap in time on one GPU share the array and race.
#include <mutex>

#include "bst_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (looked up once per device)
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" bst_status bst_backproject_noalloc(bst_plan_t plan, const float* sino, float* img, int32_t batch,
                                              void* stream) {
    if (!plan) return BST_E_NULL;
    if (batch < 0 || batch > plan->prm.max_batch) return BST_E_BATCH;
    if (batch == 0) return BST_OK;
    if (plan->device >= kMaxDevices) return BST_E_UNSUPPORTED;
    const size_t need = bst::backproject_workspace_need(plan, batch);
    if (need > kScratchBytes) {
        bst::set_last_error_text("bst_backproject_noalloc: the workspace of this batch exceeds the 256 MiB static "
                                 "scratch; use fewer slices per call or bst_backproject with a caller workspace");
        return BST_E_WORKSPACE;
    }
    void* ws = nullptr;
    const hipError_t e = scratch_address(plan->device, &ws);
    if (e != hipSuccess) {
        bst::set_last_error(e);
        return BST_E_DEVICE;
    }
    return bst::backproject_in(plan, sino, img, batch, ws, kScratchBytes, stream);
}
