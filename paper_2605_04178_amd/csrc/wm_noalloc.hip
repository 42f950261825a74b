// wm_noalloc.hip -- wm_loss_grad_noalloc: the loss + gradient call of
// wm_loss_grad with its workspace in a fixed, file-scope device array
// instead of a caller-supplied buffer, for callers that cannot allocate.
//
// The array holds the gradient sweep's partial rows and redo-flag words for
// up to WM_NOALLOC_MAX_N descriptors.  In host code `scratch` is only a
// host-side stand-in for the device symbol: its device address is looked up
// once per device with hipGetSymbolAddress and only that address is passed
// on.  Every word the kernels read is written earlier in the same call (each
// flag word and partial row exactly once), so nothing is cleared between
// calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wavemodel.h"
#include "wm_launch.hpp"

namespace {

// sized by the gradient workspace layout: partial rows of the largest
// persistent grid plus the float64 pass, 256-byte aligned, then one 64-bit
// flag word per 64 descriptors
constexpr size_t kPartialBytes =
    ((sizeof(double) * wm::kAcc * (size_t)(wm::kGradMaxBlocks + wm::kRedoMaxBlocks)) + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kPartialBytes + sizeof(uint64_t) * (size_t)(WM_NOALLOC_MAX_N / 64);
static_assert(WM_NOALLOC_MAX_N % 64 == 0, "whole flag words");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// the current device's copy of the array (looked up on its first use)
int32_t scratch_of_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return wm::record_hip_error(e);
    if (dev < 0 || dev >= kMaxDevices) return WM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return wm::record_hip_error(e);
        if (!p) return WM_EINVAL;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return WM_OK;
}

}  // namespace

extern "C" size_t wm_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int32_t wm_loss_grad_noalloc(const wm_desc_t* desc, const float* measured,
                                        const wm_params_t* params, double* out, void* stream)
{
    // every argument is checked before the first HIP call
    if (!wm::grad_args_ok(desc, measured, params, out)) return WM_EINVAL;
    if (desc->n > (int64_t)WM_NOALLOC_MAX_N) return WM_ETOOLARGE;
    if (wm_workspace_bytes(WM_OP_LOSS_GRAD, desc->n, 1, 0) > kScratchBytes) return WM_ETOOLARGE;
    void* ws = nullptr;
    const int32_t rc = scratch_of_current_device(&ws);
    if (rc != WM_OK) return rc;
    return wm_loss_grad(desc, measured, params, out, ws, kScratchBytes, stream);
}
