// fftu_execute_noalloc: fftu_execute_ws with a fixed device array as the
// workspace, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable of this library's code object:
// each device the library runs on holds its own copy, at its own address, from
// the time the code object is loaded there until the process ends. Host code
// never passes the array's name to a kernel (in host code that name is a
// host-side stand-in, not a device address): on the first call on a device,
// with that device current, hipGetSymbolAddress looks up the device address
// once, and every call on that device passes that address as the workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fftu.h"
#include "fftu_internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(FFTU_NOALLOC_MAX_BYTES);
static_assert(kScratchBytes % 256 == 0, "whole 256-byte granules");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be the current device.
hipError_t scratch_address(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_once[device], [device] {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
    });
    *ptr = g_ptr[device];
    return g_err[device];
}

}  // namespace

extern "C" fftu_status fftu_execute_noalloc(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    if (!plan || fftu::plan_is_batch(plan)) return fftu::record_status(FFTU_ERROR_INVALID_VALUE);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fftu::record_status(FFTU_ERROR_DEVICE);
    if (cur != fftu::plan_device(plan)) return fftu::record_status(FFTU_ERROR_INVALID_VALUE);
    if (fftu::plan_workspace_bytes(plan) > kScratchBytes) return fftu::record_status(FFTU_ERROR_OUT_OF_MEMORY);
    void *ws = nullptr;
    if (scratch_address(cur, &ws) != hipSuccess || !ws) return fftu::record_status(FFTU_ERROR_DEVICE);
    return fftu_execute_ws(plan, in, out, ws, stream);   // its checks, its kernels, its status
}
