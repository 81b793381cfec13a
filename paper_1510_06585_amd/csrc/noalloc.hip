// Allocation-free execution requests: skel_plan_run with the plan's device
// scratch taken from one static device array instead of hipMalloc.
//
// For callers that cannot allocate device memory at run time (code under HIP
// graph capture, serving loops that forbid allocation).  The array is a
// file-scope __device__ object, so every GPU the library runs on holds its own
// copy of it from module load until the process ends.  In host code the
// array's name is only a host-side stand-in: its device address on each GPU is
// looked up once with hipGetSymbolAddress (by skel_init, or by the entry
// point's first call on a device) and only that address is ever passed to
// kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

using namespace skel;

static __device__ __align__(256) unsigned char scratch[SKEL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = (size_t)SKEL_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch` per device (null: not resolved yet)

}  // namespace

skel_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(SKEL_EUNSUPPORTED, "device %d: the static scratch table covers devices 0..%d", device,
                         kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return SKEL_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(SKEL_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                         hipGetErrorString(e));
    g_ptr[device] = ptr;
    return SKEL_OK;
}

extern "C" skel_status skel_plan_run_noalloc(skel_plan p, const skel_buffer* args, int32_t nargs, void* stream) {
    clear_error();
    NoallocLayout L;
    skel_status st = noalloc_prepare(p, args, nargs, kScratchBytes, L);
    if (st) return st;
    int device = 0;
    const hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return set_error(SKEL_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if ((st = noalloc_setup(device))) return st;
    void* region;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        region = g_ptr[device];
    }
    return noalloc_run(p, args, stream, (char*)region, L);
}
