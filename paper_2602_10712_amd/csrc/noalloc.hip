// srp_trace_noalloc: the forward trace (srp_trace) with its workspace -- the per-direction grid
// frames and the FP64 per-workgroup partial sums -- in one fixed device array of this library
// instead of memory the scene allocates, so that a call allocates nothing.
//
// Host code never passes the array's name to a kernel or a copy: in host code `scratch` is only a
// stand-in for the device symbol.  The array's address on a device is looked up once per device
// (hipGetSymbolAddress, with that device current) and that address is what the kernels receive.
// Each device holds its own copy of the array for the life of the process; every call on a
// device shares it, so calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/srp.h"
#include "scene.h"
#include "srp_internal.h"

static __device__ __align__(256) unsigned char scratch[SRP_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};  // device address of `scratch` per device, once looked up

// Device address of the workspace array on `device`, which must be the current device.
srp_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return srp_fail(SRP_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return srp_fail(SRP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return SRP_OK;
}

}  // namespace

extern "C" srp_status srp_trace_noalloc(srp_scene s, const double* sun_dirs, int64_t D,
                                        const srp_trace_params* params, const double* frames, double* force,
                                        double* torque, void* stream)
{
    if (!s) return srp_fail(SRP_EINVAL, "scene is NULL");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return srp_fail(SRP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != s->device) {
        e = hipSetDevice(s->device);
        if (e != hipSuccess) return srp_fail(SRP_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    void* base = nullptr;
    const srp_status st = scratch_address(s->device, &base);
    if (st != SRP_OK) return st;
    const srp::TraceWorkspace ws{base, static_cast<size_t>(SRP_NOALLOC_WORKSPACE_BYTES)};
    return srp::trace_into(s, sun_dirs, D, params, frames, force, torque, static_cast<hipStream_t>(stream), &ws);
}
