// tnrd_forward_noalloc: the forward of tnrd_forward for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The forward's scratch (domain flag,
// ping-pong planes, prepared stage constants) lives in one fixed device array
// per GPU instead of a caller workspace; the stage kernels are the same ones
// tnrd_forward launches.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tnrd.h"
#include "tnrd_api_internal.hpp"

namespace {

// The fixed scratch.  Each GPU the library runs on holds its own copy, at its
// own address, until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a host-side stand-in,
// not a device address): it uses the address hipGetSymbolAddress returned for
// the current device.
static __device__ __align__(256) unsigned char scratch[TNRD_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
};

DeviceScratch g_scratch[MAX_DEVICES];

// Device address of the current device's copy of `scratch`, looked up once per
// device (with that device current) on its first call; nullptr on failure.
void *device_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    DeviceScratch &d = g_scratch[dev];
    std::call_once(d.once, [&d]() {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (d.err == hipSuccess) d.ptr = p;
        (void)hipGetLastError();
    });
    return d.ptr;
}

}  // namespace

extern "C" int tnrd_forward_noalloc(const float *f, int N, int H, int W, int L,
                                    const tnrd_model *m, float *u_out, float *states,
                                    const tnrd_opts *o, void *stream)
{
    tnrd_opts oo;
    tnrd::resolve_opts(o, &oo);
    tnrd::ForwardPlan p;
    int st = tnrd::plan_forward(f, N, H, W, L, m, u_out, states, oo, &p);
    if (st != TNRD_OK) return st;
    if (N == 0) return TNRD_OK;
    if (p.ws_bytes > (size_t)TNRD_NOALLOC_SCRATCH_BYTES) return TNRD_ERR_CAPACITY;
    void *ws = device_scratch();
    if (!ws) return TNRD_ERR_HIP;
    return tnrd::run_forward(f, N, H, W, m, u_out, states, oo, p, ws, (hipStream_t)stream);
}
