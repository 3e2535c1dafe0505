// stencil_apply without any allocation: the workspace of the sweep is a
// fixed device array of this library instead of caller memory.
#include <mutex>

#include "plan.h"

namespace {

constexpr size_t kNoAllocBytes = size_t(64) << 20;   // 64 MiB per GPU

// The sweep's scratch space.  Each device holds its own copy for the life
// of the process.  Host code never passes `scratch` itself (its host-side
// name is not a device address): it passes the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_on_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" st_status stencil_apply_noalloc(const st_plan* plan, const void* u_in, void* u_out, int32_t steps,
                                           const st_wave_args* wave, void* stream) {
    stk::set_error("%s", "");
    if (!plan) {
        stk::set_error("plan is NULL");
        return ST_EINVAL;
    }
    if (plan->batched || plan->prob.update == ST_VARCOEF) {
        stk::set_error("stencil_apply_noalloc takes single-grid linear or wave plans");
        return ST_EINVAL;
    }
    if (steps < 0) {
        stk::set_error("steps must be >= 0");
        return ST_EINVAL;
    }
    const size_t need = stencil_workspace_bytes(plan, steps, 0);
    if (need > kNoAllocBytes) {
        stk::set_error("needs %zu bytes of scratch; the no-allocation entry point holds %zu", need,
                       kNoAllocBytes);
        return ST_EWORKSPACE;
    }
    void* ws = nullptr;
    const hipError_t e = scratch_on_current_device(&ws);
    if (e != hipSuccess) {
        stk::set_error("hipGetSymbolAddress failed: %s", hipGetErrorString(e));
        return ST_EHIP;
    }
    return stencil_apply(plan, u_in, u_out, steps, wave, ws, kNoAllocBytes, stream);
}

extern "C" size_t stencil_noalloc_capacity(void) { return kNoAllocBytes; }
