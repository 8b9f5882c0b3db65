// The allocation-free variant of pint_solve (include/pint.h,
// pint_solve_noalloc): the solve's workspace (spectrum, starting-step
// corrections, norm partials, direct-form source spectrum) lives in a
// file-scope device array instead of caller- or library-allocated memory.
#include "../../include/pint.h"
#include "pint_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: its device address comes from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// with that device current.
pint_status scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pint::set_error(PINT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return pint::set_error(PINT_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pint::set_error(PINT_E_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PINT_OK;
}

}  // namespace

extern "C" {

pint_status pint_solve_noalloc(pint_plan* plan, const double* v, const double* f, const double* fder, double* U,
                               double* upd, double* upd_l2T, int* sweeps) {
    void* ws = nullptr;
    const pint_status rc = scratch_ptr(&ws);
    if (rc != PINT_OK) return rc;
    return pint::solve_in_workspace(plan, ws, kScratchBytes, v, f, fder, U, upd, upd_l2T, sweeps);
}

}  // extern "C"
