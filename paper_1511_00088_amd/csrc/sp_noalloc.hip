// sp_cg_force_noalloc: the adjoint link and mass gradient of sp_cg_force for callers that cannot allocate
// device memory (code under stream capture, tight serving loops). Its kernels are sp_cg_force's; their scratch
// (packed x and lambda, D_oe x, D_oe lambda, the reduction partials) lives in `scratch`, a file-scope device
// array of SP_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, looked up once per device (with that device current) on the first call there, and
// only that address is ever handed to a kernel.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "sp_entry.h"

static __device__ __align__(256) unsigned char scratch[SP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first call on that device.
int scratch_of_current_device(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sp::set_error(SP_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return sp::set_error(SP_ERR_UNSUPPORTED, "device index beyond 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            return sp::set_error(SP_ERR_HIP, e != hipSuccess ? hipGetErrorString(e)
                                                              : "hipGetSymbolAddress returned a null address");
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (char*)g_scratch_ptr[dev];
    return SP_OK;
}

}  // namespace

extern "C" int sp_cg_force_noalloc(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e,
                                   const double* lambda_e, double* gamma, double* force, double* grad_mass,
                                   void* stream) {
    sp::Geom G;
    int rc = sp::force_check(g, U, mass, x_e, lambda_e, gamma, &G);
    if (rc) return rc;
    const size_t need = sp::force_scratch_bytes(G);
    if (need > (size_t)SP_NOALLOC_SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "lattice needs %zu scratch bytes, above the fixed %zu of sp_cg_force_noalloc", need,
                 (size_t)SP_NOALLOC_SCRATCH_BYTES);
        return sp::set_error(SP_ERR_WORKSPACE, msg);
    }
    char* base = nullptr;
    if ((rc = scratch_of_current_device(&base))) return rc;
    return sp::force_enqueue(g, G, U, mass, x_e, lambda_e, gamma, force, grad_mass, base, (hipStream_t)stream);
}
