// Matvec entry point that allocates nothing: the five-pass workspace lives in
// a fixed device array of the library instead of a caller buffer.
//
// The array below is a device symbol.  In host code its name is only a
// host-side stand-in, so host code never passes it to a kernel or a copy:
// each device's address is looked up once with hipGetSymbolAddress and kept
// in g_scratch_dev, and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "vie.h"
#include "vie_internal.h"

namespace vie {
vie_status fail(vie_status st, const std::string& msg);
vie_status hip_fail(hipError_t e, const char* where);
vie_status matvec_common(const vie_op* op, int mode, int dtype, int recon, const void* eps, const void* x,
                         void* y, int nrhs, void* ws, size_t ws_bytes, void* stream, const int* rhs_map);
}  // namespace vie

namespace {

constexpr size_t kScratchBytes = VIE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once per
// device, with that device current).
hipError_t scratch_address(int dev, void** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t vie_noalloc_scratch_bytes(void) { return kScratchBytes; }

vie_status vie_matvec_noalloc(const vie_op* op, int kind, int adjoint, int dtype, int recon, const void* eps_c,
                              const void* x, void* y, int nrhs, void* stream)
{
    using namespace vie;
    if (!op || !x || !y || nrhs < 1) return fail(VIE_E_ARG, "vie_matvec_noalloc: null argument or nrhs < 1");
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_noalloc: bad kind");
    if (adjoint != 0 && adjoint != 1) return fail(VIE_E_ARG, "vie_matvec_noalloc: adjoint must be 0 or 1");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_noalloc: bad dtype");
    // per-pass profiling records its own events, which this entry point does not create
    if (prof_is_enabled())
        return fail(VIE_E_UNSUPPORTED, "vie_matvec_noalloc: not available while per-pass profiling is on");
    const size_t need = vie_workspace_bytes(op, dtype, nrhs);
    if (need == 0 || need > kScratchBytes)
        return fail(VIE_E_ARG, "vie_matvec_noalloc: needs " + std::to_string(need) +
                                   " workspace bytes, above the fixed scratch of " +
                                   std::to_string(kScratchBytes) + " bytes (use vie_matvec with a workspace)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "vie_matvec_noalloc: hipGetDevice");
    if (dev != op->d.device)
        return fail(VIE_E_ARG, "vie_matvec_noalloc: the current device is not the operator's device");
    if (dev < 0 || dev >= kMaxDevices) return fail(VIE_E_UNSUPPORTED, "vie_matvec_noalloc: device index too large");
    void* ws = nullptr;
    e = scratch_address(dev, &ws);
    if (e != hipSuccess) return hip_fail(e, "vie_matvec_noalloc: hipGetSymbolAddress");
    int mode;
    if (kind == VIE_OP_A)
        mode = adjoint ? MODE_AH : MODE_A;
    else
        mode = adjoint ? MODE_NH : MODE_N;
    return matvec_common(op, mode, dtype, recon, eps_c, x, y, nrhs, ws, kScratchBytes, stream, nullptr);
}

}  // extern "C"
