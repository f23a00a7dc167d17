// The transient Phi for callers that cannot allocate device memory: its
// scratch (the sorted copy of one mode and the sort's temporaries) lives in a
// static device array of the library instead of a caller workspace.
#include <mutex>

#include "internal.hpp"

// File-scope device scratch: every GPU the library runs on holds its own copy
// until the process ends. In host code `scratch` is only a stand-in for the
// symbol; its address on the current device comes from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[CPAPR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // per device: the device address of `scratch`

// The address of `scratch` on the current device, looked up once per device
// (with that device current) on the first call there.
cpapr::Error scratch_address(void** out)
{
    int dev = -1;
    CPAPR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return {CPAPR_EUNSUPPORTED, "device index outside the supported range"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        CPAPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) return {CPAPR_EHIP, "hipGetSymbolAddress gave no address for the scratch array"};
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return {CPAPR_OK, ""};
}

int fail(const cpapr::Error& e)
{
    if (e.code) cpapr::set_last_error(e.msg);
    return e.code;
}

}  // namespace

extern "C" int cpapr_phi_coo_noalloc(const cpapr_coo* X, int32_t mode, int32_t R, const double* B,
                                     const double* const* A, double eps, double* Phi, void* stream)
{
    try {
        cpapr::Error e = cpapr::check_transient(X, mode, R, true);
        if (e.code) return fail(e);
        const size_t need = cpapr::transient_bytes(X->nmodes, X->nnz);
        if (need > (size_t)CPAPR_NOALLOC_SCRATCH_BYTES)
            return fail({CPAPR_EUNSUPPORTED, "the tensor needs " + std::to_string(need) +
                                                 " bytes of scratch, more than the no-allocation entry point's " +
                                                 std::to_string((size_t)CPAPR_NOALLOC_SCRATCH_BYTES) +
                                                 "; use cpapr_phi_coo with a workspace"});
        void* ws = nullptr;
        e = scratch_address(&ws);
        if (e.code) return fail(e);
        return fail(cpapr::phi_transient(X, mode, R, B, A, eps, Phi, (char*)ws, (size_t)CPAPR_NOALLOC_SCRATCH_BYTES,
                                         (hipStream_t)stream));
    } catch (...) {
        return fail({CPAPR_EINVAL, "unexpected exception"});
    }
}
