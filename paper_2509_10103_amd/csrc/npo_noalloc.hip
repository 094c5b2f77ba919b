// Fixed device workspace of npo_forward_step_noalloc.
//
// The forward step needs a workspace (vorticity parts, nonlinear terms, stage
// iterates, axially transformed intermediates).  Callers that cannot allocate
// device memory get it from `scratch`, a file-scope device array of
// NPO_SCRATCH_BYTES that every device the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel: that is
// a host-side stand-in, not a device address.  npo_plan_create (the library's
// set-up call) resolves the array's device address once per device, with that
// device current, and the entry point launches its kernels with that address.
// Every call on one device shares that device's array, so calls that overlap
// on one device race; the array keeps the last call's contents, and the
// forward step writes every part of it that it reads before reading it, so
// nothing needs clearing between calls.
#include "npo_internal.h"
#include "../../include/npo.h"

#include <mutex>

static __device__ __align__(256) unsigned char scratch[NPO_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};
}  // namespace

namespace npo {

hipError_t scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return g_err[device];
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_done[device] = true;
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? ptr : nullptr;
    return e;
}

void* scratch_ptr(int device, hipError_t* err) {
    if (device < 0 || device >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    *err = g_done[device] ? g_err[device] : hipErrorNotInitialized;
    return g_ptr[device];
}

}  // namespace npo
