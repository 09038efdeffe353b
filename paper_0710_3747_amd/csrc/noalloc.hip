// noalloc.hip -- spin_trotter_evolve_noalloc: the evolve call for callers
// that cannot allocate device memory.  Its per-workgroup partial sums live
// in a fixed device array of this file instead of the library's grow-only
// workspace; plans must have been prepared beforehand.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "../../include/spin.h"
#include "abi_internal.hpp"

namespace spinqp {

// 1 MiB of FP64 partial sums: 2 values per workgroup per step slot, enough
// for 1024 workgroups x 64 step slots.  Each GPU holds its own copy for the
// life of the process.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 17;
static_assert(kNoAllocScratchDoubles * sizeof(double) == SPIN_NOALLOC_SCRATCH_BYTES,
              "scratch size differs from the header's");

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

std::mutex g_mu;
std::map<int, double*> g_ptr;   // device -> address of that device's `scratch`

// Address of the current device's array, looked up once per device (with
// that device current).  The array's name in host code is not a device
// address; only this pointer is passed to kernels.
int scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ptr.find(dev);
    if (it == g_ptr.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SPIN_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_ptr.emplace(dev, static_cast<double*>(p)).first;
    }
    *out = it->second;
    return SPIN_OK;
}

}  // namespace
}  // namespace spinqp

using namespace spinqp;

extern "C" int spin_trotter_evolve_noalloc(void* psi, int32_t prec, int32_t M, const spin_coupling* J,
                                           int32_t K, double dt, int64_t n_steps, int32_t observed_site,
                                           double* P_dev, double* N_dev, const spin_options* opt,
                                           void* stream) {
    try {
        double* ws = nullptr;
        int rc = scratch_ptr(&ws);
        if (rc) return rc;
        return evolve_with_workspace(psi, prec, M, J, K, dt, n_steps, observed_site, P_dev, N_dev, opt,
                                     stream, ws, kNoAllocScratchDoubles);
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
