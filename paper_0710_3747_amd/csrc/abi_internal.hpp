// abi_internal.hpp -- helpers shared by the C-ABI translation units.
#pragma once

#include <cstddef>
#include <hip/hip_runtime.h>
#include <string>
#include <vector>

#include "../../include/spin.h"
#include "planner.hpp"

namespace spinqp {

int fail(int code, const std::string& msg);
int validate_common(const void* psi, int32_t prec, int32_t M);
int validate_couplings(int32_t M, const spin_coupling* J, int64_t K, std::vector<Coupling>* out);

// Launch geometry of the fused path for one call.
struct Shape {
    int r = 5;          // register bits
    int nt = 512;       // lanes per workgroup
    int k = 14;         // tile bits = r + log2(nt)
    int c = 3;          // low address bits every tile keeps (coalescing)
    int res_cap = 14;   // largest M held by one workgroup
    int engine = 0;     // 0: VALU butterflies, 1: MFMA stage matrices
    bool half = false;  // half-tile exchanges (two workgroups per CU)
    bool resident = false;
    bool valid = true;  // a pass kernel exists for (r, nt, engine)
};
Shape choose_shape(int prec, int M, const spin_options* opt);

// Caller-provided device workspace for the per-workgroup partial sums (the
// allocation-free entry point); with one, plans must already be cached.
struct Workspace {
    double* ptr;
    size_t doubles;
};
// spin_trotter_evolve_ex with partial sums in `ws` (ws_doubles doubles):
// no device allocation; SPIN_EUNSUPPORTED when the plan is not cached, when
// graph capture or the all-site profile is asked for, or when `ws` is too
// small for the plan's workgroups.
int evolve_with_workspace(void* psi, int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                          double dt, int64_t n_steps, int32_t observed_site, double* P_dev,
                          double* N_dev, const spin_options* opt, void* stream, double* ws,
                          size_t ws_doubles);
// Grow-only device scratch of at least `bytes`, one per (device, stream,
// slot); slot 0 is the fused path's partial sums.  Growing it waits for
// the stream.
int scratch_get_slot(hipStream_t st, int slot, size_t bytes, void** out);
void release_batch_caches();
void release_tune_cache();

}  // namespace spinqp
