// abi_internal.hpp -- helpers shared by the C-ABI translation units.
#pragma once

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
void release_batch_caches();
void release_tune_cache();

}  // namespace spinqp
