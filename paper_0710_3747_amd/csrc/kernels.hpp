// kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_plan.hpp"

namespace spinqp {

// One problem owned by one workgroup for its whole run.
struct ResidentJob {
    void* psi;
    double* P;
    double* N;
    uint64_t seed;
    int32_t M, polarized, init;
    int32_t pro_stage0, pro_nstage, step_stage0, step_nstage;
    int32_t pad_;
};

struct PassShape {
    int r;    // register bits (amplitudes per lane = 2^r)
    int nt;   // lanes per workgroup; tile bits k = r + log2(nt)
    bool writes = true;   // false: read-only pass (observables only)
};

template <typename T>
hipError_t launch_init(void* psi, int M, int n, uint64_t seed, hipStream_t st);
template <typename T>
hipError_t launch_observe(const void* psi, int M, int site, double* partials, int nblk,
                          hipStream_t st);
hipError_t launch_reduce(const double* partials, int nwg, int ch, int64_t s0, int64_t count,
                         double* P, double* N, hipStream_t st);
template <typename T>
hipError_t launch_factor(void* psi, int M, int lo, int hi, double t, double s, double pr,
                         double pim, int zz, hipStream_t st);
template <typename T>
hipError_t launch_pass(const PassShape& sh, void* psi, const DevPass* passes,
                       const DevStage* stages, const DevOp<T>* ops, int pass_index,
                       int64_t tiles_per_wg, int nwg, double* partials, int64_t step_offset,
                       int ch, hipStream_t st);
template <typename T>
hipError_t launch_resident(int r, int nt, const ResidentJob& job0, const ResidentJob* jobs,
                           int njobs, const DevStage* stages, const DevOp<T>* ops,
                           int64_t n_steps, hipStream_t st);

}  // namespace spinqp
