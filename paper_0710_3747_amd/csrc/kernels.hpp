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
    double* Pall;     // all-site profile [step][M] (profile launches only)
    uint64_t seed;
    int32_t M, polarized, init;
    int32_t pro_stage0, pro_nstage, step_stage0, step_nstage;
    int32_t pad_;
};

// One problem of a persistent batch launch.
struct BatchProblem {
    void* psi;
    double* P;
    double* N;
    uint64_t seed;
    int32_t M, polarized, init, gsize;   // gsize 1 with M <= tile bits: held in LDS
    // held in LDS: stage ranges of the prologue and of one step
    int32_t pro_stage0, pro_nstage, step_stage0, step_nstage;
    // gang: pass templates, launch list (template, step offset), tiles
    int32_t pass0, nlaunch;
    int64_t launch0, ntiles, part0;
    int32_t counter, pad_;
};

struct BatchJob {
    int32_t problem, rank;
};

struct PassShape {
    int r;    // register bits (amplitudes per lane = 2^r)
    int nt;   // lanes per workgroup; tile bits k = r + log2(nt)
    bool writes = true;   // false: read-only pass (observables only)
    int engine = 0;       // 0: VALU butterflies; 1: MFMA stage matrices (complex64, r = 5, nt = 512)
    const float* mats = nullptr;   // engine 1: device matrix table
    bool profile = false;          // per-site observables: profile partials [slot][nwg][M + 1]
    bool half = false;             // half-tile exchanges, two workgroups per CU (engine 0)
};
// Whether a pass kernel is instantiated for (precision, r, nt, engine).
bool pass_shape_exists(bool f32, int r, int nt, int engine);
// Whether a half-tile-exchange pass kernel is instantiated for (precision, r, nt).
bool pass_half_exists(bool f32, int r, int nt);

template <typename T>
hipError_t launch_init(void* psi, int M, int n, uint64_t seed, hipStream_t st);
template <typename T>
hipError_t launch_init_product(void* psi, int M, int n, uint64_t seed, hipStream_t st);
// Ensemble members first .. first + count - 1 stacked as one state of
// M + cbits sites (member index on the top cbits bits, zeros beyond count).
template <typename T>
hipError_t launch_init_members(void* psi, int M, int cbits, int polarized, uint64_t first,
                               uint64_t count, hipStream_t st);
// acc[i] = (acc[i] + add[i]) * scale for i < n (add may be null).
hipError_t launch_accumulate(double* acc, const double* add, int64_t n, double scale,
                             hipStream_t st);
template <typename T>
hipError_t launch_observe(const void* psi, int M, int site, double* partials, int nblk,
                          hipStream_t st);
hipError_t launch_reduce(const double* partials, int nwg, int ch, int64_t s0, int64_t count,
                         double* P, double* N, hipStream_t st);
hipError_t launch_reduce_profile(const double* partials, int nwg, int ch, int M, int64_t s0,
                                 int64_t count, double* Pall, double* N, hipStream_t st);
template <typename T>
hipError_t launch_factor(void* psi, int M, int lo, int hi, double t, double s, double pr,
                         double pim, int zz, hipStream_t st);
template <typename T>
hipError_t launch_pass(const PassShape& sh, void* psi, const DevPass* passes,
                       const DevStage* stages, const DevOp<T>* ops, int pass_index,
                       int64_t tiles_per_wg, int nwg, double* partials, int64_t step_offset,
                       int ch, hipStream_t st);
// Persistent batch launch over `nslots` workgroups (all resident at once);
// a gang-barrier time-out sets `err` and is or-ed into `*status`.  half:
// gangs run half-tile passes (two workgroups per CU) and problems held in
// LDS have at most tile bits - 1 sites.  Launch shape: batch_shape.
template <typename T>
hipError_t launch_batch(int nslots, bool half, const BatchProblem* probs, const BatchJob* jobs,
                        const int* job_start, const DevPass* passes, const DevStage* stages,
                        const DevOp<T>* ops, const int2* launches, double* partials, int* counters,
                        int ncounters, int* err, int* status, int64_t n_steps, hipStream_t st);
int batch_tile_bits(bool f32);
struct BatchShape {
    bool half;
    int r, nt;    // register bits, lanes; tile bits r + log2(nt) = batch_tile_bits
};
BatchShape batch_shape(bool f32, bool half);
// Workgroups of the batch kernel that fit one CU at once (0 on error).
int batch_blocks_per_cu(bool f32, bool half);

template <typename T>
hipError_t launch_resident(int r, int nt, const ResidentJob& job0, const ResidentJob* jobs,
                           int njobs, const DevStage* stages, const DevOp<T>* ops,
                           int64_t n_steps, hipStream_t st);

}  // namespace spinqp
