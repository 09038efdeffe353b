// device_plan.hpp -- plain-old-data plan records shared by the host planner
// and the gfx950 kernels, plus the LDS address swizzle both sides use.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define SPIN_HD __host__ __device__
#else
#define SPIN_HD
#endif

namespace spinqp {

constexpr int kMaxTileBits = 14;    // 2^14 amplitudes: 128 KiB of complex64 in LDS
constexpr int kMaxRegBits = 6;      // at most 64 amplitudes per lane
constexpr int kMaxMeas = 4;         // observable slots one pass can hold
constexpr int kMaxSites = 40;
constexpr int kBatchRing = 16;      // observable slots per gang problem (steps mod 16)
constexpr int kMaxMeasProfile = 64; // per-site observables one pass can hold (all-site profile)

// Op codes.  A two-spin factor on register bits (qa < qb) of a stage has
// code qa*8 + qb; kOpZZ is or-ed in when the factor carries an I^z I^z
// phase.  kOpMeas accumulates the observable of the state at that point.
constexpr int32_t kOpZZ = 64;
constexpr int32_t kOpMeas = 255;
// kOpMat (matrix engine, 32 registers per lane): multiply the lane's
// registers by a dense 32 x 32 complex matrix, the product of consecutive
// factors of the stage, on MFMA.  aux = index of the matrix in the matrix
// table: kMatFloats floats per matrix, the real 64 x 64 form
// W = [[Re U, -Im U], [Im U, Re U]] in MFMA A-operand order
// (W[32 b + (l % 32)][2 p + l / 32] at float (32 b + p) * 64 + l).
constexpr int32_t kOpMat = 254;
constexpr int kMatFloats = 64 * 64;

// One op of a stage.  For a factor with integrated strengths
// (A, B) = (sum a*tau, sum b*tau) over the merged two-spin propagators:
//   theta = B/2, t = tan(theta/2), s = sin(theta)     (three-shear rotation)
//   (pr, pi) = exp(+i A/4)                             (anti-aligned phase)
// For kOpMeas, aux is the measurement slot of the pass (resident kernels:
// unused).  In all-site profile plans every site has its own kOpMeas and
// aux = slot | kind << 6 | index << 8 | (norm slot + 1) << 14 | site << 17:
// the site's bit is thread bit `index` of the stage (kind 0), register bit
// `index` (kind 1) or global address bit `index` of the tile base (kind 2);
// norm slot + 1 = 0 when this observable does not also carry the norm.
template <typename T>
struct DevOp {
    int32_t code;
    int32_t aux;
    T t, s, pr, pi;
};

// One stage: the amplitudes of a tile are gathered from LDS into registers
// with register bit q <-> tile-local position rpos[q], the stage's ops run
// on registers, and the registers are scattered back.
struct DevStage {
    int32_t op0, nop;         // op range
    int32_t ntb;              // number of thread bits (tile bits - register bits)
    int32_t obs_tq;           // thread bit holding the observed site, or -1
    int32_t obs_mask;         // register-index mask of the observed site (0 if none)
    int32_t xnext;            // 1: the exchange after this stage moves amplitudes between
                              // waves (workgroup barrier); 0: within each wave only
    uint32_t tmask[16];       // LDS byte offset of thread bit q (zero past ntb)
    uint32_t rbit[8];         // LDS byte offset of register bit q
    // Global element offsets of thread bit q / register bit q, for the first
    // stage of a pass (loaded straight from HBM, input layout) and the last
    // (stored straight to HBM, output layout).
    int64_t gt_in[16], gr_in[8], gt_out[16], gr_out[8];
};

// One tiled pass over the whole state.
struct DevPass {
    int32_t k;                // tile bits
    int32_t stage0, nstage;   // stage range (at least one stage)
    int32_t writes;           // 0: read-only pass (observable only)
    int32_t nfree;            // number of non-tile bits
    int32_t obs_free_bit;     // global bit of the observed site if it is not a tile bit, else -1
    int32_t nmeas;            // measurements in this pass
    int32_t tile_barrier;     // 1: workgroup barrier after each tile's stores
    int32_t half;             // 1: half-tile exchanges (the top register bit of every stage
                              // is the same tile position, which has no LDS image)
    int32_t pad_;
    int64_t meas_step[kMaxMeas];   // step label of measurement slot m (plus launch offset)
    int64_t free_mask;        // mask of the global bits not in the tile
    int32_t tbit[16];         // global bit of tile-local position p (input layout)
    int32_t tbit_out[16];     // global bit of tile-local position p (output layout)
    // All-site profile plans: per-site measurement slots and norm slots.
    int32_t pmeas, pnorm;
    int64_t pmeas_step[kMaxMeasProfile];   // step label of slot m
    int8_t pmeas_site[kMaxMeasProfile];    // site of slot m
    int32_t pnorm_meas[kMaxMeas];          // measurement slot whose step the norm slot carries
};

// Fixed LDS swizzle of the one-workgroup kernel (tiled passes use a layout
// searched per pass, see encode_pass): xor a band of higher local-index bits into the lowest bits
// so that lanes striding by a power of two spread over the banks.  It is
// linear over GF(2): swz(a ^ b) = swz(a) ^ swz(b).
template <int ElemBytes>
SPIN_HD inline uint32_t lds_swizzle(uint32_t l) {
    // 8-byte elements: 32 per 256-byte bank row; 16-byte elements: 16.
    constexpr uint32_t shift = ElemBytes == 8 ? 5 : 4;
    constexpr uint32_t mask = ElemBytes == 8 ? 31 : 15;
    return l ^ ((l >> shift) & mask);
}

}  // namespace spinqp
