// kernels.hip -- gfx950 kernels of the random-phase Trotter path.
//
//  k_init        random-phase state (counter-based SplitMix64 phases)
//  k_init_product  product state of M-1 random single-spin phases
//  k_init_members  2^c basis-state members of the ensemble stacked as one
//                state of M + c sites (member index on the top c bits)
//  k_accumulate  member sums of consecutive evolutions, in order
//  k_pass        one tiled sweep: a 2^k-amplitude tile per workgroup is
//                staged through LDS; register stages apply the two-spin
//                factors as three-shear rotations; observables are
//                accumulated in FP64 and reduced per workgroup
//  k_resident    whole state in one workgroup's LDS for every step
//  k_factor      one factor over the whole state (the unfused schedule)
//  k_observe     observable of a state as it is
//  k_reduce      fixed-order reduction of per-workgroup partial sums
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_plan.hpp"
#include "kernels.hpp"

namespace spinqp {

template <typename T> struct CT;
template <> struct CT<float> {
    using c = float2;
    using v = float4;       // 16-byte global access: two amplitudes
    static constexpr int V = 2;
};
template <> struct CT<double> {
    using c = double2;
    using v = double2;      // 16-byte global access: one amplitude
    static constexpr int V = 1;
};

// ------------------------------------------------------------ SplitMix64
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// u(seed, r) = (z >> 11) 2^-53 with z output r+1 of the SplitMix64 stream
// started at `seed`, read directly at that counter.
__device__ __forceinline__ double sm64_uniform(uint64_t seed, uint64_t r) {
    const uint64_t z = sm64_mix(seed + (r + 1ull) * 0x9E3779B97F4A7C15ull);
    return double(z >> 11) * 0x1.0p-53;
}

// Amplitude of basis state x of the random-phase state, FP64.
__device__ __forceinline__ void random_phase_amp(uint64_t x, int n, uint64_t seed, double scale,
                                                 double* re, double* im) {
    if ((x >> n) & 1ull) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    const uint64_t r = (x & ((1ull << n) - 1ull)) | ((x >> (n + 1)) << n);
    double s, c;
    sincospi(2.0 * sm64_uniform(seed, r), &s, &c);      // phi = 2 pi u
    *re = c * scale;
    *im = s * scale;
}

// Amplitude of basis state x of the product state: site n up, every other
// site l in (|down> + exp(-i phi_l)|up>)/sqrt(2) with phi_l = 2 pi u(seed, l),
// so psi[x] = 2^-(M-1)/2 exp(-i 2 pi sum of u(seed, l) over the up sites l != n).
// `u` holds u(seed, l) for l < M (or is null: drawn here).
__device__ __forceinline__ void product_amp(uint64_t x, int M, int n, uint64_t seed,
                                            const double* u, double scale, double* re,
                                            double* im) {
    if ((x >> n) & 1ull) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    double acc = 0.0;
    for (int l = 0; l < M; ++l)
        if (l != n && !((x >> l) & 1ull)) acc += u ? u[l] : sm64_uniform(seed, uint64_t(l));
    acc -= floor(acc);               // the phase modulo 2 pi
    double s, c;
    sincospi(-2.0 * acc, &s, &c);
    *re = c * scale;
    *im = s * scale;
}

// Initial amplitude of basis state x: init 1 = the random-phase state,
// init 2 = the basis state |seed> (one ensemble member of Eq. (1)), init 3 =
// the product state of the random phases of `seed`.
__device__ __forceinline__ void init_amp(uint64_t x, int M, int init, int polarized, uint64_t seed,
                                         double scale, double* re, double* im) {
    if (init == 2) {
        *re = x == seed ? 1.0 : 0.0;
        *im = 0.0;
    } else if (init == 3) {
        product_amp(x, M, polarized, seed, nullptr, scale, re, im);
    } else {
        random_phase_amp(x, polarized, seed, scale, re, im);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init(typename CT<T>::c* __restrict__ psi, int M, int n,
                                              uint64_t seed, double scale) {
    const uint64_t dim = 1ull << M;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < dim; x += stride) {
        double re, im;
        random_phase_amp(x, n, seed, scale, &re, &im);
        typename CT<T>::c v;
        v.x = T(re);
        v.y = T(im);
        psi[x] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_product(typename CT<T>::c* __restrict__ psi, int M,
                                                      int n, uint64_t seed, double scale) {
    __shared__ double u[64];
    if (threadIdx.x < 64) u[threadIdx.x] = sm64_uniform(seed, threadIdx.x);
    __syncthreads();
    const uint64_t dim = 1ull << M;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < dim; x += stride) {
        double re, im;
        product_amp(x, M, n, seed, u, scale, &re, &im);
        typename CT<T>::c v;
        v.x = T(re);
        v.y = T(im);
        psi[x] = v;
    }
}

// Ensemble members stacked as one state of M + cbits sites: amplitude
// x = (m << M) | y is 1 when m < count and y is the basis state of member
// first + m (its bits spread over the sites other than `polarized`, whose
// bit is 0: spin up), and 0 otherwise.
template <typename T>
__global__ __launch_bounds__(256) void k_init_members(typename CT<T>::c* __restrict__ psi, int M,
                                                      int cbits, int polarized, uint64_t first,
                                                      uint64_t count) {
    const uint64_t dim = 1ull << (M + cbits);
    const uint64_t ymask = (1ull << M) - 1;
    const uint64_t low = (1ull << polarized) - 1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < dim; x += stride) {
        const uint64_t m = x >> M;
        const uint64_t r = first + m;
        const uint64_t basis = ((r & ~low) << 1) | (r & low);
        typename CT<T>::c v;
        v.x = T((m < count && (x & ymask) == basis) ? 1 : 0);
        v.y = T(0);
        psi[x] = v;
    }
}

// acc[i] = (acc[i] + add[i]) * scale (add may be null), i < n.
__global__ void k_accumulate(double* __restrict__ acc, const double* __restrict__ add, int64_t n,
                             double scale) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        acc[i] = (acc[i] + (add ? add[i] : 0.0)) * scale;
}

// ---------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of (p, n) over the workgroup, fixed order; result valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum2(double& p, double& n, double* red) {
    p = wave_sum(p);
    n = wave_sum(n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wave] = p;
        red[2 * wave + 1] = n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sp = 0.0, sn = 0.0;
        for (int w = 0; w < (NT + 63) / 64; ++w) {
            sp += red[2 * w];
            sn += red[2 * w + 1];
        }
        p = sp;
        n = sn;
    }
    __syncthreads();
}

// Workgroup sum of v (result valid in thread 0).
template <int NT>
__device__ __forceinline__ double block_sum1(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (NT + 63) / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Profile partials [slot][nwg][M + 1] -> Pall[s * M + site], N[s]; one
// workgroup per (step, site or norm).
__global__ __launch_bounds__(256) void k_reduce_profile(const double* __restrict__ partials, int nwg,
                                                        int ch, int M, int64_t s0,
                                                        double* __restrict__ Pall,
                                                        double* __restrict__ N) {
    __shared__ double red[8];
    const int64_t s = s0 + blockIdx.x / (M + 1);
    const int site = int(blockIdx.x % (M + 1));
    const double* src = partials + (size_t)(s % ch) * nwg * (M + 1);
    double v = 0.0;
    for (int w = threadIdx.x; w < nwg; w += 256) v += src[(size_t)w * (M + 1) + site];
    v = block_sum1<256>(v, red);
    if (threadIdx.x == 0) {
        if (site < M) Pall[s * M + site] = v;
        else if (N) N[s] = v;
    }
}

// partials: [slot][nwg][2]; P/N for steps s0..s1-1, slot = s % ch.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int nwg, int ch,
                                                int64_t s0, double* __restrict__ P,
                                                double* __restrict__ N) {
    __shared__ double red[8];
    const int64_t s = s0 + blockIdx.x;
    const double* base = partials + (size_t)(s % ch) * nwg * 2;
    double p = 0.0, n = 0.0;
    for (int w = threadIdx.x; w < nwg; w += 256) {
        p += base[2 * w];
        n += base[2 * w + 1];
    }
    block_sum2<256>(p, n, red);
    if (threadIdx.x == 0) {
        P[s] = p;
        if (N) N[s] = n;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_observe(const typename CT<T>::c* __restrict__ psi, int M,
                                                 int site, double* __restrict__ partials) {
    __shared__ double red[8];
    const uint64_t dim = 1ull << M;
    const uint64_t stride = uint64_t(gridDim.x) * 256;
    double p = 0.0, n = 0.0;
    for (uint64_t x = uint64_t(blockIdx.x) * 256 + threadIdx.x; x < dim; x += stride) {
        const typename CT<T>::c v = psi[x];
        const double w = double(v.x) * double(v.x) + double(v.y) * double(v.y);
        n += w;
        p += ((x >> site) & 1ull) ? -w : w;
    }
    block_sum2<256>(p, n, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = p;
        partials[2 * blockIdx.x + 1] = n;
    }
}

// ------------------------------------------------------ unfused factor
// exp(-i tau H_ij) over the whole state; lane = one anti-aligned pair.
template <typename T>
__global__ __launch_bounds__(256) void k_factor(typename CT<T>::c* __restrict__ psi, int M, int lo,
                                                int hi, T t, T s, T pr, T pim, int zz) {
    using C = typename CT<T>::c;
    const uint64_t npairs = 1ull << (M - 2);
    const uint64_t stride = uint64_t(gridDim.x) * 256;
    for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npairs; p += stride) {
        uint64_t x = p;
        x = ((x >> lo) << (lo + 1)) | (x & ((1ull << lo) - 1ull));
        x = ((x >> hi) << (hi + 1)) | (x & ((1ull << hi) - 1ull));
        const uint64_t xa = x | (1ull << hi), xb = x | (1ull << lo);
        C a = psi[xa], b = psi[xb];
        // (a_re, b_im) rotate by [[c, s], [-s, c]]; (a_im, b_re) by [[c, -s], [s, c]]
        T u = a.x, v = b.y;
        u = fma(t, v, u); v = fma(-s, u, v); u = fma(t, v, u);
        a.x = u; b.y = v;
        u = a.y; v = b.x;
        u = fma(-t, v, u); v = fma(s, u, v); u = fma(-t, v, u);
        a.y = u; b.x = v;
        if (zz) {
            C a2, b2;
            a2.x = pr * a.x - pim * a.y; a2.y = pr * a.y + pim * a.x;
            b2.x = pr * b.x - pim * b.y; b2.y = pr * b.y + pim * b.x;
            a = a2; b = b2;
            C c0 = psi[x], c1 = psi[x | (1ull << lo) | (1ull << hi)];
            C d0, d1;
            d0.x = pr * c0.x + pim * c0.y; d0.y = pr * c0.y - pim * c0.x;
            d1.x = pr * c1.x + pim * c1.y; d1.y = pr * c1.y - pim * c1.x;
            psi[x] = d0;
            psi[x | (1ull << lo) | (1ull << hi)] = d1;
        }
        psi[xa] = a;
        psi[xb] = b;
    }
}

// ------------------------------------------------------- register ops
// Rotation of the anti-aligned pairs (bit A, bit B) = (0, 1) <-> (1, 0) of
// the register index: psi_x <- c psi_x - i s psi_y, psi_y <- -i s psi_x + c psi_y,
// done as two real three-shear rotations (exactly area preserving):
// (Re x, Im y) by [[c, s], [-s, c]] and (Im x, Re y) by [[c, -s], [s, c]],
// each as u += t v; v -= s u; u += t v with t = tan(theta/2).
template <int R, int A, int B, typename C, typename T>
__device__ __forceinline__ void reg_xy(C (&v)[1 << R], T t, T s) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (((j >> A) & 1) == 0 && ((j >> B) & 1) == 1) {
            const int k = j ^ (1 << A) ^ (1 << B);
            T u = v[j].x, w = v[k].y;
            u = fma(t, w, u); w = fma(-s, u, w); u = fma(t, w, u);
            v[j].x = u; v[k].y = w;
            u = v[j].y; w = v[k].x;
            u = fma(-t, w, u); w = fma(s, u, w); u = fma(-t, w, u);
            v[j].y = u; v[k].x = w;
        }
    }
}

// I^z I^z phase: anti-aligned amplitudes times (pr + i pi), aligned times
// its conjugate.
template <int R, int A, int B, typename C, typename T>
__device__ __forceinline__ void reg_zz(C (&v)[1 << R], T pr, T pim) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        const bool anti = ((j >> A) & 1) != ((j >> B) & 1);
        const T q = anti ? pim : -pim;
        const T x = v[j].x, y = v[j].y;
        v[j].x = fma(pr, x, -q * y);
        v[j].y = fma(pr, y, q * x);
    }
}

template <int R, typename C, typename T>
__device__ __forceinline__ void reg_op(C (&v)[1 << R], int code, T t, T s, T pr, T pim) {
#define SPIN_CASE(A, B)                                        \
    case A * 8 + B:                                            \
        if constexpr (B < R) {                                 \
            reg_xy<R, A, B>(v, t, s);                          \
            if (code & kOpZZ) reg_zz<R, A, B>(v, pr, pim);     \
        }                                                      \
        break;
    switch (code & 63) {
        SPIN_CASE(0, 1) SPIN_CASE(0, 2) SPIN_CASE(1, 2) SPIN_CASE(0, 3) SPIN_CASE(1, 3)
        SPIN_CASE(2, 3) SPIN_CASE(0, 4) SPIN_CASE(1, 4) SPIN_CASE(2, 4) SPIN_CASE(3, 4)
        SPIN_CASE(0, 5) SPIN_CASE(1, 5) SPIN_CASE(2, 5) SPIN_CASE(3, 5) SPIN_CASE(4, 5)
        default: break;
    }
#undef SPIN_CASE
}

// sum of (sign * |psi|^2, |psi|^2) over the lane's registers, FP64
template <int R, typename C>
__device__ __forceinline__ void reg_observe(const C (&v)[1 << R], int sign, int mask, double& p,
                                            double& n) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        const double w = double(v[j].x) * double(v[j].x) + double(v[j].y) * double(v[j].y);
        n += w;
        const int neg = sign ^ ((j & mask) ? 1 : 0);
        p += neg ? -w : w;
    }
}

// LDS byte address of the lane's register 0 in stage S (thread bits only;
// entries past the stage's thread bits are zero).
__device__ __forceinline__ uint32_t stage_base(const DevStage& S, int tid) {
    uint32_t b = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) b ^= S.tmask[q] & (0u - ((uint32_t(tid) >> q) & 1u));
    return b;
}

// Barrier for LDS traffic only: global loads in flight (the next tile's
// prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Ordering of a wave's own LDS scatter before its gather: the exchange
// moves amplitudes only between lanes of the wave, so no other wave reads
// the slots (LDS operations of one wave complete in issue order; the fences
// keep the compiler from moving the gather above the scatter).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Deposit of the bits of `x` into the set bits of `mask`, lowest first.
__device__ __forceinline__ int64_t deposit(int64_t x, int64_t mask) {
    int64_t out = 0;
    while (x && mask) {
        const int64_t low = mask & -mask;
        if (x & 1) out |= low;
        mask ^= low;
        x >>= 1;
    }
    return out;
}

// Next value, in increasing order, among the submasks of `mask`.
__device__ __forceinline__ int64_t next_submask(int64_t cur, int64_t mask) {
    return ((cur | ~mask) + 1) & mask;
}

// Gather / scatter of a lane's 2^R registers in Gray-code order: register
// j = i ^ (i >> 1) sits at pb ^ (xor of rbit[q] over the set bits q of j),
// and consecutive Gray codes differ in bit ctz(i).
template <int R, typename C, typename Stage>
__device__ __forceinline__ void gather(C (&v)[1 << R], const char* lds, uint32_t pb,
                                       const Stage& S) {
    uint32_t a = pb;
    v[0] = *reinterpret_cast<const C*>(lds + a);
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) {
        a ^= S.rbit[__builtin_ctz(i)];
        v[i ^ (i >> 1)] = *reinterpret_cast<const C*>(lds + a);
    }
}

template <int R, typename C, typename Stage>
__device__ __forceinline__ void scatter(const C (&v)[1 << R], char* lds, uint32_t pb,
                                        const Stage& S) {
    uint32_t a = pb;
    *reinterpret_cast<C*>(lds + a) = v[0];
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) {
        a ^= S.rbit[__builtin_ctz(i)];
        *reinterpret_cast<C*>(lds + a) = v[i ^ (i >> 1)];
    }
}

// Gather / scatter of the half of a lane's registers whose top register bit
// is H (the split position's value in a half-tile exchange), Gray-code order
// over the lower R - 1 register bits.  The split position has no LDS image:
// both halves use the same slots, one after the other.
template <int R, int H, typename C, typename Stage>
__device__ __forceinline__ void gather_half(C (&v)[1 << R], const char* lds, uint32_t pb,
                                            const Stage& S) {
    constexpr int B = 1 << (R - 1);
    uint32_t a = pb;
    v[H * B] = *reinterpret_cast<const C*>(lds + a);
#pragma unroll
    for (int i = 1; i < B; ++i) {
        a ^= S.rbit[__builtin_ctz(i)];
        v[H * B + (i ^ (i >> 1))] = *reinterpret_cast<const C*>(lds + a);
    }
}

template <int R, int H, typename C, typename Stage>
__device__ __forceinline__ void scatter_half(const C (&v)[1 << R], char* lds, uint32_t pb,
                                             const Stage& S) {
    constexpr int B = 1 << (R - 1);
    uint32_t a = pb;
    *reinterpret_cast<C*>(lds + a) = v[H * B];
#pragma unroll
    for (int i = 1; i < B; ++i) {
        a ^= S.rbit[__builtin_ctz(i)];
        *reinterpret_cast<C*>(lds + a) = v[H * B + (i ^ (i >> 1))];
    }
}

// Register offsets of a stage read into scalar registers together with its
// lane offsets (one round trip for both before the gather).
template <int R>
struct RegBits {
    uint32_t rbit[R];
};

// Runs ops from index o up to the stage end o1 or the next observable op
// (whichever comes first) on the lane's registers; returns the index of
// the first op not run.  Each op's record is loaded one op ahead.
template <int R, typename C, typename T>
__device__ __forceinline__ int run_factors(C (&v)[1 << R], const DevOp<T>* __restrict__ ops, int o,
                                           int o1) {
    if (o >= o1) return o;
    DevOp<T> cur = ops[o];
    while (cur.code != kOpMeas) {
        const int on = o + 1;
        const DevOp<T> nxt = ops[on < o1 ? on : o];
        reg_op<R>(v, cur.code, cur.t, cur.s, cur.pr, cur.pi);
        o = on;
        if (o >= o1) break;
        cur = nxt;
    }
    return o;
}

// ------------------------------------------------------- matrix engine
// Dense 32 x 32 complex matrix U on the 32 registers of every lane, as the
// real product Y = W X with X = (Re v_0..Re v_31, Im v_0..Im v_31) per lane
// (column) and W = [[Re U, -Im U], [Im U, Re U]], on v_mfma_f32_32x32x2f32.
// A wave holds 64 columns.  One v_permlane32_swap per pair of rows (2p,
// 2p+1) turns the lane-per-column registers into the instruction's B
// operands (lane l: row 2p + l/32 of column 32h + l%32, h = 0, 1); the A
// operands are read from the matrix table (lane l: W[32b + l%32][2p + l/32]).
// The accumulators hold Y[32b + 8(r/4) + 4(l/32) + r%4][32h + l%32] in
// register r; one swap per register pair of h = 0, 1 returns them to the
// lane-per-column layout.
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <typename C>
__device__ __forceinline__ float mat_row(const C (&v)[32], int m) {
    return m < 32 ? v[m].x : v[m - 32].y;
}
template <typename C>
__device__ __forceinline__ void mat_set(C (&v)[32], int m, float x) {
    if (m < 32) v[m].x = x;
    else v[m - 32].y = x;
}

template <typename C>
__device__ __forceinline__ void mfma_stage(C (&v)[32], const float* __restrict__ W) {
    const int lane = threadIdx.x & 63;
    float bop[64];
#pragma unroll
    for (int p = 0; p < 32; ++p) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(mat_row(v, 2 * p)),
                                                        __float_as_uint(mat_row(v, 2 * p + 1)),
                                                        false, false);
        bop[2 * p] = __uint_as_float(r[0]);
        bop[2 * p + 1] = __uint_as_float(r[1]);
    }
    f32x16 d00 = {}, d01 = {}, d10 = {}, d11 = {};
#pragma unroll
    for (int p = 0; p < 32; ++p) {
        const float a0 = W[p * 64 + lane], a1 = W[(32 + p) * 64 + lane];
        d00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bop[2 * p], d00, 0, 0, 0);
        d01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bop[2 * p + 1], d01, 0, 0, 0);
        d10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bop[2 * p], d10, 0, 0, 0);
        d11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bop[2 * p + 1], d11, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + r % 4;
        const auto s0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(d00[r]), __float_as_uint(d01[r]),
                                                         false, false);
        mat_set(v, row, __uint_as_float(s0[0]));
        mat_set(v, row + 4, __uint_as_float(s0[1]));
        const auto s1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(d10[r]), __float_as_uint(d11[r]),
                                                         false, false);
        mat_set(v, 32 + row, __uint_as_float(s1[0]));
        mat_set(v, 32 + row + 4, __uint_as_float(s1[1]));
    }
}

template <typename C>
__device__ __forceinline__ C& lds_at(char* lds, uint32_t byte) {
    return *reinterpret_cast<C*>(lds + byte);
}

// ------------------------------------------------------------ tiled pass
// One pass over the tiles of a group of G workgroups (G a power of two):
// member w takes the tiles whose index is w' + i*G (w' = w in the group's
// order), i = 0 .. tiles_per_member-1.  The first register stage of a tile
// is loaded straight from HBM (lanes along the low address bits, so the
// wave's accesses are contiguous runs) and the last one stored straight
// back, in the pass's output layout; the stages in between exchange through
// LDS, with a workgroup barrier where the exchange moves amplitudes between
// waves and a wave-level ordering where it does not.  Every wave has
// consumed its loads of a tile before the first workgroup barrier, so the
// stores after it cannot overtake another wave's loads; a pass without such
// a barrier keeps its wave positions and their address bits from the first
// stage to the last, so each wave stores only addresses it loaded itself.  A
// one-stage pass never touches LDS: its lanes store exactly the addresses
// they loaded (the planner only makes one-stage passes that keep the
// layout).  The next tile is prefetched into registers while
// the current one is worked on.  Observables accumulate into accP/accN per
// measurement slot of the pass.
template <int R, typename C>
__device__ __forceinline__ void load_direct(C (&v)[1 << R], const C* __restrict__ psi, int64_t g,
                                            const int64_t* gr) {
    v[0] = psi[g];
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) {
        g ^= gr[__builtin_ctz(i)];
        v[i ^ (i >> 1)] = psi[g];
    }
}

template <int R, typename C>
__device__ __forceinline__ void store_direct(const C (&v)[1 << R], C* __restrict__ psi, int64_t g,
                                             const int64_t* gr) {
    psi[g] = v[0];
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) {
        g ^= gr[__builtin_ctz(i)];
        psi[g] = v[i ^ (i >> 1)];
    }
}

__device__ __forceinline__ int64_t lane_offset(const int64_t* gt, int tid) {
    int64_t o = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) o ^= gt[q] & (int64_t(0) - int64_t((uint32_t(tid) >> q) & 1u));
    return o;
}

// Wave sum of a double, valid in lane 63: DPP adds over pairs, quads,
// half rows, rows, then rows 0+1 into row 1 and 2+3 into row 3
// (row_bcast:15), then rows 0..1 into rows 2..3 (row_bcast:31).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
    const uint64_t b = uint64_t(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, ROW_MASK, 0xF, false);
    return v + __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// Squared magnitudes of the lane's 2^R registers in FP64: their total and,
// for each register bit b, the half sum over registers with bit b set.
// Pairwise: the sums over bit b's pairs feed bit b+1 (2^R - 1 adds for the
// total, 2^R - 1 - R for the half sums).
template <int R, typename C>
__device__ __forceinline__ void reg_half_sums(const C (&v)[1 << R], double& tot, double (&half)[R]) {
    double w[1 << R];
#pragma unroll
    for (int j = 0; j < (1 << R); ++j)
        w[j] = double(v[j].x) * double(v[j].x) + double(v[j].y) * double(v[j].y);
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int n = (1 << R) >> (b + 1);    // pairs at this level
        double h = w[1];
#pragma unroll
        for (int i = 1; i < n; ++i) h += w[2 * i + 1];
        half[b] = h;
#pragma unroll
        for (int i = 0; i < n; ++i) w[i] = w[2 * i] + w[2 * i + 1];
    }
    tot = w[0];
}

// Same sums accumulated one register at a time (fewer live registers, more
// adds), for kernels that share the CU with a second workgroup.
template <int R, typename C>
__device__ __forceinline__ void reg_half_sums_seq(const C (&v)[1 << R], double& tot, double (&half)[R]) {
    tot = 0.0;
#pragma unroll
    for (int b = 0; b < R; ++b) half[b] = 0.0;
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        const double w = double(v[j].x) * double(v[j].x) + double(v[j].y) * double(v[j].y);
        tot += w;
#pragma unroll
        for (int b = 0; b < R; ++b)
            if ((j >> b) & 1) half[b] += w;
    }
}

__device__ __forceinline__ double wave_sum_last(double v) {
    v = dpp_add<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xF>(v);    // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);    // row_mirror
    v = dpp_add<0x142, 0xA>(v);    // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xC>(v);    // row_bcast:31 into rows 2, 3
    return v;
}

// One per-site observable (profile kOpMeas) of the lane's registers: the
// sign of each amplitude follows the site's bit (thread bit, register bit or
// a bit of the tile base).
template <int R, typename C>
__device__ __forceinline__ void prof_observe(const C (&v)[1 << R], int aux, int64_t base,
                                             double& p, double& n, int& slot, int& nslot) {
    slot = aux & 63;
    const int kind = (aux >> 6) & 3, idx = (aux >> 8) & 63;
    nslot = ((aux >> 14) & 7) - 1;
    const int sign = kind == 0 ? ((int(threadIdx.x) >> idx) & 1)
                   : kind == 2 ? int((base >> idx) & 1) : 0;
    const int mask = kind == 1 ? (1 << idx) : 0;
    p = 0.0;
    n = 0.0;
    reg_observe<R>(v, sign, mask, p, n);
}

template <typename T, int R, int NT, bool WRITES, int ENGINE = 0, bool PROFILE = false,
          bool HALF = false>
__device__ __forceinline__ void pass_tiles(typename CT<T>::c* __restrict__ psi, const DevPass& P,
                                           const DevStage* __restrict__ stages,
                                           const DevOp<T>* __restrict__ ops, unsigned wperm,
                                           unsigned G, int64_t tiles_per_member, char* ldsb,
                                           double (&accP)[kMaxMeas], double (&accN)[kMaxMeas],
                                           const float* __restrict__ mats = nullptr,
                                           double* pacc = nullptr, double* nacc = nullptr) {
    using C = typename CT<T>::c;
    const int tid = threadIdx.x;
    const DevStage& S0 = stages[P.stage0];
    const DevStage& SL = stages[P.stage0 + P.nstage - 1];
    const int64_t gin_t = lane_offset(S0.gt_in, tid);
    const int64_t gout_t = lane_offset(SL.gt_out, tid);

    // Tile bases: tile = wperm + i * G, so base = deposit(wperm) | (i-th
    // submask of the free bits above the lowest log2(G) ones).
    const int64_t base_w = deposit(wperm, P.free_mask);
    int64_t m_hi = P.free_mask;
    for (unsigned g = G; g > 1; g >>= 1) m_hi &= m_hi - 1;

    // Full-tile exchanges: the next tile's loads are issued into `pre` at
    // the start of a tile and always (the last tile re-reads itself), so
    // every iteration ends with the same memory ops outstanding -- prefetch
    // loads, then stores -- and the copy out of `pre` only waits for the
    // loads.  Half-tile exchanges leave room for a second workgroup on the
    // CU instead of a prefetch: a tile's loads go straight into `v` and the
    // other workgroup's work covers their latency.
    C pre[HALF ? 1 : (1 << R)];
    int64_t hi = 0;
    if constexpr (!HALF) load_direct<R>(pre, psi, base_w + gin_t, S0.gr_in);

    auto tile_body = [&](int64_t it_tile) {
        const int64_t base = base_w | hi;
        const int tile_sign = P.obs_free_bit >= 0 ? int((base >> P.obs_free_bit) & 1) : 0;
        C v[1 << R];
        if constexpr (HALF) {
            load_direct<R>(v, psi, base + gin_t, S0.gr_in);
            if (it_tile + 1 < tiles_per_member) hi = next_submask(hi, m_hi);
        } else {
#pragma unroll
            for (int j = 0; j < (1 << R); ++j) v[j] = pre[j];
            if (it_tile + 1 < tiles_per_member) hi = next_submask(hi, m_hi);
            load_direct<R>(pre, psi, (base_w | hi) + gin_t, S0.gr_in);
        }

        for (int si = 0; si < P.nstage; ++si) {
            const DevStage& S = stages[P.stage0 + si];
            RegBits<R> rb;
#pragma unroll
            for (int b = 0; b < R; ++b) rb.rbit[b] = S.rbit[b];
            const uint32_t pb = stage_base(S, tid);
            if constexpr (!HALF)
                if (si > 0) gather<R>(v, ldsb, pb, rb);
            const int sign = tile_sign ^ (S.obs_tq >= 0 ? ((tid >> S.obs_tq) & 1) : 0);
            const int o1 = S.op0 + S.nop;
            int o = S.op0;
            while (o < o1) {
                if constexpr (ENGINE == 1) {
                    const DevOp<T> op = ops[o];
                    if (op.code == kOpMat) {
                        if constexpr (sizeof(T) == 4 && R == 5) mfma_stage(v, mats + size_t(op.aux) * kMatFloats);
                        ++o;
                        continue;
                    }
                } else {
                    o = run_factors<R>(v, ops, o, o1);
                }
                if (o < o1) {    // observable of the state at this point
                    if constexpr (PROFILE) {
                        // Every per-site observable at this point from the
                        // lane's total weight and its register-bit half sums,
                        // each squared once; wave sums go to the wave's LDS
                        // row (pacc / nacc), one row per wave.
                        double tot, half[R];
                        if constexpr (HALF) reg_half_sums_seq<R>(v, tot, half);
                        else reg_half_sums<R>(v, tot, half);
                        const bool last = (tid & 63) == 63;
                        while (o < o1 && ops[o].code == kOpMeas) {
                            const int aux = ops[o].aux;
                            const int slot = aux & 63, kind = (aux >> 6) & 3, idx = (aux >> 8) & 63;
                            const int nslot = ((aux >> 14) & 7) - 1;
                            double p;
                            if (kind == 1) {
                                double h = half[0];
#pragma unroll
                                for (int b = 1; b < R; ++b)
                                    if (b == idx) h = half[b];
                                p = tot - 2.0 * h;
                            } else {
                                const int neg = kind == 0 ? ((tid >> idx) & 1) : int((base >> idx) & 1);
                                p = neg ? -tot : tot;
                            }
                            p = wave_sum_last(p);
                            if (last) pacc[slot] += p;
                            if (nslot >= 0) {
                                const double n = wave_sum_last(tot);
                                if (last) nacc[nslot] += n;
                            }
                            ++o;
                        }
                        continue;
                    } else if constexpr (HALF) {
                        // wave sums into the wave's own LDS row (pacc: slot
                        // m holds P at 2m, N at 2m + 1), no accumulator
                        // registers
                        const int slot = ops[o].aux;
                        double p = 0.0, n = 0.0;
                        reg_observe<R>(v, sign, S.obs_mask, p, n);
                        p = wave_sum_last(p);
                        n = wave_sum_last(n);
                        if ((tid & 63) == 63) {
                            pacc[2 * slot] += p;
                            pacc[2 * slot + 1] += n;
                        }
                    } else {
                        const int slot = ops[o].aux;
                        double p = 0.0, n = 0.0;
                        reg_observe<R>(v, sign, S.obs_mask, p, n);
#pragma unroll
                        for (int m = 0; m < kMaxMeas; ++m)
                            if (m == slot) { accP[m] += p; accN[m] += n; }
                    }
                    ++o;
                }
            }
            if (si + 1 < P.nstage) {
                // A lane scatters to exactly the LDS slots the next stage's
                // lanes gather after the barrier.  When both stages keep the
                // same positions on the wave bits, those slots belong to the
                // wave's own lanes and only the wave is ordered.
                const bool xw = S.xnext != 0;
                auto sync = [&]() {
                    if (xw) lds_barrier();
                    else wave_lds_sync();
                };
                if constexpr (HALF) {
                    // The split position stays on the top register bit:
                    // half 0 through the LDS, then half 1 through the same
                    // slots.  A lane's gather slots in the next stage are its
                    // scatter slots there, so the next exchange needs no
                    // ordering before its first scatter; inside this one the
                    // second scatter waits for every first gather.
                    const DevStage& S2 = stages[P.stage0 + si + 1];
                    RegBits<R> rb2;
#pragma unroll
                    for (int b = 0; b < R; ++b) rb2.rbit[b] = S2.rbit[b];
                    const uint32_t pb2 = stage_base(S2, tid);
                    scatter_half<R, 0>(v, ldsb, pb, rb);
                    sync();
                    gather_half<R, 0>(v, ldsb, pb2, rb2);
                    sync();
                    scatter_half<R, 1>(v, ldsb, pb, rb);
                    sync();
                    gather_half<R, 1>(v, ldsb, pb2, rb2);
                } else {
                    scatter<R>(v, ldsb, pb, rb);
                    sync();
                }
            }
        }
        if constexpr (WRITES) store_direct<R>(v, psi, base + gout_t, SL.gr_out);
        // the last gathers are done before the next tile's scatters, unless
        // the last and first stages keep the same wave positions (then every
        // wave's slots are its own across the tile boundary)
        if (P.tile_barrier) lds_barrier();
    };
    tile_body(0);
    for (int64_t it_tile = 1; it_tile < tiles_per_member; ++it_tile) tile_body(it_tile);
}

// Workgroup sum of measurement slot m of the accumulators (thread 0).
template <int NT>
__device__ __forceinline__ void slot_sum(const double (&accP)[kMaxMeas],
                                         const double (&accN)[kMaxMeas], int m, double* red,
                                         double& p, double& n) {
    p = accP[0];
    n = accN[0];
#pragma unroll
    for (int mm = 1; mm < kMaxMeas; ++mm)
        if (mm == m) { p = accP[mm]; n = accN[mm]; }
    block_sum2<NT>(p, n, red);
}

// --------------------------------------------------------------- k_pass
// partials: [slot][nwg][2] (P, N), or with PROFILE [slot][nwg][M + 1] (P of
// every site, then N).
// HALF: half-tile exchanges, LDS for half a tile, no register prefetch, and
// registers capped so that two workgroups share a CU.
// Waves per SIMD a half-tile pass kernel is built for: two workgroups per
// CU when their half-tile LDS buffers fit the CU's 160 KiB together (with
// room for the small arrays), else one (complex128 tiles of 2^14).
template <typename T, int R, int NT>
__host__ __device__ constexpr int half_waves_per_eu() {
    return ((sizeof(typename CT<T>::c) << (R + __builtin_ctz(NT) - 1)) <= 72 * 1024 ? 2 : 1) * NT / 256;
}

template <typename T, int R, int NT, bool WRITES, int ENGINE, bool PROFILE, bool HALF>
__global__ __launch_bounds__(NT, (HALF ? half_waves_per_eu<T, R, NT>() : 1)) void k_pass(typename CT<T>::c* __restrict__ psi,
                                             const DevPass* __restrict__ passes,
                                             const DevStage* __restrict__ stages,
                                             const DevOp<T>* __restrict__ ops, int pass_index,
                                             int64_t tiles_per_wg, double* __restrict__ partials,
                                             int64_t step_offset, int ch, int nwg,
                                             const float* __restrict__ mats) {
    using C = typename CT<T>::c;
    constexpr int K = R + __builtin_ctz(NT);
    __shared__ C lds[HALF ? (1 << (K - 1)) : (1 << K)];
    __shared__ double red[2 * (NT / 64)];
    const DevPass& P = passes[pass_index];
    double accP[kMaxMeas], accN[kMaxMeas];
#pragma unroll
    for (int m = 0; m < kMaxMeas; ++m) accP[m] = accN[m] = 0.0;
    // XCD-aware order: workgroups are dispatched round-robin over the 8
    // XCDs, so w and w + 8 share an L2.  They take adjacent tile indices,
    // i.e. tiles that differ only in the lowest non-tile address bit and so
    // share cache lines when the tile's contiguous runs are shorter than a
    // line.
    const unsigned G = gridDim.x, w = blockIdx.x;
    const unsigned wperm = (G >= 8) ? (w % 8u) * (G / 8u) + w / 8u : w;
    if constexpr (PROFILE) {
        // Per-wave accumulator rows; lane 63 of each wave owns its row.
        constexpr int NW = NT / 64;
        __shared__ double pacc[NW][kMaxMeasProfile];
        __shared__ double nacc[NW][kMaxMeas];
        const int wave = threadIdx.x / 64;
        if ((threadIdx.x & 63) == 63) {
            for (int m = 0; m < kMaxMeasProfile; ++m) pacc[wave][m] = 0.0;
            for (int m = 0; m < kMaxMeas; ++m) nacc[wave][m] = 0.0;
        }
        pass_tiles<T, R, NT, WRITES, ENGINE, true, HALF>(psi, P, stages, ops, wperm, G, tiles_per_wg,
                                                         reinterpret_cast<char*>(lds), accP, accN, mats,
                                                         pacc[wave], nacc[wave]);
        __syncthreads();
        const int M = P.k + P.nfree;
        auto dst = [&](int64_t step) {
            return partials + ((size_t)((step_offset + step) % ch) * nwg + blockIdx.x) * (M + 1);
        };
        // fixed-order sums over the waves
        for (int m = threadIdx.x; m < P.pmeas; m += NT) {
            double v = 0.0;
            for (int w = 0; w < NW; ++w) v += pacc[w][m];
            dst(P.pmeas_step[m])[P.pmeas_site[m]] = v;
        }
        if (threadIdx.x >= NT - kMaxMeas) {
            const int m = threadIdx.x - (NT - kMaxMeas);
            if (m < P.pnorm) {
                double v = 0.0;
                for (int w = 0; w < NW; ++w) v += nacc[w][m];
                dst(P.pmeas_step[P.pnorm_meas[m]])[M] = v;
            }
        }
        return;
    }
    if constexpr (HALF) {
        // per-wave observable rows; fixed-order sum over the waves
        constexpr int NW = NT / 64;
        __shared__ double wacc[NW][2 * kMaxMeas];
        const int wave = threadIdx.x / 64;
        if ((threadIdx.x & 63) == 63)
            for (int m = 0; m < 2 * kMaxMeas; ++m) wacc[wave][m] = 0.0;
        pass_tiles<T, R, NT, WRITES, ENGINE, false, true>(psi, P, stages, ops, wperm, G, tiles_per_wg,
                                                          reinterpret_cast<char*>(lds), accP, accN,
                                                          mats, wacc[wave]);
        __syncthreads();
        if (threadIdx.x < P.nmeas) {
            const int m = threadIdx.x;
            double p = 0.0, n = 0.0;
            for (int w = 0; w < NW; ++w) {
                p += wacc[w][2 * m];
                n += wacc[w][2 * m + 1];
            }
            const int64_t s = step_offset + P.meas_step[m];
            double* dst = partials + ((size_t)(s % ch) * nwg + blockIdx.x) * 2;
            dst[0] = p;
            dst[1] = n;
        }
        return;
    }
    pass_tiles<T, R, NT, WRITES, ENGINE, false, false>(psi, P, stages, ops, wperm, G, tiles_per_wg,
                                                       reinterpret_cast<char*>(lds), accP, accN, mats);
    for (int m = 0; m < P.nmeas; ++m) {
        double p, n;
        slot_sum<NT>(accP, accN, m, red, p, n);
        if (threadIdx.x == 0) {
            const int64_t s = step_offset + P.meas_step[m];
            double* dst = partials + ((size_t)(s % ch) * nwg + blockIdx.x) * 2;
            dst[0] = p;
            dst[1] = n;
        }
    }
}

// ------------------------------------------------------------ resident run
// One workgroup owns one whole state (2^M <= NT << R amplitudes) in LDS and
// runs the prologue stages once and the step stages n_steps times, writing
// P[k], N[k] itself.
template <typename T, int R, int NT, bool PROFILE = false>
__device__ __forceinline__ void resident_run(const ResidentJob& J, const DevStage* __restrict__ stages,
                                             const DevOp<T>* __restrict__ ops, int64_t n_steps,
                                             typename CT<T>::c* lds, double* red) {
    using C = typename CT<T>::c;
    constexpr int EB = sizeof(C);
    const int tid = threadIdx.x;
    const int M = J.M;
    const uint32_t dim = 1u << M;
    const int nact = (M >= R) ? (1 << (M - R)) : 1;
    C* psi = reinterpret_cast<C*>(J.psi);
    char* ldsb = reinterpret_cast<char*>(lds);
    if (J.init) {
        const double scale = 1.0 / sqrt(ldexp(1.0, M - 1));
        for (uint32_t x = tid; x < dim; x += NT) {
            double re, im;
            init_amp(x, M, J.init, J.polarized, J.seed, scale, &re, &im);
            C c;
            c.x = T(re);
            c.y = T(im);
            lds[lds_swizzle<EB>(x)] = c;
        }
    } else {
        for (uint32_t x = tid; x < dim; x += NT) lds[lds_swizzle<EB>(x)] = psi[x];
    }
    __syncthreads();

    auto run = [&](int st0, int nst, int64_t step) {
        for (int si = st0; si < st0 + nst; ++si) {
            const DevStage& S = stages[si];
            // Lanes past the state's size shadow an active lane (same LDS
            // slots) so that the op loop below stays free of divergence;
            // they never scatter and contribute nothing to observables.
            const bool act = tid < nact;
            const uint32_t pb = stage_base(S, tid & (nact - 1));
            C v[1 << R];
            gather<R>(v, ldsb, pb, S);
            const int sign = S.obs_tq >= 0 ? ((tid >> S.obs_tq) & 1) : 0;
            const int o1 = S.op0 + S.nop;
            int o = S.op0;
            while (o < o1) {
                o = run_factors<R>(v, ops, o, o1);
                if (o < o1) {    // observable: reduce over the workgroup now
                    if constexpr (PROFILE) {
                        const int aux = ops[o].aux;
                        double p, n;
                        int slot, nslot;
                        prof_observe<R>(v, aux, 0, p, n, slot, nslot);
                        p = act ? p : 0.0;
                        n = act ? n : 0.0;
                        block_sum2<NT>(p, n, red);
                        if (tid == 0) {
                            J.Pall[step * M + ((aux >> 17) & 63)] = p;
                            if (nslot >= 0 && J.N) J.N[step] = n;
                        }
                    } else {
                        double p = 0.0, n = 0.0;
                        reg_observe<R>(v, sign, S.obs_mask, p, n);
                        p = act ? p : 0.0;
                        n = act ? n : 0.0;
                        block_sum2<NT>(p, n, red);
                        if (tid == 0) {
                            J.P[step] = p;
                            if (J.N) J.N[step] = n;
                        }
                    }
                    ++o;
                }
            }
            __syncthreads();    // every shadow lane has gathered
            if (act) scatter<R>(v, ldsb, pb, S);
            __syncthreads();
        }
    };
    run(J.pro_stage0, J.pro_nstage, 0);
    for (int64_t k = 1; k <= n_steps; ++k) run(J.step_stage0, J.step_nstage, k);

    for (uint32_t x = tid; x < dim; x += NT) psi[x] = lds[lds_swizzle<EB>(x)];
    __syncthreads();
}

template <typename T, int R, int NT, bool PROFILE>
__global__ __launch_bounds__(NT) void k_resident(ResidentJob job0,
                                                 const ResidentJob* __restrict__ jobs,
                                                 const DevStage* __restrict__ stages,
                                                 const DevOp<T>* __restrict__ ops,
                                                 int64_t n_steps) {
    using C = typename CT<T>::c;
    __shared__ C lds[NT << R];
    __shared__ double red[2 * ((NT + 63) / 64)];
    const ResidentJob J = jobs ? jobs[blockIdx.x] : job0;
    resident_run<T, R, NT, PROFILE>(J, stages, ops, n_steps, lds, red);
}

// ---------------------------------------------------------------- k_batch
// Persistent batch: each workgroup runs its list of jobs in order.  A job
// is a whole problem held in LDS (gang size 1, M <= tile bits), or one
// member's share of a problem run as tiled passes by a gang of G
// workgroups that meet at a counter after every pass.  The host orders all
// job lists consistently (a global order of gang start times), so every
// wait is on members busy with earlier jobs: no cycle, no deadlock.  Each
// wait is bounded; on time-out the problem is flagged and its P set to NaN.
// Waits at most kGangWaitTicks of the 100 MHz real-time counter, and gives
// up at once when any workgroup has flagged an error.
constexpr uint64_t kGangWaitTicks = 20ull * 100000000ull;   // 20 s

__device__ __forceinline__ bool gang_barrier(int* counter, int target, int* err) {
    // release: this workgroup's global stores, visible device-wide
    __threadfence();
    __syncthreads();
    __shared__ int ok_s;
    if (threadIdx.x == 0) {
        int ok = 1;
        atomicAdd(counter, 1);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(4);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                wall_clock64() - t0 > kGangWaitTicks) {
                atomicOr(err, 1);
                ok = 0;
                break;
            }
        }
        __threadfence();    // acquire
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

// HALF: gangs run half-tile passes and two workgroups share a CU, so
// problems held in LDS are limited to half a tile.
template <typename T, int R, int NT, bool HALF>
__global__ __launch_bounds__(NT, HALF ? 2 * NT / 256 : 1) void k_batch(const BatchProblem* __restrict__ probs,
                                              const BatchJob* __restrict__ jobs,
                                              const int* __restrict__ job_start,
                                              const DevPass* __restrict__ passes,
                                              const DevStage* __restrict__ stages,
                                              const DevOp<T>* __restrict__ ops,
                                              const int2* __restrict__ launches,
                                              double* __restrict__ partials,
                                              int* __restrict__ counters, int* __restrict__ err,
                                              int64_t n_steps) {
    using C = typename CT<T>::c;
    constexpr int K = R + __builtin_ctz(NT);
    constexpr int KL = HALF ? K - 1 : K;    // largest problem held in LDS
    constexpr int NW = NT / 64;
    __shared__ C lds[1 << KL];
    __shared__ double red[2 * NW];
    __shared__ double wacc[HALF ? NW : 1][2 * kMaxMeas];
    const int tid = threadIdx.x;
    const int wave = tid / 64;
    for (int jb = job_start[blockIdx.x]; jb < job_start[blockIdx.x + 1]; ++jb) {
        const BatchJob job = jobs[jb];
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        const BatchProblem& B = probs[job.problem];
        if (B.gsize == 1 && B.M <= KL) {
            ResidentJob J{};
            J.psi = B.psi;
            J.P = B.P;
            J.N = B.N;
            J.seed = B.seed;
            J.M = B.M;
            J.polarized = B.polarized;
            J.init = B.init;
            J.pro_stage0 = B.pro_stage0;
            J.pro_nstage = B.pro_nstage;
            J.step_stage0 = B.step_stage0;
            J.step_nstage = B.step_nstage;
            resident_run<T, R, NT>(J, stages, ops, n_steps, lds, red);
            continue;
        }
        // gang member `rank` of `gsize`
        C* psi = reinterpret_cast<C*>(B.psi);
        const unsigned G = unsigned(B.gsize), rank = unsigned(job.rank);
        int* ctr = counters + B.counter;
        int epoch = 0;
        bool ok = true;
        if (B.init) {
            const uint64_t dim = 1ull << B.M;
            const double scale = 1.0 / sqrt(ldexp(1.0, B.M - 1));
            for (uint64_t x = uint64_t(rank) * NT + tid; x < dim; x += uint64_t(G) * NT) {
                double re, im;
                init_amp(x, B.M, B.init, B.polarized, B.seed, scale, &re, &im);
                C c;
                c.x = T(re);
                c.y = T(im);
                psi[x] = c;
            }
            ok = gang_barrier(ctr, ++epoch * int(G), err);
        }
        const int64_t tpm = B.ntiles / G;
        for (int l = 0; l < B.nlaunch && ok; ++l) {
            const int2 la = launches[B.launch0 + l];
            const DevPass& P = passes[B.pass0 + la.x];
            double accP[kMaxMeas], accN[kMaxMeas];
#pragma unroll
            for (int m = 0; m < kMaxMeas; ++m) accP[m] = accN[m] = 0.0;
            if constexpr (HALF) {
                // per-wave observable rows (as k_pass), summed over the
                // waves in a fixed order; the previous pass's reads of the
                // rows finished before the gang barrier
                if ((tid & 63) == 63)
                    for (int m = 0; m < 2 * kMaxMeas; ++m) wacc[wave][m] = 0.0;
                if (P.writes)
                    pass_tiles<T, R, NT, true, 0, false, true>(psi, P, stages, ops, rank, G, tpm,
                                                               reinterpret_cast<char*>(lds), accP, accN,
                                                               nullptr, wacc[wave]);
                else
                    pass_tiles<T, R, NT, false, 0, false, true>(psi, P, stages, ops, rank, G, tpm,
                                                                reinterpret_cast<char*>(lds), accP, accN,
                                                                nullptr, wacc[wave]);
                __syncthreads();
                if (tid < P.nmeas) {
                    const int m = tid;
                    double p = 0.0, n = 0.0;
                    for (int w = 0; w < NW; ++w) {
                        p += wacc[w][2 * m];
                        n += wacc[w][2 * m + 1];
                    }
                    const int64_t s = int64_t(la.y) + P.meas_step[m];
                    double* dst = partials + B.part0 + ((s % kBatchRing) * G + rank) * 2;
                    dst[0] = p;
                    dst[1] = n;
                }
            } else {
                if (P.writes)
                    pass_tiles<T, R, NT, true>(psi, P, stages, ops, rank, G, tpm,
                                               reinterpret_cast<char*>(lds), accP, accN);
                else
                    pass_tiles<T, R, NT, false>(psi, P, stages, ops, rank, G, tpm,
                                                reinterpret_cast<char*>(lds), accP, accN);
                for (int m = 0; m < P.nmeas; ++m) {
                    double p, n;
                    slot_sum<NT>(accP, accN, m, red, p, n);
                    if (tid == 0) {
                        const int64_t s = int64_t(la.y) + P.meas_step[m];
                        double* dst = partials + B.part0 + ((s % kBatchRing) * G + rank) * 2;
                        dst[0] = p;
                        dst[1] = n;
                    }
                }
            }
            ok = gang_barrier(ctr, ++epoch * int(G), err);
            if (rank == 0 && tid == 0 && ok) {
                for (int m = 0; m < P.nmeas; ++m) {
                    const int64_t s = int64_t(la.y) + P.meas_step[m];
                    const double* src = partials + B.part0 + (s % kBatchRing) * G * 2;
                    double p = 0.0, n = 0.0;
                    for (unsigned r = 0; r < G; ++r) {
                        p += src[2 * r];
                        n += src[2 * r + 1];
                    }
                    B.P[s] = p;
                    if (B.N) B.N[s] = n;
                }
            }
        }
        if (!ok && rank == 0 && tid == 0)
            for (int64_t s = 0; s <= n_steps; ++s) B.P[s] = __builtin_nan("");
    }
}

__global__ void k_fill_int(int* p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Folds a launch's error flag into the device's sticky batch status word.
__global__ void k_status_or(const int* err, int* status) {
    if (threadIdx.x == 0 && *err != 0) atomicOr(status, *err);
}

// ------------------------------------------------------------- launchers
static inline int grid_for(uint64_t n, int per_block, int cap) {
    uint64_t g = (n + per_block - 1) / per_block;
    if (g > uint64_t(cap)) g = cap;
    if (g < 1) g = 1;
    return int(g);
}

template <typename T>
hipError_t launch_init(void* psi, int M, int n, uint64_t seed, hipStream_t st) {
    const double scale = 1.0 / sqrt(ldexp(1.0, M - 1));
    const int grid = grid_for(1ull << M, 256, 1 << 16);
    hipLaunchKernelGGL(k_init<T>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<typename CT<T>::c*>(psi), M, n, seed, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_product(void* psi, int M, int n, uint64_t seed, hipStream_t st) {
    const double scale = 1.0 / sqrt(ldexp(1.0, M - 1));
    const int grid = grid_for(1ull << M, 256, 1 << 16);
    hipLaunchKernelGGL(k_init_product<T>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<typename CT<T>::c*>(psi), M, n, seed, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_members(void* psi, int M, int cbits, int polarized, uint64_t first,
                               uint64_t count, hipStream_t st) {
    const int grid = grid_for(1ull << (M + cbits), 256, 1 << 16);
    hipLaunchKernelGGL(k_init_members<T>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<typename CT<T>::c*>(psi), M, cbits, polarized, first, count);
    return hipGetLastError();
}

hipError_t launch_accumulate(double* acc, const double* add, int64_t n, double scale,
                             hipStream_t st) {
    const int grid = grid_for(uint64_t(n), 256, 1024);
    hipLaunchKernelGGL(k_accumulate, dim3(grid), dim3(256), 0, st, acc, add, n, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_observe(const void* psi, int M, int site, double* partials, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_observe<T>, dim3(nblk), dim3(256), 0, st,
                       reinterpret_cast<const typename CT<T>::c*>(psi), M, site, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_profile(const double* partials, int nwg, int ch, int M, int64_t s0,
                                 int64_t count, double* Pall, double* N, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_profile, dim3(unsigned(count * (M + 1))), dim3(256), 0, st, partials,
                       nwg, ch, M, s0, Pall, N);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nwg, int ch, int64_t s0, int64_t count,
                         double* P, double* N, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(unsigned(count)), dim3(256), 0, st, partials, nwg, ch, s0,
                       P, N);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_factor(void* psi, int M, int lo, int hi, double t, double s, double pr,
                         double pim, int zz, hipStream_t st) {
    const int grid = grid_for(1ull << (M - 2), 256, 1 << 16);
    hipLaunchKernelGGL(k_factor<T>, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<typename CT<T>::c*>(psi), M, lo, hi, T(t), T(s), T(pr),
                       T(pim), zz);
    return hipGetLastError();
}

template <typename T, int R, int NT, int ENGINE = 0, bool PROFILE = false, bool HALF = false>
static hipError_t pass_one(bool writes, void* psi, const DevPass* passes, const DevStage* stages,
                           const DevOp<T>* ops, int pass_index, int64_t tiles_per_wg, int nwg,
                           double* partials, int64_t step_offset, int ch, const float* mats,
                           hipStream_t st) {
    if (writes)
        hipLaunchKernelGGL((k_pass<T, R, NT, true, ENGINE, PROFILE, HALF>), dim3(nwg), dim3(NT), 0, st,
                           reinterpret_cast<typename CT<T>::c*>(psi), passes, stages, ops,
                           pass_index, tiles_per_wg, partials, step_offset, ch, nwg, mats);
    else
        hipLaunchKernelGGL((k_pass<T, R, NT, false, ENGINE, PROFILE, HALF>), dim3(nwg), dim3(NT), 0, st,
                           reinterpret_cast<typename CT<T>::c*>(psi), passes, stages, ops,
                           pass_index, tiles_per_wg, partials, step_offset, ch, nwg, mats);
    return hipGetLastError();
}

bool pass_half_exists(bool f32, int r, int nt) {
    if (f32) return (r == 5 && nt == 512) || (r == 6 && nt == 256);
    return (r == 4 && nt == 512) || (r == 5 && nt == 256) || (r == 5 && nt == 512);
}

bool pass_shape_exists(bool f32, int r, int nt, int engine) {
    if (engine == 1) return f32 && r == 5 && nt == 512;
    if (engine != 0) return false;
    if (f32) return (r == 4 && nt == 256) || (r == 5 && nt == 256) || (r == 5 && nt == 512) ||
                    (r == 6 && nt == 256) || (r == 4 && nt == 512) || (r == 4 && nt == 1024);
    return (r == 4 && nt == 256) || (r == 5 && nt == 256) || (r == 4 && nt == 512) ||
           (r == 3 && nt == 512) || (r == 3 && nt == 1024);
}

template <typename T>
hipError_t launch_pass(const PassShape& sh, void* psi, const DevPass* passes,
                       const DevStage* stages, const DevOp<T>* ops, int pass_index,
                       int64_t tiles_per_wg, int nwg, double* partials, int64_t step_offset,
                       int ch, hipStream_t st) {
    if constexpr (sizeof(T) == 4) {
        if (sh.engine == 1) {
            if (sh.r == 5 && sh.nt == 512 && sh.mats)
                return pass_one<T, 5, 512, 1>(sh.writes, psi, passes, stages, ops, pass_index,
                                              tiles_per_wg, nwg, partials, step_offset, ch, sh.mats, st);
            return hipErrorInvalidValue;
        }
    }
    if (sh.engine != 0) return hipErrorInvalidValue;
    if (sh.half) {
#define SPIN_HALF(RR, NTT)                                                                        \
    if (sh.r == RR && sh.nt == NTT)                                                               \
        return sh.profile                                                                         \
                   ? pass_one<T, RR, NTT, 0, true, true>(sh.writes, psi, passes, stages, ops,     \
                                                         pass_index, tiles_per_wg, nwg, partials, \
                                                         step_offset, ch, nullptr, st)            \
                   : pass_one<T, RR, NTT, 0, false, true>(sh.writes, psi, passes, stages, ops,    \
                                                          pass_index, tiles_per_wg, nwg, partials,\
                                                          step_offset, ch, nullptr, st);
        if constexpr (sizeof(T) == 4) {
            SPIN_HALF(5, 512) SPIN_HALF(6, 256)
        } else {
            SPIN_HALF(4, 512) SPIN_HALF(5, 256) SPIN_HALF(5, 512)
        }
#undef SPIN_HALF
        return hipErrorInvalidValue;
    }
#define SPIN_PASS(RR, NTT)                                                                   \
    if (sh.r == RR && sh.nt == NTT)                                                          \
        return sh.profile                                                                    \
                   ? pass_one<T, RR, NTT, 0, true>(sh.writes, psi, passes, stages, ops, pass_index, \
                                                   tiles_per_wg, nwg, partials, step_offset, ch,   \
                                                   nullptr, st)                                    \
                   : pass_one<T, RR, NTT>(sh.writes, psi, passes, stages, ops, pass_index,          \
                                          tiles_per_wg, nwg, partials, step_offset, ch, nullptr, st);
    if constexpr (sizeof(T) == 4) {
        SPIN_PASS(5, 256) SPIN_PASS(5, 512) SPIN_PASS(4, 256) SPIN_PASS(6, 256)
        SPIN_PASS(4, 512) SPIN_PASS(4, 1024)
    } else {
        SPIN_PASS(4, 256) SPIN_PASS(5, 256) SPIN_PASS(4, 512) SPIN_PASS(3, 512) SPIN_PASS(3, 1024)
    }
#undef SPIN_PASS
    return hipErrorInvalidValue;
}

template <typename T, int R, int NT>
static hipError_t res_one(const ResidentJob& job0, const ResidentJob* jobs, int njobs,
                          const DevStage* stages, const DevOp<T>* ops, int64_t n_steps,
                          hipStream_t st) {
    if (!jobs && job0.Pall)    // one problem with the all-site profile
        hipLaunchKernelGGL((k_resident<T, R, NT, true>), dim3(njobs), dim3(NT), 0, st, job0, jobs,
                           stages, ops, n_steps);
    else
        hipLaunchKernelGGL((k_resident<T, R, NT, false>), dim3(njobs), dim3(NT), 0, st, job0, jobs,
                           stages, ops, n_steps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_resident(int r, int nt, const ResidentJob& job0, const ResidentJob* jobs,
                           int njobs, const DevStage* stages, const DevOp<T>* ops,
                           int64_t n_steps, hipStream_t st) {
#define SPIN_RES(RR, NTT)                                                              \
    if (r == RR && nt == NTT)                                                          \
        return res_one<T, RR, NTT>(job0, jobs, njobs, stages, ops, n_steps, st);
    SPIN_RES(1, 64) SPIN_RES(2, 64) SPIN_RES(3, 64) SPIN_RES(4, 64) SPIN_RES(5, 64)
    SPIN_RES(4, 256) SPIN_RES(5, 256)
    if constexpr (sizeof(T) == 4) {
        SPIN_RES(5, 512)
    } else {
        SPIN_RES(4, 512)
    }
#undef SPIN_RES
    return hipErrorInvalidValue;
}

int batch_tile_bits(bool f32) { return f32 ? 14 : 13; }

// Launch shapes of the batch kernel: whole tiles 2^R x 512 lanes (one
// workgroup per CU); half tiles 2^(R+1) x 256 lanes (two per CU), whose
// larger register stages take fewer LDS exchanges on dense coupling graphs.
BatchShape batch_shape(bool f32, bool half) {
    if (half) return BatchShape{true, f32 ? 6 : 5, 256};
    return BatchShape{false, f32 ? 5 : 4, 512};
}

int batch_blocks_per_cu(bool f32, bool half) {
    int n = 0;
    hipError_t e;
    if (f32)
        e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<float, 6, 256, true>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<float, 5, 512, false>, 512, 0);
    else
        e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<double, 5, 256, true>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<double, 4, 512, false>, 512, 0);
    return e == hipSuccess ? n : 0;
}

template <typename T>
hipError_t launch_batch(int nslots, bool half, const BatchProblem* probs, const BatchJob* jobs,
                        const int* job_start, const DevPass* passes, const DevStage* stages,
                        const DevOp<T>* ops, const int2* launches, double* partials, int* counters,
                        int ncounters, int* err, int* status, int64_t n_steps, hipStream_t st) {
    // counters and the error flag start at zero (a fill kernel, not a
    // memset node, so the pair can sit in a captured graph)
    hipLaunchKernelGGL(k_fill_int, dim3(64), dim3(256), 0, st, counters, ncounters, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, err, 1, 0);
    constexpr bool F = sizeof(T) == 4;
    if (half)
        hipLaunchKernelGGL((k_batch<T, F ? 6 : 5, 256, true>), dim3(nslots), dim3(256), 0, st, probs,
                           jobs, job_start, passes, stages, ops, launches, partials, counters, err,
                           n_steps);
    else
        hipLaunchKernelGGL((k_batch<T, F ? 5 : 4, 512, false>), dim3(nslots), dim3(512), 0, st, probs,
                           jobs, job_start, passes, stages, ops, launches, partials, counters, err,
                           n_steps);
    hipLaunchKernelGGL(k_status_or, dim3(1), dim3(64), 0, st, err, status);
    return hipGetLastError();
}

template hipError_t launch_batch<float>(int, bool, const BatchProblem*, const BatchJob*, const int*,
                                        const DevPass*, const DevStage*, const DevOp<float>*,
                                        const int2*, double*, int*, int, int*, int*, int64_t,
                                        hipStream_t);
template hipError_t launch_batch<double>(int, bool, const BatchProblem*, const BatchJob*, const int*,
                                         const DevPass*, const DevStage*, const DevOp<double>*,
                                         const int2*, double*, int*, int, int*, int*, int64_t,
                                         hipStream_t);
template hipError_t launch_init<float>(void*, int, int, uint64_t, hipStream_t);
template hipError_t launch_init<double>(void*, int, int, uint64_t, hipStream_t);
template hipError_t launch_init_product<float>(void*, int, int, uint64_t, hipStream_t);
template hipError_t launch_init_product<double>(void*, int, int, uint64_t, hipStream_t);
template hipError_t launch_init_members<float>(void*, int, int, int, uint64_t, uint64_t, hipStream_t);
template hipError_t launch_init_members<double>(void*, int, int, int, uint64_t, uint64_t, hipStream_t);
template hipError_t launch_observe<float>(const void*, int, int, double*, int, hipStream_t);
template hipError_t launch_observe<double>(const void*, int, int, double*, int, hipStream_t);
template hipError_t launch_factor<float>(void*, int, int, int, double, double, double, double, int,
                                         hipStream_t);
template hipError_t launch_factor<double>(void*, int, int, int, double, double, double, double,
                                          int, hipStream_t);
template hipError_t launch_pass<float>(const PassShape&, void*, const DevPass*, const DevStage*,
                                       const DevOp<float>*, int, int64_t, int, double*, int64_t,
                                       int, hipStream_t);
template hipError_t launch_pass<double>(const PassShape&, void*, const DevPass*, const DevStage*,
                                        const DevOp<double>*, int, int64_t, int, double*, int64_t,
                                        int, hipStream_t);
template hipError_t launch_resident<float>(int, int, const ResidentJob&, const ResidentJob*, int,
                                           const DevStage*, const DevOp<float>*, int64_t,
                                           hipStream_t);
template hipError_t launch_resident<double>(int, int, const ResidentJob&, const ResidentJob*, int,
                                            const DevStage*, const DevOp<double>*, int64_t,
                                            hipStream_t);

}  // namespace spinqp
