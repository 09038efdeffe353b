// kernels.hip -- gfx950 kernels of the random-phase Trotter path.
//
//  k_init        random-phase state (counter-based SplitMix64 phases)
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

// Amplitude of basis state x of the random-phase state, FP64.
__device__ __forceinline__ void random_phase_amp(uint64_t x, int n, uint64_t seed, double scale,
                                                 double* re, double* im) {
    if ((x >> n) & 1ull) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    const uint64_t r = (x & ((1ull << n) - 1ull)) | ((x >> (n + 1)) << n);
    const uint64_t z = sm64_mix(seed + (r + 1ull) * 0x9E3779B97F4A7C15ull);
    const double u = double(z >> 11) * 0x1.0p-53;
    double s, c;
    sincospi(2.0 * u, &s, &c);      // phi = 2 pi u
    *re = c * scale;
    *im = s * scale;
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
// done as two real three-shear rotations (exactly area preserving).
template <int R, int A, int B, typename T>
__device__ __forceinline__ void reg_xy(T (&re)[1 << R], T (&im)[1 << R], T t, T s) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (((j >> A) & 1) == 0 && ((j >> B) & 1) == 1) {
            const int k = j ^ (1 << A) ^ (1 << B);
            T u = re[j], v = im[k];
            u = fma(t, v, u); v = fma(-s, u, v); u = fma(t, v, u);
            re[j] = u; im[k] = v;
            u = im[j]; v = re[k];
            u = fma(-t, v, u); v = fma(s, u, v); u = fma(-t, v, u);
            im[j] = u; re[k] = v;
        }
    }
}

// I^z I^z phase: anti-aligned amplitudes times (pr + i pi), aligned times
// its conjugate.
template <int R, int A, int B, typename T>
__device__ __forceinline__ void reg_zz(T (&re)[1 << R], T (&im)[1 << R], T pr, T pim) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        const bool anti = ((j >> A) & 1) != ((j >> B) & 1);
        const T q = anti ? pim : -pim;
        const T x = re[j], y = im[j];
        re[j] = fma(pr, x, -q * y);
        im[j] = fma(pr, y, q * x);
    }
}

template <int R, typename T>
__device__ __forceinline__ void reg_op(T (&re)[1 << R], T (&im)[1 << R], int code, T t, T s,
                                       T pr, T pim) {
#define SPIN_CASE(A, B)                                   \
    case A * 8 + B:                                       \
        if constexpr (B < R) {                            \
            reg_xy<R, A, B>(re, im, t, s);                \
            if (code & kOpZZ) reg_zz<R, A, B>(re, im, pr, pim); \
        }                                                 \
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
template <int R, typename T>
__device__ __forceinline__ void reg_observe(const T (&re)[1 << R], const T (&im)[1 << R], int sign,
                                            int mask, double& p, double& n) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        const double w = double(re[j]) * double(re[j]) + double(im[j]) * double(im[j]);
        n += w;
        const int neg = sign ^ ((j & mask) ? 1 : 0);
        p += neg ? -w : w;
    }
}

// --------------------------------------------------------------- k_pass
template <typename T, int R, int NT>
__global__ __launch_bounds__(NT) void k_pass(typename CT<T>::c* __restrict__ psi,
                                             const DevPass* __restrict__ passes,
                                             const DevStage* __restrict__ stages,
                                             const DevOp<T>* __restrict__ ops, int pass_index,
                                             int64_t tiles_per_wg, double* __restrict__ partials,
                                             int64_t step_offset, int ch, int nwg) {
    using C = typename CT<T>::c;
    using VEC = typename CT<T>::v;
    constexpr int V = CT<T>::V;
    constexpr int K = R + __builtin_ctz(NT);        // tile bits
    constexpr int NIT = (1 << R) / V;               // load/store iterations per lane
    constexpr int EB = sizeof(C);
    __shared__ C lds[1 << K];
    __shared__ double red[2 * (NT / 64)];

    const DevPass& P = passes[pass_index];
    const int tid = threadIdx.x;

    // per-lane load/store offsets: element e = it*NT*V + tid*V (+ v)
    int64_t goff_t = 0;
    {
        const uint32_t e = uint32_t(tid) * V;
#pragma unroll
        for (int p = 0; p < K; ++p)
            if (e & (1u << p)) goff_t |= int64_t(1) << P.tbit[p];
    }
    const uint32_t soff_t = lds_swizzle<EB>(uint32_t(tid) * V);

    double accP[kMaxMeas], accN[kMaxMeas];
#pragma unroll
    for (int m = 0; m < kMaxMeas; ++m) accP[m] = accN[m] = 0.0;

    for (int64_t it_tile = 0; it_tile < tiles_per_wg; ++it_tile) {
        const int64_t tile = int64_t(blockIdx.x) + it_tile * int64_t(gridDim.x);
        int64_t base = 0;
        for (int f = 0; f < P.nfree; ++f)
            if ((tile >> f) & 1) base |= int64_t(1) << P.fbit[f];
        const int tile_sign = P.obs_free_bit >= 0 ? int((base >> P.obs_free_bit) & 1) : 0;

        // global -> LDS
        {
            VEC buf[NIT];
#pragma unroll
            for (int it = 0; it < NIT; ++it)
                buf[it] = *reinterpret_cast<const VEC*>(psi + base + goff_t + P.iter_goff[it]);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const uint32_t a = soff_t ^ P.iter_soff[it];
                if constexpr (V == 2) {
                    C lo, hi;
                    lo.x = buf[it].x; lo.y = buf[it].y;
                    hi.x = buf[it].z; hi.y = buf[it].w;
                    lds[a] = lo;
                    lds[a ^ 1] = hi;
                } else {
                    C c;
                    c.x = buf[it].x; c.y = buf[it].y;
                    lds[a] = c;
                }
            }
        }
        __syncthreads();

        for (int si = 0; si < P.nstage; ++si) {
            const DevStage& S = stages[P.stage0 + si];
            uint32_t lb = 0;
            for (int q = 0; q < S.ntb; ++q)
                if ((tid >> q) & 1) lb |= 1u << S.tpos[q];
            const uint32_t pb = lds_swizzle<EB>(lb);
            T re[1 << R], im[1 << R];
#pragma unroll
            for (int j = 0; j < (1 << R); ++j) {
                const C c = lds[pb ^ S.soff[j]];
                re[j] = c.x;
                im[j] = c.y;
            }
            const int sign = tile_sign ^ (S.obs_tq >= 0 ? ((tid >> S.obs_tq) & 1) : 0);
            for (int o = S.op0; o < S.op0 + S.nop; ++o) {
                const DevOp<T> op = ops[o];
                if (op.code == kOpMeas) {
                    double p = 0.0, n = 0.0;
                    reg_observe<R, T>(re, im, sign, S.obs_mask, p, n);
#pragma unroll
                    for (int m = 0; m < kMaxMeas; ++m)
                        if (m == op.aux) { accP[m] += p; accN[m] += n; }
                } else {
                    reg_op<R, T>(re, im, op.code, op.t, op.s, op.pr, op.pi);
                }
            }
            // A lane scatters to exactly the LDS slots it gathered, so the
            // only hazard is with the next stage's gathers (barrier below).
#pragma unroll
            for (int j = 0; j < (1 << R); ++j) {
                C c;
                c.x = re[j];
                c.y = im[j];
                lds[pb ^ S.soff[j]] = c;
            }
            __syncthreads();
        }

        // LDS -> global
        if (P.writes) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const uint32_t a = soff_t ^ P.iter_soff[it];
                VEC v;
                if constexpr (V == 2) {
                    const C lo = lds[a], hi = lds[a ^ 1];
                    v.x = lo.x; v.y = lo.y; v.z = hi.x; v.w = hi.y;
                } else {
                    const C c = lds[a];
                    v.x = c.x; v.y = c.y;
                }
                *reinterpret_cast<VEC*>(psi + base + goff_t + P.iter_goff[it]) = v;
            }
        }
        __syncthreads();
    }

    for (int m = 0; m < P.nmeas; ++m) {
        double p = accP[0], n = accN[0];
#pragma unroll
        for (int mm = 1; mm < kMaxMeas; ++mm)
            if (mm == m) { p = accP[mm]; n = accN[mm]; }
        block_sum2<NT>(p, n, red);
        if (tid == 0) {
            const int64_t s = step_offset + P.meas_step[m];
            double* dst = partials + ((size_t)(s % ch) * nwg + blockIdx.x) * 2;
            dst[0] = p;
            dst[1] = n;
        }
    }
}

// ------------------------------------------------------------ k_resident
// One workgroup owns one whole state (2^M <= NT << R amplitudes) in LDS and
// runs the prologue stages once and the step stages n_steps times,
// writing P[k], N[k] itself.
template <typename T, int R, int NT>
__global__ __launch_bounds__(NT) void k_resident(ResidentJob job0,
                                                 const ResidentJob* __restrict__ jobs,
                                                 const DevStage* __restrict__ stages,
                                                 const DevOp<T>* __restrict__ ops,
                                                 int64_t n_steps) {
    using C = typename CT<T>::c;
    constexpr int EB = sizeof(C);
    __shared__ C lds[NT << R];
    __shared__ double red[2 * ((NT + 63) / 64)];
    const ResidentJob J = jobs ? jobs[blockIdx.x] : job0;
    const int tid = threadIdx.x;
    const int M = J.M;
    const uint32_t dim = 1u << M;
    const int nact = (M >= R) ? (1 << (M - R)) : 1;
    C* psi = reinterpret_cast<C*>(J.psi);

    if (J.init) {
        const double scale = 1.0 / sqrt(ldexp(1.0, M - 1));
        for (uint32_t x = tid; x < dim; x += NT) {
            double re, im;
            random_phase_amp(x, J.polarized, J.seed, scale, &re, &im);
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
            uint32_t lb = 0;
            for (int q = 0; q < S.ntb; ++q)
                if ((tid >> q) & 1) lb |= 1u << S.tpos[q];
            const uint32_t pb = lds_swizzle<EB>(lb);
            const bool act = tid < nact;
            T re[1 << R], im[1 << R];
            if (act) {
#pragma unroll
                for (int j = 0; j < (1 << R); ++j) {
                    const C c = lds[pb ^ S.soff[j]];
                    re[j] = c.x;
                    im[j] = c.y;
                }
            } else {
#pragma unroll
                for (int j = 0; j < (1 << R); ++j) re[j] = im[j] = T(0);
            }
            const int sign = S.obs_tq >= 0 ? ((tid >> S.obs_tq) & 1) : 0;
            for (int o = S.op0; o < S.op0 + S.nop; ++o) {
                const DevOp<T> op = ops[o];
                if (op.code == kOpMeas) {
                    double p = 0.0, n = 0.0;
                    reg_observe<R, T>(re, im, sign, S.obs_mask, p, n);
                    block_sum2<NT>(p, n, red);
                    if (tid == 0) {
                        J.P[step] = p;
                        if (J.N) J.N[step] = n;
                    }
                } else {
                    reg_op<R, T>(re, im, op.code, op.t, op.s, op.pr, op.pi);
                }
            }
            if (act) {
#pragma unroll
                for (int j = 0; j < (1 << R); ++j) {
                    C c;
                    c.x = re[j];
                    c.y = im[j];
                    lds[pb ^ S.soff[j]] = c;
                }
            }
            __syncthreads();
        }
    };
    run(J.pro_stage0, J.pro_nstage, 0);
    for (int64_t k = 1; k <= n_steps; ++k) run(J.step_stage0, J.step_nstage, k);

    for (uint32_t x = tid; x < dim; x += NT) psi[x] = lds[lds_swizzle<EB>(x)];
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
hipError_t launch_observe(const void* psi, int M, int site, double* partials, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_observe<T>, dim3(nblk), dim3(256), 0, st,
                       reinterpret_cast<const typename CT<T>::c*>(psi), M, site, partials);
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

template <typename T, int R, int NT>
static hipError_t pass_one(void* psi, const DevPass* passes, const DevStage* stages,
                           const DevOp<T>* ops, int pass_index, int64_t tiles_per_wg, int nwg,
                           double* partials, int64_t step_offset, int ch, hipStream_t st) {
    hipLaunchKernelGGL((k_pass<T, R, NT>), dim3(nwg), dim3(NT), 0, st,
                       reinterpret_cast<typename CT<T>::c*>(psi), passes, stages, ops, pass_index,
                       tiles_per_wg, partials, step_offset, ch, nwg);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass(const PassShape& sh, void* psi, const DevPass* passes,
                       const DevStage* stages, const DevOp<T>* ops, int pass_index,
                       int64_t tiles_per_wg, int nwg, double* partials, int64_t step_offset,
                       int ch, hipStream_t st) {
#define SPIN_PASS(RR, NTT)                                                                   \
    if (sh.r == RR && sh.nt == NTT)                                                          \
        return pass_one<T, RR, NTT>(psi, passes, stages, ops, pass_index, tiles_per_wg, nwg, \
                                    partials, step_offset, ch, st);
    if constexpr (sizeof(T) == 4) {
        SPIN_PASS(5, 256) SPIN_PASS(5, 512) SPIN_PASS(4, 256) SPIN_PASS(6, 256)
    } else {
        SPIN_PASS(4, 256) SPIN_PASS(5, 256) SPIN_PASS(4, 512)
    }
#undef SPIN_PASS
    return hipErrorInvalidValue;
}

template <typename T, int R, int NT>
static hipError_t res_one(const ResidentJob& job0, const ResidentJob* jobs, int njobs,
                          const DevStage* stages, const DevOp<T>* ops, int64_t n_steps,
                          hipStream_t st) {
    hipLaunchKernelGGL((k_resident<T, R, NT>), dim3(njobs), dim3(NT), 0, st, job0, jobs, stages,
                       ops, n_steps);
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

template hipError_t launch_init<float>(void*, int, int, uint64_t, hipStream_t);
template hipError_t launch_init<double>(void*, int, int, uint64_t, hipStream_t);
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
