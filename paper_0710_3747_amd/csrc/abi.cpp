// abi.cpp -- the C ABI of include/spin.h: argument validation, plan caches,
// workspaces and launch orchestration.  Every step of the path runs in the
// kernels of kernels.hip; this file only plans and enqueues.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/spin.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "abi_internal.hpp"

namespace spinqp {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SPIN_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

// ------------------------------------------------------------- validation
int validate_common(const void* psi, int32_t prec, int32_t M) {
    if (!psi) return fail(SPIN_EINVAL, "psi is NULL");
    if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "prec must be SPIN_C64 or SPIN_C128");
    const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
    if (M < 1 || M > maxM) {
        std::ostringstream os;
        os << "M = " << M << " out of range 1.." << maxM;
        return fail(SPIN_EINVAL, os.str());
    }
    if (reinterpret_cast<uintptr_t>(psi) % 16 != 0) return fail(SPIN_EINVAL, "psi must be 16-byte aligned");
    return SPIN_OK;
}

int validate_couplings(int32_t M, const spin_coupling* J, int64_t K, std::vector<Coupling>* out) {
    if (K < 0) return fail(SPIN_EINVAL, "K < 0");
    if (K > 0 && !J) return fail(SPIN_EINVAL, "J is NULL with K > 0");
    out->clear();
    out->reserve(size_t(K));
    for (int64_t g = 0; g < K; ++g) {
        const spin_coupling& c = J[g];
        std::ostringstream os;
        if (c.i < 0 || c.i >= M || c.j < 0 || c.j >= M) {
            os << "coupling " << g << ": site out of range 0.." << M - 1;
            return fail(SPIN_EINVAL, os.str());
        }
        if (c.i == c.j) {
            os << "coupling " << g << ": i == j";
            return fail(SPIN_EINVAL, os.str());
        }
        if (!std::isfinite(c.a) || !std::isfinite(c.b)) {
            os << "coupling " << g << ": non-finite a or b";
            return fail(SPIN_EINVAL, os.str());
        }
        out->push_back(Coupling{c.i, c.j, c.a, c.b});
    }
    return SPIN_OK;
}

// ------------------------------------------------------------ workspaces
// Device scratch, grow-only, one per (device, stream, slot): calls on
// different streams never share one.  Slot 0 holds per-workgroup partial
// sums, slot 1 the per-evolution member sums of spin_ensemble_evolve.
struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};
static std::mutex g_mu;
static std::map<std::tuple<int, hipStream_t, int>, Scratch> g_scratch;

int scratch_get_slot(hipStream_t st, int slot, size_t bytes, void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch& s = g_scratch[std::make_tuple(dev, st, slot)];
    if (s.bytes < bytes) {
        if (s.ptr) {
            // previous work on this stream may still read it
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipFree(s.ptr));
            s.ptr = nullptr;
            s.bytes = 0;
        }
        size_t want = std::max(bytes, size_t(1) << 20);
        if (hipMalloc(&s.ptr, want) != hipSuccess) {
            s.ptr = nullptr;
            return fail(SPIN_ENOMEM, "workspace allocation failed");
        }
        s.bytes = want;
    }
    *out = s.ptr;
    return SPIN_OK;
}

int scratch_get(hipStream_t st, size_t bytes, void** out) { return scratch_get_slot(st, 0, bytes, out); }

// ------------------------------------------------------------- plan cache
struct PlanKey {
    int dev, prec, M, observed, k, r, nt, c, merge, engine, profile, half;
    double dt;
    int64_t n_steps;
    std::vector<double> J;    // flattened couplings
    bool operator<(const PlanKey& o) const {
        return std::tie(dev, prec, M, observed, k, r, nt, c, merge, engine, profile, half, dt, n_steps, J) <
               std::tie(o.dev, o.prec, o.M, o.observed, o.k, o.r, o.nt, o.c, o.merge, o.engine,
                        o.profile, o.half, o.dt, o.n_steps, o.J);
    }
};

struct DevicePlan {
    bool resident = false;
    StreamPlan sp;
    PassShape shape{};
    int k = 0, nwg = 0;
    int64_t tiles_per_wg = 0;
    // device tables
    void* d_passes = nullptr;
    void* d_stages = nullptr;
    void* d_ops = nullptr;
    void* d_mats = nullptr;     // matrix engine
    // resident
    int res_r = 0, res_nt = 0;
    int pro_stage0 = 0, pro_nstage = 0, step_stage0 = 0, step_nstage = 0;
    // per template: measurement steps (relative) and their sites
    std::vector<std::vector<int64_t>> meas;
    std::vector<std::vector<int>> meas_site;
    bool profile = false;
    size_t stages_total = 0;
    ~DevicePlan() {
        if (d_passes) (void)hipFree(d_passes);
        if (d_stages) (void)hipFree(d_stages);
        if (d_ops) (void)hipFree(d_ops);
        if (d_mats) (void)hipFree(d_mats);
    }
};

static std::map<PlanKey, std::shared_ptr<DevicePlan>> g_plans;

template <typename T>
static int upload_tables(const DevTables<T>& tb, DevicePlan* dp) {
    auto up = [&](const void* src, size_t n, void** dst) -> int {
        if (n == 0) n = 16;
        if (hipMalloc(dst, n) != hipSuccess) return fail(SPIN_ENOMEM, "plan table allocation failed");
        if (src) HIP_TRY(hipMemcpy(*dst, src, n, hipMemcpyHostToDevice));
        return SPIN_OK;
    };
    int rc;
    if ((rc = up(tb.passes.data(), tb.passes.size() * sizeof(DevPass), &dp->d_passes))) return rc;
    if ((rc = up(tb.stages.data(), tb.stages.size() * sizeof(DevStage), &dp->d_stages))) return rc;
    if ((rc = up(tb.ops.data(), tb.ops.size() * sizeof(DevOp<T>), &dp->d_ops))) return rc;
    if (!tb.mats.empty() && (rc = up(tb.mats.data(), tb.mats.size() * sizeof(float), &dp->d_mats))) return rc;
    return SPIN_OK;
}

// Launch shape: tile bits k = r + log2(nt).  Defaults: complex64 tiles of
// 2^14 amplitudes, complex128 tiles of 2^13 (128 KiB either way), exchanged
// through LDS in halves where a kernel exists (two workgroups per CU).
Shape choose_shape(int prec, int M, const spin_options* opt) {
    Shape s;
    const bool f32 = prec == SPIN_C64;
    const int ex = opt ? opt->exchange : 0;
    int k = f32 ? 14 : 13;
    // complex128 tiles: 16 amplitudes per lane with half-tile exchanges
    // (two 256-lane workgroups per CU), 8 with whole tiles
    s.r = (f32 || ex != 1) ? 5 : 4;
    // 4 low address bits in every tile: 128-byte runs of complex64 (fewer
    // passes than 256-byte runs, which outweighs the slower sweep on the
    // ladders), 256-byte runs of complex128
    s.c = 4;
    if (opt && opt->tile_bits > 0) {
        k = opt->tile_bits;
        // complex128: 32 amplitudes per lane with half tiles of 2^13 (two
        // 256-lane workgroups per CU) or 2^14 (one 512-lane workgroup)
        s.r = f32 ? (k <= 12 ? 4 : 5) : (ex != 1 && (k == 13 || k == 14) ? 5 : 4);
    }
    if (opt && opt->reg_bits > 0) s.r = opt->reg_bits;
    if (opt && opt->coalesce_bits > 0) s.c = opt->coalesce_bits;
    if (f32 && s.c < 1) s.c = 1;     // two-amplitude vector accesses need bit 0
    s.nt = (k - s.r >= 0 && k - s.r < 16) ? (1 << (k - s.r)) : 0;
    s.k = k;
    s.engine = opt ? opt->engine : 0;
    const bool half_ok = s.engine == 0 && pass_half_exists(f32, s.r, s.nt);
    s.half = ex == 2 || (ex == 0 && half_ok);
    s.valid = s.half ? half_ok : pass_shape_exists(f32, s.r, s.nt, s.engine);
    s.res_cap = f32 ? 14 : 13;
    s.resident = M <= s.res_cap;
    return s;
}

static int res_shape(int prec, int M, int* r, int* nt) {
    const int rmax = prec == SPIN_C64 ? 5 : 4;
    *r = std::min(rmax, M);
    const int tb = M - *r;    // thread bits
    if (tb <= 6) *nt = 64;
    else if (tb <= 8) *nt = 256;
    else *nt = 512;
    return SPIN_OK;
}

template <typename T>
static int build_plan(const PlanKey& key, const std::vector<Coupling>& J, const Shape& sh,
                      std::shared_ptr<DevicePlan>* out) {
    auto dp = std::make_shared<DevicePlan>();
    DevTables<T> tb;
    try {
        if (sh.resident) {
            dp->resident = true;
            res_shape(key.prec, key.M, &dp->res_r, &dp->res_nt);
            ResidentPlan rp = plan_resident(key.M, J, key.dt, key.observed, key.merge != 0, dp->res_r,
                                            key.profile != 0);
            dp->pro_stage0 = 0;
            encode_pass<T>(rp.prologue, key.M, key.observed, tb, true, 0, key.profile != 0);
            dp->pro_nstage = int(tb.stages.size());
            dp->step_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.step, key.M, key.observed, tb, true, 0, key.profile != 0);
            dp->step_nstage = int(tb.stages.size()) - dp->step_stage0;
            dp->stages_total = tb.stages.size();
        } else {
            PassParams pp;
            pp.k = sh.k;
            pp.r = sh.r;
            pp.c = sh.c;
            pp.profile = key.profile != 0;
            pp.half = sh.half;
            if (pp.profile) pp.max_meas = kMaxMeasProfile;
            dp->sp = plan_stream_best(key.M, J, key.dt, key.n_steps, key.observed, key.merge != 0, pp);
            dp->shape = PassShape{sh.r, sh.nt};
            dp->shape.engine = sh.engine;
            dp->shape.profile = pp.profile;
            dp->shape.half = sh.half;
            dp->profile = pp.profile;
            dp->k = sh.k;
            const int64_t ntiles = int64_t(1) << (key.M - sh.k);
            int dev_cu = 256;
            {
                hipDeviceProp_t prop;
                if (hipGetDeviceProperties(&prop, key.dev) == hipSuccess) dev_cu = prop.multiProcessorCount;
            }
            // persistent grid: a power of two <= tiles, ~4 workgroups per CU
            int64_t nwg = 1;
            while (nwg * 2 <= ntiles && nwg * 2 <= int64_t(dev_cu) * 4) nwg *= 2;
            dp->nwg = int(nwg);
            dp->tiles_per_wg = ntiles / nwg;
            for (const HostPass& hp : dp->sp.passes) {
                encode_pass<T>(hp, key.M, key.observed, tb, false, sh.engine, key.profile != 0);
                std::vector<int64_t> ms;
                std::vector<int> mst;
                for (const Op& op : hp.ops)
                    if (op.kind == 1) {
                        ms.push_back(op.step);
                        mst.push_back(op.i);
                    }
                dp->meas.push_back(ms);
                dp->meas_site.push_back(mst);
            }
            dp->stages_total = tb.stages.size();
        }
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("planning failed: ") + e.what());
    }
    int rc = upload_tables<T>(tb, dp.get());
    if (rc) return rc;
    *out = dp;
    return SPIN_OK;
}

int get_plan(int prec, int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
             int observed, const spin_options* opt, bool profile,
             std::shared_ptr<DevicePlan>* out, Shape* shape_out, bool lookup_only = false) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Shape sh = choose_shape(prec, M, opt);
    if (!sh.resident && !sh.valid) {
        std::ostringstream os;
        os << "no pass kernel for tile_bits " << sh.k << " with reg_bits " << sh.r
           << (sh.engine ? " and the matrix engine (complex64, tile_bits 14, reg_bits 5 only)" : "")
           << (sh.half ? " and half-tile exchanges" : "");
        return fail(SPIN_EUNSUPPORTED, os.str());
    }
    PlanKey key{dev, prec, M, observed, sh.k, sh.r, sh.nt, sh.c,
                (opt && opt->no_merge) ? 0 : 1, sh.resident ? 0 : sh.engine,
                profile ? 1 : 0, (sh.half && !sh.resident) ? 1 : 0, dt, sh.resident ? 0 : n_steps, {}};
    key.J.reserve(J.size() * 4);
    for (const Coupling& c : J) {
        key.J.push_back(c.i);
        key.J.push_back(c.j);
        key.J.push_back(c.a);
        key.J.push_back(c.b);
    }
    if (shape_out) *shape_out = sh;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            *out = it->second;
            return SPIN_OK;
        }
    }
    if (lookup_only)
        return fail(SPIN_EUNSUPPORTED, "no prepared plan for these arguments: call spin_prepare_plan with "
                                       "the same arguments first (this entry point allocates nothing)");
    std::shared_ptr<DevicePlan> dp;
    int rc = prec == SPIN_C64 ? build_plan<float>(key, J, sh, &dp) : build_plan<double>(key, J, sh, &dp);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans[key] = dp;
    *out = dp;
    return SPIN_OK;
}

// ------------------------------------------------------------- graphs
// The launch sequence of one tiled evolve call, captured once per plan and
// set of buffers baked into the kernel arguments, and replayed on a library
// stream that is ordered after the caller's stream and before its later
// work (the call stays asynchronous).
struct GraphKey {
    const void* plan;
    void* psi;
    double* P;
    double* N;
    void* part;
    int dev;
    bool operator<(const GraphKey& o) const {
        return std::tie(plan, psi, P, N, part, dev) < std::tie(o.plan, o.psi, o.P, o.N, o.part, o.dev);
    }
};
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
static std::mutex g_graph_mu;
static std::map<GraphKey, GraphEntry> g_graphs;
static std::map<int, hipStream_t> g_graph_stream;

template <typename F>
static int run_as_graph(const GraphKey& key, F&& enqueue, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    hipStream_t& side = g_graph_stream[key.dev];
    if (!side) HIP_TRY(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        HIP_TRY(hipStreamBeginCapture(side, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue(side);
        GraphEntry ge;
        const hipError_t e = hipStreamEndCapture(side, &ge.graph);
        if (rc != SPIN_OK || e != hipSuccess) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return rc != SPIN_OK ? rc : fail(SPIN_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(ge.graph);
            return fail(SPIN_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        }
        it = g_graphs.emplace(key, ge).first;
    }
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ev, 0);
    if (e == hipSuccess) e = hipGraphLaunch(it->second.exec, side);
    if (e == hipSuccess) e = hipEventRecord(ev, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
    return SPIN_OK;
}

static void release_graphs() {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& kv : g_graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
    for (auto& kv : g_graph_stream)
        if (kv.second) (void)hipStreamDestroy(kv.second);
    g_graph_stream.clear();
}

// ------------------------------------------------------------- evolve
template <typename T>
static int evolve_naive(void* psi, int M, const std::vector<Coupling>& J, double dt,
                        int64_t n_steps, int observed, double* P, double* N, bool profile,
                        const Workspace* ws, hipStream_t st) {
    const int nblk = 1024;
    void* scratch = nullptr;
    int rc;
    if (ws) {
        if (ws->doubles < size_t(nblk) * 2) return fail(SPIN_EUNSUPPORTED, "workspace too small");
        scratch = ws->ptr;
    } else if ((rc = scratch_get(st, size_t(nblk) * 2 * sizeof(double), &scratch))) {
        return rc;
    }
    double* part = static_cast<double*>(scratch);
    // With `profile`, P holds M values per step (row k = every site after k
    // steps) and N is taken with the observed site's value.
    auto observe = [&](int64_t k) -> int {
        for (int site = profile ? 0 : observed; site < (profile ? M : observed + 1); ++site) {
            double* dstP = profile ? P + k * M + site : P + k;
            double* dstN = (N && site == observed) ? N + k : nullptr;
            HIP_TRY((launch_observe<T>(psi, M, site, part, nblk, st)));
            HIP_TRY(launch_reduce(part, nblk, 1, 0, 1, dstP, dstN, st));
        }
        return SPIN_OK;
    };
    if ((rc = observe(0))) return rc;
    const double tau = 0.5 * dt;
    for (int64_t k = 1; k <= n_steps; ++k) {
        for (int dir = 0; dir < 2; ++dir) {
            for (size_t n = 0; n < J.size(); ++n) {
                const Coupling& c = dir == 0 ? J[n] : J[J.size() - 1 - n];
                const double th = 0.5 * c.b * tau;
                int pieces = 1;
                while (std::fabs(th / pieces) > 1.5707963267948966) pieces *= 2;
                for (int pc = 0; pc < pieces; ++pc) {
                    const double t = th / pieces;
                    const double A = pc == 0 ? c.a * tau : 0.0;
                    HIP_TRY((launch_factor<T>(psi, M, std::min(c.i, c.j), std::max(c.i, c.j),
                                              std::tan(0.5 * t), std::sin(t), std::cos(0.25 * A),
                                              std::sin(0.25 * A), A != 0.0 ? 1 : 0, st)));
                }
            }
        }
        if ((rc = observe(k))) return rc;
    }
    return SPIN_OK;
}

// All-site profile through the fused plan: P is [n_steps + 1][M].  A pass
// measures some sites of some steps; a step is complete once every site has
// been measured for it (each site's measurements run in step order), and
// complete steps are reduced in chunks out of a ring of `ch` step slots.
template <typename T>
static int evolve_profile(void* psi, int M, const DevicePlan& dp, int64_t n_steps, double* P,
                          double* N, bool graph, hipStream_t st) {
    if (dp.resident) {
        ResidentJob job{};
        job.psi = psi;
        job.Pall = P;
        job.N = N;
        job.M = M;
        job.init = 0;
        job.pro_stage0 = dp.pro_stage0;
        job.pro_nstage = dp.pro_nstage;
        job.step_stage0 = dp.step_stage0;
        job.step_nstage = dp.step_nstage;
        HIP_TRY((launch_resident<T>(dp.res_r, dp.res_nt, job, nullptr, 1,
                                    static_cast<const DevStage*>(dp.d_stages),
                                    static_cast<const DevOp<T>*>(dp.d_ops), n_steps, st)));
        return SPIN_OK;
    }
    const int64_t total = n_steps + 1;
    const int ch = int(std::min<int64_t>(total, 64));
    void* scratch = nullptr;
    int rc = scratch_get(st, size_t(ch) * dp.nwg * (M + 1) * sizeof(double), &scratch);
    if (rc) return rc;
    double* part = static_cast<double*>(scratch);
    auto enqueue = [&](hipStream_t st) -> int {
        std::vector<int64_t> next(M, 0);    // per site: steps measured so far
        int64_t complete = 0, reduced = 0, highest = 0;
        const size_t nl = dp.sp.launch_tmpl.size();
        for (size_t l = 0; l < nl; ++l) {
            const int t = dp.sp.launch_tmpl[l];
            const int64_t off = dp.sp.launch_offset[l];
            for (int64_t s : dp.meas[t]) highest = std::max(highest, s + off + 1);
            if (highest - reduced > ch) {
                std::ostringstream os;
                os << "internal: profile measurements run " << highest - reduced
                   << " steps ahead of the reduction (ring of " << ch << ")";
                return fail(SPIN_EUNSUPPORTED, os.str());
            }
            PassShape shp = dp.shape;
            shp.writes = dp.sp.passes[t].writes;
            HIP_TRY((launch_pass<T>(shp, psi, static_cast<const DevPass*>(dp.d_passes),
                                    static_cast<const DevStage*>(dp.d_stages),
                                    static_cast<const DevOp<T>*>(dp.d_ops), t, dp.tiles_per_wg,
                                    dp.nwg, part, off, ch, st)));
            for (size_t m = 0; m < dp.meas[t].size(); ++m) {
                int64_t& nx = next[dp.meas_site[t][m]];
                nx = std::max(nx, dp.meas[t][m] + off + 1);
            }
            complete = *std::min_element(next.begin(), next.end());
            if (complete - reduced >= ch / 2 || (l + 1 == nl && complete > reduced)) {
                HIP_TRY(launch_reduce_profile(part, dp.nwg, ch, M, reduced, complete - reduced, P, N, st));
                reduced = complete;
            }
        }
        if (reduced != total) {
            std::ostringstream os;
            os << "internal: profile plan measured " << reduced << " of " << total << " steps";
            return fail(SPIN_EUNSUPPORTED, os.str());
        }
        return SPIN_OK;
    };
    if (graph) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        return run_as_graph(GraphKey{&dp, psi, P, N, part, dev}, enqueue, st);
    }
    return enqueue(st);
}

template <typename T>
static int evolve_fused(void* psi, int M, const std::vector<Coupling>& J, double dt,
                        int64_t n_steps, int observed, double* P, double* N,
                        const spin_options* opt, bool profile, const Workspace* ws, hipStream_t st) {
    std::shared_ptr<DevicePlan> dp;
    Shape sh;
    const bool graph = opt && opt->use_graph;
    if (ws && (graph || profile))
        return fail(SPIN_EUNSUPPORTED, "the allocation-free call supports neither graph capture nor the "
                                       "all-site profile");
    int rc = get_plan(sizeof(T) == 4 ? SPIN_C64 : SPIN_C128, M, J, dt, n_steps, observed, opt,
                      profile, &dp, &sh, ws != nullptr);
    if (rc) return rc;
    if (profile) return evolve_profile<T>(psi, M, *dp, n_steps, P, N, graph, st);
    if (dp->resident) {
        ResidentJob job{};
        job.psi = psi;
        job.P = P;
        job.N = N;
        job.M = M;
        job.init = 0;
        job.pro_stage0 = dp->pro_stage0;
        job.pro_nstage = dp->pro_nstage;
        job.step_stage0 = dp->step_stage0;
        job.step_nstage = dp->step_nstage;
        HIP_TRY((launch_resident<T>(dp->res_r, dp->res_nt, job, nullptr, 1,
                                    static_cast<const DevStage*>(dp->d_stages),
                                    static_cast<const DevOp<T>*>(dp->d_ops), n_steps, st)));
        return SPIN_OK;
    }
    const int64_t total = n_steps + 1;
    int ch = int(std::min<int64_t>(total, 1024));
    void* scratch = nullptr;
    if (ws) {
        // as many step slots as the workspace holds; a launch measures at
        // most kMaxMeas consecutive steps and the slots are reduced once half
        // of them are in use, so 2 * kMaxMeas slots suffice
        const int64_t fit = int64_t(ws->doubles / (size_t(2) * size_t(dp->nwg)));
        ch = int(std::min<int64_t>(ch, fit));
        if (ch < std::min<int64_t>(total, 2 * kMaxMeas)) {
            std::ostringstream os;
            os << "workspace too small: " << dp->nwg << " workgroups need " << 2 * kMaxMeas * 2 * dp->nwg
               << " doubles, the allocation-free workspace holds " << ws->doubles;
            return fail(SPIN_EUNSUPPORTED, os.str());
        }
        scratch = ws->ptr;
    } else if ((rc = scratch_get(st, size_t(ch) * dp->nwg * 2 * sizeof(double), &scratch))) {
        return rc;
    }
    double* part = static_cast<double*>(scratch);
    auto enqueue = [&](hipStream_t st) -> int {
        int64_t measured = 0, reduced = 0;
        const size_t nl = dp->sp.launch_tmpl.size();
        for (size_t l = 0; l < nl; ++l) {
            const int t = dp->sp.launch_tmpl[l];
            const int64_t off = dp->sp.launch_offset[l];
            PassShape shp = dp->shape;
            shp.mats = static_cast<const float*>(dp->d_mats);
            shp.writes = dp->sp.passes[t].writes;
            HIP_TRY((launch_pass<T>(shp, psi, static_cast<const DevPass*>(dp->d_passes),
                                    static_cast<const DevStage*>(dp->d_stages),
                                    static_cast<const DevOp<T>*>(dp->d_ops), t, dp->tiles_per_wg,
                                    dp->nwg, part, off, ch, st)));
            for (int64_t s : dp->meas[t]) measured = std::max(measured, s + off + 1);
            if (measured - reduced >= ch / 2 || (l + 1 == nl && measured > reduced)) {
                HIP_TRY(launch_reduce(part, dp->nwg, ch, reduced, measured - reduced, P, N, st));
                reduced = measured;
            }
        }
        if (reduced != total) {
            std::ostringstream os;
            os << "internal: plan measured " << reduced << " of " << total << " steps";
            return fail(SPIN_EUNSUPPORTED, os.str());
        }
        return SPIN_OK;
    };
    if (graph) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        return run_as_graph(GraphKey{dp.get(), psi, P, N, part, dev}, enqueue, st);
    }
    return enqueue(st);
}

}  // namespace spinqp

using namespace spinqp;

extern "C" {

const char* spin_last_error(void) { return g_err.c_str(); }

const char* spin_version(void) { return "spinqp 0.1 (gfx950)"; }

int spin_init_random_phase(void* psi, int32_t prec, int32_t M, int32_t polarized_site,
                           uint64_t seed, void* stream) {
    int rc = validate_common(psi, prec, M);
    if (rc) return rc;
    if (polarized_site < 0 || polarized_site >= M) return fail(SPIN_EINVAL, "polarized_site out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = prec == SPIN_C64 ? launch_init<float>(psi, M, polarized_site, seed, st)
                                    : launch_init<double>(psi, M, polarized_site, seed, st);
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("init launch: ") + hipGetErrorString(e));
    g_err.clear();
    return SPIN_OK;
}

int spin_init_product(void* psi, int32_t prec, int32_t M, int32_t polarized_site, uint64_t seed,
                      void* stream) {
    int rc = validate_common(psi, prec, M);
    if (rc) return rc;
    if (polarized_site < 0 || polarized_site >= M) return fail(SPIN_EINVAL, "polarized_site out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = prec == SPIN_C64 ? launch_init_product<float>(psi, M, polarized_site, seed, st)
                                    : launch_init_product<double>(psi, M, polarized_site, seed, st);
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("init launch: ") + hipGetErrorString(e));
    g_err.clear();
    return SPIN_OK;
}

int spin_local_polarization_ex(const void* psi, int32_t prec, int32_t M, int32_t site,
                               double* P_dev, double* N_dev, void* stream) {
    int rc = validate_common(psi, prec, M);
    if (rc) return rc;
    if (site < 0 || site >= M) return fail(SPIN_EINVAL, "site out of range");
    if (!P_dev) return fail(SPIN_EINVAL, "P_dev is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblk = 1024;
    void* scratch = nullptr;
    if ((rc = scratch_get(st, size_t(nblk) * 2 * sizeof(double), &scratch))) return rc;
    double* part = static_cast<double*>(scratch);
    hipError_t e = prec == SPIN_C64 ? launch_observe<float>(psi, M, site, part, nblk, st)
                                    : launch_observe<double>(psi, M, site, part, nblk, st);
    if (e == hipSuccess) e = launch_reduce(part, nblk, 1, 0, 1, P_dev, N_dev, st);
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("observe launch: ") + hipGetErrorString(e));
    g_err.clear();
    return SPIN_OK;
}

int spin_local_polarization(const void* psi, int32_t prec, int32_t M, int32_t site, double* P_dev,
                            void* stream) {
    return spin_local_polarization_ex(psi, prec, M, site, P_dev, nullptr, stream);
}

}  // extern "C"

namespace spinqp {
// Shared body of spin_trotter_evolve_ex (one observed site) and
// spin_trotter_evolve_profile (every site; the norm rides on site 0).
static int evolve_entry(void* psi, int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                        double dt, int64_t n_steps, int32_t observed_site, bool profile,
                        double* P_dev, double* N_dev, const spin_options* opt, void* stream,
                        const Workspace* ws = nullptr) {
    try {
        int rc = validate_common(psi, prec, M);
        if (rc) return rc;
        if (!P_dev) return fail(SPIN_EINVAL, profile ? "Pall_dev is NULL" : "P_dev is NULL");
        if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
        if (n_steps < 0) return fail(SPIN_EINVAL, "n_steps < 0");
        if (observed_site < 0 || observed_site >= M) return fail(SPIN_EINVAL, "observed_site out of range");
        if (opt && (opt->schedule < 0 || opt->schedule > 1)) return fail(SPIN_EINVAL, "bad schedule option");
        if (opt && (opt->engine < 0 || opt->engine > 1)) return fail(SPIN_EINVAL, "bad engine option");
        if (opt && (opt->exchange < 0 || opt->exchange > 2)) return fail(SPIN_EINVAL, "bad exchange option");
        if (opt && opt->engine == 1 && opt->exchange == 2)
            return fail(SPIN_EUNSUPPORTED, "the matrix engine exchanges whole tiles");
        if (profile && opt && opt->engine != 0)
            return fail(SPIN_EUNSUPPORTED, "the all-site profile runs on the butterfly engine only");
        std::vector<Coupling> Jv;
        if ((rc = validate_couplings(M, J, K, &Jv))) return rc;
        hipStream_t st = static_cast<hipStream_t>(stream);
        const bool naive = opt && opt->schedule == 1;
        if (naive) {
            rc = prec == SPIN_C64
                     ? evolve_naive<float>(psi, M, Jv, dt, n_steps, observed_site, P_dev, N_dev, profile, ws, st)
                     : evolve_naive<double>(psi, M, Jv, dt, n_steps, observed_site, P_dev, N_dev, profile, ws, st);
        } else {
            rc = prec == SPIN_C64
                     ? evolve_fused<float>(psi, M, Jv, dt, n_steps, observed_site, P_dev, N_dev, opt, profile, ws, st)
                     : evolve_fused<double>(psi, M, Jv, dt, n_steps, observed_site, P_dev, N_dev, opt, profile, ws,
                                            st);
        }
        if (rc == SPIN_OK) g_err.clear();
        return rc;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
int evolve_with_workspace(void* psi, int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                          double dt, int64_t n_steps, int32_t observed_site, double* P_dev,
                          double* N_dev, const spin_options* opt, void* stream, double* ws,
                          size_t ws_doubles) {
    if (!ws) return fail(SPIN_EINVAL, "workspace is NULL");
    const Workspace w{ws, ws_doubles};
    return evolve_entry(psi, prec, M, J, K, dt, n_steps, observed_site, false, P_dev, N_dev, opt,
                        stream, &w);
}

}  // namespace spinqp

extern "C" {

int spin_trotter_evolve_ex(void* psi, int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                           double dt, int64_t n_steps, int32_t observed_site, double* P_dev,
                           double* N_dev, const spin_options* opt, void* stream) {
    return evolve_entry(psi, prec, M, J, K, dt, n_steps, observed_site, false, P_dev, N_dev, opt,
                        stream);
}

int spin_trotter_evolve_profile(void* psi, int32_t prec, int32_t M, const spin_coupling* J,
                                int32_t K, double dt, int64_t n_steps, double* Pall_dev,
                                double* N_dev, const spin_options* opt, void* stream) {
    return evolve_entry(psi, prec, M, J, K, dt, n_steps, 0, true, Pall_dev, N_dev, opt, stream);
}

int spin_prepare_plan(int32_t prec, int32_t M, const spin_coupling* J, int32_t K, double dt,
                      int64_t n_steps, int32_t observed_site, const spin_options* opt) {
    try {
        if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "prec must be SPIN_C64 or SPIN_C128");
        const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
        if (M < 1 || M > maxM) return fail(SPIN_EINVAL, "M out of range");
        if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
        if (n_steps < 0) return fail(SPIN_EINVAL, "n_steps < 0");
        const bool profile = observed_site == SPIN_ALL_SITES;
        if (profile) observed_site = 0;
        if (observed_site < 0 || observed_site >= M) return fail(SPIN_EINVAL, "observed_site out of range");
        if (opt && (opt->schedule < 0 || opt->schedule > 1)) return fail(SPIN_EINVAL, "bad schedule option");
        if (opt && (opt->engine < 0 || opt->engine > 1)) return fail(SPIN_EINVAL, "bad engine option");
        if (opt && (opt->exchange < 0 || opt->exchange > 2)) return fail(SPIN_EINVAL, "bad exchange option");
        if (opt && opt->engine == 1 && opt->exchange == 2)
            return fail(SPIN_EUNSUPPORTED, "the matrix engine exchanges whole tiles");
        if (profile && opt && opt->engine != 0)
            return fail(SPIN_EUNSUPPORTED, "the all-site profile runs on the butterfly engine only");
        std::vector<Coupling> Jv;
        int rc = validate_couplings(M, J, K, &Jv);
        if (rc) return rc;
        if (opt && opt->schedule == 1) {
            g_err.clear();
            return SPIN_OK;     // the unfused schedule has no plan
        }
        std::shared_ptr<DevicePlan> dp;
        rc = get_plan(prec, M, Jv, dt, n_steps, observed_site, opt, profile, &dp, nullptr);
        if (rc == SPIN_OK) g_err.clear();
        return rc;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}

int spin_trotter_evolve(void* psi, int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                        double dt, int64_t n_steps, int32_t observed_site, double* P_dev,
                        double* N_dev, void* stream) {
    return spin_trotter_evolve_ex(psi, prec, M, J, K, dt, n_steps, observed_site, P_dev, N_dev,
                                  nullptr, stream);
}

void spin_release_caches(void) {
    release_graphs();
    release_batch_caches();
    release_tune_cache();
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.clear();
    for (auto& kv : g_scratch)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    g_scratch.clear();
}

}  // extern "C"

// ---------------------------------------------------------- introspection
namespace {

int host_args(int32_t prec, int32_t M, const spin_coupling* J, int32_t K, double dt,
              int64_t n_steps, int32_t observed, std::vector<Coupling>* Jv) {
    if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "bad prec");
    const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
    if (M < 1 || M > maxM) return fail(SPIN_EINVAL, "M out of range");
    if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
    if (n_steps < 0) return fail(SPIN_EINVAL, "n_steps < 0");
    if ((observed < 0 || observed >= M) && observed != SPIN_ALL_SITES)
        return fail(SPIN_EINVAL, "observed_site out of range");
    return validate_couplings(M, J, K, Jv);
}

struct HostPlan {
    int path = 2;
    Shape sh;
    StreamPlan sp;
    ResidentPlan rp;
    int res_r = 0, res_nt = 0;
    bool profile = false;
};

int host_plan(int32_t prec, int32_t M, const std::vector<Coupling>& Jv, double dt, int64_t n_steps,
              int32_t observed, const spin_options* opt, HostPlan* hp) {
    if (opt && (opt->schedule < 0 || opt->schedule > 1)) return fail(SPIN_EINVAL, "bad schedule option");
    if (opt && (opt->engine < 0 || opt->engine > 1)) return fail(SPIN_EINVAL, "bad engine option");
    if (opt && (opt->exchange < 0 || opt->exchange > 2)) return fail(SPIN_EINVAL, "bad exchange option");
    if (opt && opt->engine == 1 && opt->exchange == 2)
        return fail(SPIN_EUNSUPPORTED, "the matrix engine exchanges whole tiles");
    const bool profile = observed == SPIN_ALL_SITES;
    if (profile) observed = 0;
    if (profile && opt && opt->engine != 0)
        return fail(SPIN_EUNSUPPORTED, "the all-site profile runs on the butterfly engine only");
    hp->profile = profile;
    hp->sh = choose_shape(prec, M, opt);
    if (!(opt && opt->schedule == 1) && !hp->sh.resident && !hp->sh.valid)
        return fail(SPIN_EUNSUPPORTED, "no pass kernel for the requested tile shape");
    const bool merge = !(opt && opt->no_merge);
    try {
        if (opt && opt->schedule == 1) {
            hp->path = 0;
        } else if (hp->sh.resident) {
            hp->path = 1;
            const int rmax = prec == SPIN_C64 ? 5 : 4;
            hp->res_r = std::min(rmax, int(M));
            hp->rp = plan_resident(M, Jv, dt, observed, merge, hp->res_r, profile);
        } else {
            hp->path = 2;
            PassParams pp;
            pp.k = hp->sh.k;
            pp.r = hp->sh.r;
            pp.c = hp->sh.c;
            pp.profile = profile;
            pp.half = hp->sh.half;
            if (profile) pp.max_meas = kMaxMeasProfile;
            hp->sp = plan_stream_best(M, Jv, dt, n_steps, observed, merge, pp);
        }
        // encode the tables as the evolve call would (nothing is uploaded),
        // so that the host-only calls report the errors that call would
        auto encode_all = [&](auto tag) {
            using T = decltype(tag);
            DevTables<T> tb;
            if (hp->path == 1) {
                encode_pass<T>(hp->rp.prologue, M, observed, tb, true, 0, profile);
                encode_pass<T>(hp->rp.step, M, observed, tb, true, 0, profile);
            } else if (hp->path == 2) {
                for (const HostPass& p : hp->sp.passes)
                    encode_pass<T>(p, M, observed, tb, false, hp->sh.engine, profile);
            }
        };
        if (prec == SPIN_C64) encode_all(float{});
        else encode_all(double{});
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("planning failed: ") + e.what());
    }
    return SPIN_OK;
}

}  // namespace

extern "C" int spin_describe_plan(int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                                  double dt, int64_t n_steps, int32_t observed_site,
                                  const spin_options* opt, spin_plan_info* info) {
    if (!info) return fail(SPIN_EINVAL, "info is NULL");
    std::vector<Coupling> Jv;
    int rc = host_args(prec, M, J, K, dt, n_steps, observed_site, &Jv);
    if (rc) return rc;
    HostPlan hp;
    if ((rc = host_plan(prec, M, Jv, dt, n_steps, observed_site, opt, &hp))) return rc;
    std::memset(info, 0, sizeof(*info));
    info->path = hp.path;
    if (hp.path == 0) {
        info->launches = n_steps * int64_t(2 * Jv.size());
        info->factor_ops = info->launches;
        info->passes_per_step = 2.0 * Jv.size();
    } else if (hp.path == 1) {
        info->tile_bits = M;
        info->reg_bits = hp.res_r;
        info->launches = 1;
        info->stages_total = int(hp.rp.prologue.stages.size() + hp.rp.step.stages.size());
        info->exchanges = int64_t(hp.rp.prologue.stages.size()) + n_steps * int64_t(hp.rp.step.stages.size());
        int64_t f = 0;
        for (const Op& op : hp.rp.step.ops) f += op.kind == 0;
        info->factor_ops = f * n_steps;
    } else {
        info->tile_bits = hp.sh.k;
        info->reg_bits = hp.sh.r;
        info->lanes = hp.sh.nt;
        info->coalesce_bits = hp.sh.c;
        info->engine = hp.sh.engine;
        info->exchange = hp.sh.half ? 2 : 1;
        info->templates = int(hp.sp.passes.size());
        info->period_steps = hp.sp.period_steps;
        info->period_passes = hp.sp.period_passes;
        int64_t st = 0;
        for (auto& p : hp.sp.passes) st += int64_t(p.stages.size());
        info->stages_total = int(st);
        info->launches = int64_t(hp.sp.launch_tmpl.size());
        int64_t f = 0;
        for (int t : hp.sp.launch_tmpl) {
            for (const Op& op : hp.sp.passes[t].ops) f += op.kind == 0;
            info->exchanges += int64_t(hp.sp.passes[t].stages.size()) - 1;
        }
        info->factor_ops = f;
        info->passes_per_step = hp.sp.passes_per_step();
    }
    g_err.clear();
    return SPIN_OK;
}

extern "C" int spin_plan_trace(int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                               double dt, int64_t n_steps, int32_t observed_site,
                               const spin_options* opt, double* buf, int64_t cap, int64_t* len) {
    if (!len) return fail(SPIN_EINVAL, "len is NULL");
    if (cap > 0 && !buf) return fail(SPIN_EINVAL, "buf is NULL with cap > 0");
    std::vector<Coupling> Jv;
    int rc = host_args(prec, M, J, K, dt, n_steps, observed_site, &Jv);
    if (rc) return rc;
    HostPlan hp;
    if ((rc = host_plan(prec, M, Jv, dt, n_steps, observed_site, opt, &hp))) return rc;
    int64_t n = 0;
    auto put = [&](double a, double b, double c, double d, double e) {
        if (n < cap) {
            double* r = buf + 5 * n;
            r[0] = a; r[1] = b; r[2] = c; r[3] = d; r[4] = e;
        }
        ++n;
    };
    auto put_pass = [&](const HostPass& p, int64_t off) {
        for (const HostStage& s : p.stages)
            for (int o : s.ops) {
                const Op& op = p.ops[o];
                if (op.kind == 1) put(1, double(op.step + off), op.i, 0, 0);
                else put(0, op.i, op.j, op.A, op.B);
            }
    };
    if (hp.path == 0) {
        const double tau = 0.5 * dt;
        auto observe = [&](int64_t k) {
            if (!hp.profile) put(1, double(k), observed_site, 0, 0);
            else for (int s = 0; s < M; ++s) put(1, double(k), s, 0, 0);
        };
        observe(0);
        for (int64_t k = 1; k <= n_steps; ++k) {
            for (size_t g = 0; g < Jv.size(); ++g) put(0, Jv[g].i, Jv[g].j, Jv[g].a * tau, Jv[g].b * tau);
            for (size_t g = Jv.size(); g-- > 0;) put(0, Jv[g].i, Jv[g].j, Jv[g].a * tau, Jv[g].b * tau);
            observe(k);
        }
    } else if (hp.path == 1) {
        put_pass(hp.rp.prologue, 0);
        for (int64_t k = 1; k <= n_steps; ++k) put_pass(hp.rp.step, k - 1);
    } else {
        for (size_t l = 0; l < hp.sp.launch_tmpl.size(); ++l)
            put_pass(hp.sp.passes[hp.sp.launch_tmpl[l]], hp.sp.launch_offset[l]);
    }
    *len = n;
    g_err.clear();
    return SPIN_OK;
}
