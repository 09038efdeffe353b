// batch.cpp -- spin_trotter_evolve_batch: many independent problems of
// uneven size in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <vector>

#include "../../include/spin.h"
#include "abi_internal.hpp"
#include "kernels.hpp"
#include "planner.hpp"

namespace spinqp {

// Device tables of the grouped one-workgroup launches of one batch call,
// kept (like the persistent launch's) until spin_release_caches so the call
// can return without waiting for the launches.
struct ResidentBatch {
    struct Group {
        int r = 0, nt = 0, njobs = 0;
        void *d_jobs = nullptr, *d_st = nullptr, *d_ops = nullptr;
    };
    std::vector<Group> groups;
    ~ResidentBatch() {
        for (Group& g : groups)
            for (void* p : {g.d_jobs, g.d_st, g.d_ops})
                if (p) (void)hipFree(p);
    }
};

static std::mutex g_rmu;
static std::map<std::vector<double>, std::shared_ptr<ResidentBatch>> g_rcache;

static std::vector<double> batch_key(const spin_problem* probs, int n,
                                     const std::vector<std::vector<Coupling>>& Js, int prec,
                                     double dt, int64_t n_steps, int init, int dev);

template <typename T>
static int batch_resident_build(const spin_problem* probs, int32_t n,
                                const std::vector<std::vector<Coupling>>& Js, double dt, int init,
                                ResidentBatch* rb) {
    // group problems by kernel shape; each group is one launch with one
    // workgroup per problem, largest states first
    const int rmax = sizeof(T) == 4 ? 5 : 4;
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int p = 0; p < n; ++p) {
        const int M = probs[p].M;
        const int r = std::min(rmax, M);
        const int tb = M - r;
        const int nt = tb <= 6 ? 64 : (tb <= 8 ? 256 : 512);
        groups[{r, nt}].push_back(p);
    }
    for (auto& g : groups) {
        std::vector<int>& idx = g.second;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return probs[a].M > probs[b].M; });
        DevTables<T> tb;
        std::vector<ResidentJob> jobs;
        std::map<std::vector<double>, ResidentJob> shared;   // equal problems share tables
        for (int p : idx) {
            const spin_problem& pr = probs[p];
            std::vector<double> skey{double(pr.M), double(pr.observed_site)};
            for (const Coupling& c : Js[p]) {
                skey.push_back(c.i);
                skey.push_back(c.j);
                skey.push_back(c.a);
                skey.push_back(c.b);
            }
            ResidentJob j{};
            auto hit = shared.find(skey);
            if (hit != shared.end()) j = hit->second;
            j.psi = pr.psi;
            j.P = pr.P_dev;
            j.N = pr.N_dev;
            j.seed = pr.seed;
            j.M = pr.M;
            j.polarized = pr.polarized_site;
            j.init = init;
            if (hit != shared.end()) {
                jobs.push_back(j);
                continue;
            }
            ResidentPlan rp;
            try {
                rp = plan_resident(pr.M, Js[p], dt, pr.observed_site, true, g.first.first);
            } catch (const std::exception& e) {
                return fail(SPIN_EUNSUPPORTED, std::string("planning failed: ") + e.what());
            }
            j.pro_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.prologue, pr.M, pr.observed_site, tb, true);
            j.pro_nstage = int(tb.stages.size()) - j.pro_stage0;
            j.step_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.step, pr.M, pr.observed_site, tb, true);
            j.step_nstage = int(tb.stages.size()) - j.step_stage0;
            shared[skey] = j;
            jobs.push_back(j);
        }
        ResidentBatch::Group gr;
        gr.r = g.first.first;
        gr.nt = g.first.second;
        gr.njobs = int(jobs.size());
        rb->groups.push_back(gr);
        ResidentBatch::Group& G = rb->groups.back();
        auto up = [&](const void* src, size_t bytes, void** dst) -> int {
            if (bytes == 0) bytes = 16;
            if (hipMalloc(dst, bytes) != hipSuccess) return fail(SPIN_ENOMEM, "batch table allocation failed");
            if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
                return fail(SPIN_EHIP, "batch table upload failed");
            return SPIN_OK;
        };
        int rc;
        if ((rc = up(jobs.data(), jobs.size() * sizeof(ResidentJob), &G.d_jobs))) return rc;
        if ((rc = up(tb.stages.empty() ? nullptr : tb.stages.data(), tb.stages.size() * sizeof(DevStage),
                     &G.d_st)))
            return rc;
        if ((rc = up(tb.ops.empty() ? nullptr : tb.ops.data(), tb.ops.size() * sizeof(DevOp<T>), &G.d_ops)))
            return rc;
    }
    return SPIN_OK;
}

template <typename T>
static int batch_resident(const spin_problem* probs, int32_t n, const std::vector<std::vector<Coupling>>& Js,
                          int prec, double dt, int64_t n_steps, int init, hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SPIN_EHIP, "hipGetDevice failed");
    const std::vector<double> key = batch_key(probs, n, Js, prec, dt, n_steps, init, dev);
    std::shared_ptr<ResidentBatch> rb;
    {
        std::lock_guard<std::mutex> lk(g_rmu);
        auto it = g_rcache.find(key);
        if (it != g_rcache.end()) rb = it->second;
    }
    if (!rb) {
        rb = std::make_shared<ResidentBatch>();
        const int rc = batch_resident_build<T>(probs, n, Js, dt, init, rb.get());
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(g_rmu);
        g_rcache[key] = rb;
    }
    ResidentJob none{};
    for (const ResidentBatch::Group& G : rb->groups) {
        const hipError_t e = launch_resident<T>(G.r, G.nt, none, static_cast<const ResidentJob*>(G.d_jobs),
                                                G.njobs, static_cast<const DevStage*>(G.d_st),
                                                static_cast<const DevOp<T>*>(G.d_ops), n_steps, st);
        if (e != hipSuccess) return fail(SPIN_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    return SPIN_OK;
}


// ------------------------------------------------------- persistent batch
struct BatchCache {
    void *d_probs = nullptr, *d_jobs = nullptr, *d_jstart = nullptr, *d_passes = nullptr,
         *d_stages = nullptr, *d_ops = nullptr, *d_launch = nullptr, *d_part = nullptr,
         *d_ctr = nullptr, *d_err = nullptr;
    int nslots = 0, ncounters = 0;
    bool half = false;
    hipStream_t side = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    ~BatchCache() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (side) (void)hipStreamDestroy(side);
        for (void* p : {d_probs, d_jobs, d_jstart, d_passes, d_stages, d_ops, d_launch, d_part,
                        d_ctr, d_err})
            if (p) (void)hipFree(p);
    }
};

static std::mutex g_bmu;
static std::map<std::vector<double>, std::shared_ptr<BatchCache>> g_bcache;
// Per device: sticky status word of the persistent launches (non-zero once a
// gang barrier has timed out), read and cleared by spin_batch_status.
static std::map<int, int*> g_status;

static int status_word(int dev, int** out) {
    std::lock_guard<std::mutex> lk(g_bmu);
    int*& w = g_status[dev];
    if (!w) {
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(int)) != hipSuccess) return fail(SPIN_ENOMEM, "status word allocation failed");
        const int zero = 0;
        if (hipMemcpy(p, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(p);
            return fail(SPIN_EHIP, "status word initialisation failed");
        }
        w = static_cast<int*>(p);
    }
    *out = w;
    return SPIN_OK;
}

void release_batch_caches() {
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        g_bcache.clear();
        for (auto& kv : g_status)
            if (kv.second) (void)hipFree(kv.second);
        g_status.clear();
    }
    std::lock_guard<std::mutex> lk(g_rmu);
    g_rcache.clear();
}

// Key: everything the tables and the launch depend on.
static std::vector<double> batch_key(const spin_problem* probs, int n,
                                     const std::vector<std::vector<Coupling>>& Js, int prec,
                                     double dt, int64_t n_steps, int init, int dev) {
    std::vector<double> k{double(prec), dt, double(n_steps), double(init), double(dev), double(n)};
    for (int p = 0; p < n; ++p) {
        const spin_problem& pr = probs[p];
        k.push_back(double(reinterpret_cast<uintptr_t>(pr.psi)));
        k.push_back(double(reinterpret_cast<uintptr_t>(pr.P_dev)));
        k.push_back(double(reinterpret_cast<uintptr_t>(pr.N_dev)));
        k.push_back(pr.M);
        k.push_back(pr.observed_site);
        k.push_back(pr.polarized_site);
        k.push_back(double(pr.seed >> 32));
        k.push_back(double(pr.seed & 0xffffffffu));
        for (const Coupling& c : Js[p]) {
            k.push_back(c.i);
            k.push_back(c.j);
            k.push_back(c.a);
            k.push_back(c.b);
        }
    }
    return k;
}

template <typename T>
static int batch_build(const spin_problem* probs, const std::vector<int>& sel,
                       const std::vector<std::vector<Coupling>>& Js, double dt, int64_t n_steps,
                       int init, int nslots, bool half, BatchCache* bc) {
    const bool f32 = sizeof(T) == 4;
    const int K = batch_tile_bits(f32), R = batch_shape(f32, half).r;
    const int KL = half ? K - 1 : K;    // largest problem held in LDS
    DevTables<T> tb;
    std::vector<BatchProblem> bp;
    std::vector<int2> launches;
    std::vector<double> dur;
    int64_t part = 0;
    int ncounter = 0;
    // problems with equal (M, observed site, couplings) share their tables
    // (e.g. the basis-state members of one ensemble)
    std::map<std::vector<double>, std::pair<BatchProblem, double>> shared;
    for (int p : sel) {
        const spin_problem& pr = probs[p];
        std::vector<double> skey{double(pr.M), double(pr.observed_site)};
        for (const Coupling& c : Js[p]) {
            skey.push_back(c.i);
            skey.push_back(c.j);
            skey.push_back(c.a);
            skey.push_back(c.b);
        }
        BatchProblem b{};
        double fops = 0;
        auto hit = shared.find(skey);
        if (hit != shared.end()) {
            b = hit->second.first;
            fops = hit->second.second;
            if (b.gsize > 1 || b.M > KL) {   // gang: own partial sums and counter
                b.part0 = part;
                part += int64_t(kBatchRing) * b.gsize * 2;
                b.counter = ncounter++;
            }
        }
        b.psi = pr.psi;
        b.P = pr.P_dev;
        b.N = pr.N_dev;
        b.seed = pr.seed;
        b.M = pr.M;
        b.polarized = pr.polarized_site;
        b.init = init;
        if (hit != shared.end()) {
            dur.push_back(fops);
            bp.push_back(b);
            continue;
        }
        if (pr.M <= KL) {
            ResidentPlan rp = plan_resident(pr.M, Js[p], dt, pr.observed_site, true, R);
            const int nthreads = 1 << (pr.M - R);
            b.gsize = 1;
            b.pro_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.prologue, pr.M, pr.observed_site, tb, true);
            b.pro_nstage = int(tb.stages.size()) - b.pro_stage0;
            b.step_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.step, pr.M, pr.observed_site, tb, true);
            b.step_nstage = int(tb.stages.size()) - b.step_stage0;
            for (const Op& op : rp.step.ops) fops += op.kind == 0;
            // on-chip: about half the cost per amplitude of a tiled pass
            fops = 0.5 * fops * std::ldexp(1.0, pr.M) * double(n_steps + 1);
            dur.push_back(fops);
        } else {
            PassParams pp;
            pp.k = K;
            pp.r = R;
            // the library's default launch shape; a gang plans one scheduling
            // variant (plan_stream), not the single path's variant search
            pp.c = 4;
            pp.half = half;
            StreamPlan sp = plan_stream(pr.M, Js[p], dt, n_steps, pr.observed_site, true, pp);
            b.pass0 = int(tb.passes.size());
            for (const HostPass& hp : sp.passes) encode_pass<T>(hp, pr.M, pr.observed_site, tb);
            b.launch0 = int64_t(launches.size());
            b.nlaunch = int(sp.launch_tmpl.size());
            for (size_t l = 0; l < sp.launch_tmpl.size(); ++l)
                launches.push_back(make_int2(sp.launch_tmpl[l], int(sp.launch_offset[l])));
            b.ntiles = int64_t(1) << (pr.M - K);
            // Gangs of at most 8 workgroups with half tiles (two per CU):
            // more problems run at once and fewer wait at each barrier; on
            // 256 stars of M 14..20 the batch took 1.85 s with 8, 1.94 s
            // with 16, 2.25 s with 32 and 2.61 s with 4.
            b.gsize = int(std::min<int64_t>(b.ntiles, half ? 8 : 32));
            b.part0 = part;
            part += int64_t(kBatchRing) * b.gsize * 2;
            b.counter = ncounter++;
            for (int t : sp.launch_tmpl)
                for (const Op& op : sp.passes[t].ops) fops += op.kind == 0;
            // factor work plus one sweep per launch, shared by the gang
            fops = (fops + 6.0 * sp.launch_tmpl.size()) * std::ldexp(1.0, pr.M) / b.gsize;
            dur.push_back(fops);
        }
        shared[skey] = {b, fops};
        bp.push_back(b);
    }
    // Gang schedule: slots w with the same w % 8 form an XCD group; longest
    // jobs first, each onto the group where its gang can start earliest.
    const int ngroup = nslots >= 8 ? 8 : 1;
    std::vector<double> avail(nslots, 0.0);
    std::vector<std::vector<BatchJob>> lists(nslots);
    std::vector<int> order(bp.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dur[a] > dur[b]; });
    for (int q : order) {
        const int g = bp[q].gsize;
        double best_start = 1e300;
        std::vector<int> best;
        for (int x = 0; x < ngroup; ++x) {
            std::vector<int> slots;
            for (int w = x; w < nslots; w += ngroup) slots.push_back(w);
            if (int(slots.size()) < g) continue;
            std::stable_sort(slots.begin(), slots.end(), [&](int a, int b) { return avail[a] < avail[b]; });
            slots.resize(g);
            double start = 0;
            for (int w : slots) start = std::max(start, avail[w]);
            if (start < best_start) {
                best_start = start;
                best = slots;
            }
        }
        if (best.empty()) throw std::runtime_error("batch: gang larger than an XCD group");
        std::sort(best.begin(), best.end());
        for (int r = 0; r < g; ++r) {
            lists[best[r]].push_back(BatchJob{q, r});
            avail[best[r]] = best_start + dur[q];
        }
    }
    std::vector<BatchJob> jobs;
    std::vector<int> jstart(nslots + 1, 0);
    for (int w = 0; w < nslots; ++w) {
        jstart[w] = int(jobs.size());
        jobs.insert(jobs.end(), lists[w].begin(), lists[w].end());
    }
    jstart[nslots] = int(jobs.size());

    auto up = [&](const void* src, size_t n, void** dst) -> int {
        if (n == 0) n = 16;
        if (hipMalloc(dst, n) != hipSuccess) return fail(SPIN_ENOMEM, "batch table allocation failed");
        if (src && hipMemcpy(*dst, src, n, hipMemcpyHostToDevice) != hipSuccess)
            return fail(SPIN_EHIP, "batch table upload failed");
        return SPIN_OK;
    };
    int rc;
    if ((rc = up(bp.data(), bp.size() * sizeof(BatchProblem), &bc->d_probs))) return rc;
    if ((rc = up(jobs.data(), jobs.size() * sizeof(BatchJob), &bc->d_jobs))) return rc;
    if ((rc = up(jstart.data(), jstart.size() * sizeof(int), &bc->d_jstart))) return rc;
    if ((rc = up(tb.passes.data(), tb.passes.size() * sizeof(DevPass), &bc->d_passes))) return rc;
    if ((rc = up(tb.stages.data(), tb.stages.size() * sizeof(DevStage), &bc->d_stages))) return rc;
    if ((rc = up(tb.ops.data(), tb.ops.size() * sizeof(DevOp<T>), &bc->d_ops))) return rc;
    if ((rc = up(launches.data(), launches.size() * sizeof(int2), &bc->d_launch))) return rc;
    if ((rc = up(nullptr, std::max<int64_t>(part, 2) * sizeof(double), &bc->d_part))) return rc;
    if ((rc = up(nullptr, std::max(ncounter, 1) * sizeof(int), &bc->d_ctr))) return rc;
    if ((rc = up(nullptr, sizeof(int), &bc->d_err))) return rc;
    bc->nslots = nslots;
    bc->half = half;
    bc->ncounters = std::max(ncounter, 1);
    return SPIN_OK;
}

template <typename T>
static int batch_persistent(const spin_problem* probs, const std::vector<int>& sel,
                            const std::vector<std::vector<Coupling>>& Js, int prec, double dt,
                            int64_t n_steps, int init, bool use_graph, bool half, hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SPIN_EHIP, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(SPIN_EHIP, "device query failed");
    const int nslots = prop.multiProcessorCount * (half ? 2 : 1);

    // key over the selected problems only
    std::vector<spin_problem> ps;
    std::vector<std::vector<Coupling>> js;
    for (int p : sel) {
        ps.push_back(probs[p]);
        js.push_back(Js[p]);
    }
    std::vector<double> key = batch_key(ps.data(), int(ps.size()), js, prec, dt, n_steps, init, dev);
    key.push_back(use_graph ? 1 : 0);
    key.push_back(half ? 1 : 0);
    std::shared_ptr<BatchCache> bc;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_bcache.find(key);
        if (it != g_bcache.end()) bc = it->second;
    }
    if (!bc) {
        bc = std::make_shared<BatchCache>();
        int rc;
        try {
            rc = batch_build<T>(probs, sel, Js, dt, n_steps, init, nslots, half, bc.get());
        } catch (const std::exception& e) {
            return fail(SPIN_EUNSUPPORTED, std::string("batch planning failed: ") + e.what());
        }
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(g_bmu);
        g_bcache[key] = bc;
    }
    int* status = nullptr;
    if (int rc = status_word(dev, &status)) return rc;
    auto enqueue = [&](hipStream_t s) {
        return launch_batch<T>(bc->nslots, bc->half, static_cast<const BatchProblem*>(bc->d_probs),
                               static_cast<const BatchJob*>(bc->d_jobs),
                               static_cast<const int*>(bc->d_jstart),
                               static_cast<const DevPass*>(bc->d_passes),
                               static_cast<const DevStage*>(bc->d_stages),
                               static_cast<const DevOp<T>*>(bc->d_ops),
                               static_cast<const int2*>(bc->d_launch),
                               static_cast<double*>(bc->d_part), static_cast<int*>(bc->d_ctr),
                               bc->ncounters, static_cast<int*>(bc->d_err), status, n_steps, s);
    };
    hipError_t e = hipSuccess;
    if (use_graph) {
        // capture on a library stream ordered after the caller's stream
        if (!bc->side && (e = hipStreamCreateWithFlags(&bc->side, hipStreamNonBlocking)) != hipSuccess)
            return fail(SPIN_EHIP, std::string("stream: ") + hipGetErrorString(e));
        if (!bc->exec) {
            e = hipStreamBeginCapture(bc->side, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = enqueue(bc->side);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(bc->side, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&bc->exec, g, nullptr, nullptr, 0);
            bc->graph = g;
            if (e != hipSuccess) return fail(SPIN_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return fail(SPIN_EHIP, "event create failed");
        e = hipEventRecord(ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(bc->side, ev, 0);
        if (e == hipSuccess) e = hipGraphLaunch(bc->exec, bc->side);
        if (e == hipSuccess) e = hipEventRecord(ev, bc->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
        (void)hipEventDestroy(ev);
    } else {
        e = enqueue(st);
    }
    if (e != hipSuccess) return fail(SPIN_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    return SPIN_OK;
}

}  // namespace spinqp

using namespace spinqp;

extern "C" int spin_trotter_evolve_batch(const spin_problem* probs, int32_t n,
                                         const spin_coupling* J_all, int64_t K_total,
                                         int32_t prec, double dt, int64_t n_steps,
                                         int32_t init, void* stream) {
    try {
        if (init < SPIN_INIT_NONE || init > SPIN_INIT_PRODUCT) return fail(SPIN_EINVAL, "bad init");
        if (n < 0) return fail(SPIN_EINVAL, "n < 0");
        if (n > 0 && !probs) return fail(SPIN_EINVAL, "probs is NULL");
        if (K_total < 0 || (K_total > 0 && !J_all)) return fail(SPIN_EINVAL, "bad J_all / K_total");
        if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
        if (n_steps < 0) return fail(SPIN_EINVAL, "n_steps < 0");
        if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "bad prec");
        std::vector<std::vector<Coupling>> Js(n);
        const int cap = prec == SPIN_C64 ? 14 : 13;
        for (int p = 0; p < n; ++p) {
            const spin_problem& pr = probs[p];
            std::ostringstream os;
            os << "problem " << p << ": ";
            int rc = validate_common(pr.psi, prec, pr.M);
            if (rc) return fail(rc, os.str() + spin_last_error());
            if (!pr.P_dev) return fail(SPIN_EINVAL, os.str() + "P_dev is NULL");
            if (pr.observed_site < 0 || pr.observed_site >= pr.M)
                return fail(SPIN_EINVAL, os.str() + "observed_site out of range");
            if ((init == SPIN_INIT_RANDOM_PHASE || init == SPIN_INIT_PRODUCT) &&
                (pr.polarized_site < 0 || pr.polarized_site >= pr.M))
                return fail(SPIN_EINVAL, os.str() + "polarized_site out of range");
            if (init == SPIN_INIT_BASIS && (pr.seed >> pr.M) != 0)
                return fail(SPIN_EINVAL, os.str() + "basis index (seed) >= 2^M");
            if (pr.K < 0 || pr.coupling_offset < 0 || pr.coupling_offset + pr.K > K_total)
                return fail(SPIN_EINVAL, os.str() + "coupling range outside J_all");
            rc = validate_couplings(pr.M, J_all + pr.coupling_offset, pr.K, &Js[p]);
            if (rc) return fail(rc, os.str() + spin_last_error());
        }
        (void)cap;
        if (n == 0) return SPIN_OK;
        hipStream_t st = static_cast<hipStream_t>(stream);
        // Two workgroups per CU with half-tile gangs when both fit (every
        // slot of the persistent launch must be resident at once), else one
        // with whole tiles.
        const bool f32 = prec == SPIN_C64;
        const bool half = batch_blocks_per_cu(f32, true) >= 2;
        if (!half && batch_blocks_per_cu(f32, false) < 1)
            return fail(SPIN_EUNSUPPORTED, "batch kernel does not fit a CU");
        // states smaller than a lane's registers: the grouped one-workgroup
        // launches; everything else: the persistent launch
        const int rmin = batch_shape(f32, half).r;
        std::vector<int> small, big;
        for (int p = 0; p < n; ++p) (probs[p].M < rmin ? small : big).push_back(p);
        int rc = SPIN_OK;
        if (!small.empty()) {
            std::vector<spin_problem> sp;
            std::vector<std::vector<Coupling>> sj;
            for (int p : small) {
                sp.push_back(probs[p]);
                sj.push_back(Js[p]);
            }
            rc = prec == SPIN_C64 ? batch_resident<float>(sp.data(), int(sp.size()), sj, prec, dt, n_steps, init, st)
                                  : batch_resident<double>(sp.data(), int(sp.size()), sj, prec, dt, n_steps, init, st);
            if (rc) return rc;
        }
        if (!big.empty()) {
            const bool graph = true;
            rc = f32 ? batch_persistent<float>(probs, big, Js, prec, dt, n_steps, init, graph, half, st)
                     : batch_persistent<double>(probs, big, Js, prec, dt, n_steps, init, graph, half, st);
        }
        if (rc == SPIN_OK) fail(SPIN_OK, "");
        return rc;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}

extern "C" int spin_batch_status(void* stream) {
    try {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return fail(SPIN_EHIP, std::string("batch status: ") + hipGetErrorString(e));
        int* w = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_bmu);
            auto it = g_status.find(dev);
            if (it != g_status.end()) w = it->second;
        }
        if (!w) {
            fail(SPIN_OK, "");
            return SPIN_OK;      // no persistent launch on this device yet
        }
        int v = 0;
        const int zero = 0;
        e = hipMemcpy(&v, w, sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess && v != 0) e = hipMemcpy(w, &zero, sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(SPIN_EHIP, std::string("batch status: ") + hipGetErrorString(e));
        if (v != 0)
            return fail(SPIN_EHIP, "batch: a gang barrier timed out (workgroups not co-resident?); "
                                   "the affected problems' P were set to NaN");
        fail(SPIN_OK, "");
        return SPIN_OK;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
