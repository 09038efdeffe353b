// autotune.cpp -- picks the launch shape of the tiled path (tile bits k,
// register bits, lanes, coalescing bits, VALU or MFMA stage arithmetic) for
// one problem by timing trial
// runs on the device, and keeps the choice in a process cache and,
// optionally, a JSON file.  Host code only: the trials run the library's own
// entry points on a scratch state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/spin.h"
#include "abi_internal.hpp"

namespace spinqp {
namespace {

struct Tuned {
    int tile_bits, reg_bits, coalesce_bits, engine, exchange;
    double ms_per_step;
};

// Length of the run whose plan scales the trial time per pass.
constexpr int64_t kTuneLongSteps = 1000;

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;

// FNV-1a over the bytes that determine a plan.
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
};

int tune_key(int32_t prec, int32_t M, const std::vector<Coupling>& J, double dt, int32_t observed,
             std::string* key) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SPIN_EHIP, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(SPIN_EHIP, "hipGetDeviceProperties failed");
    Fnv f;
    f.add(&dt, sizeof dt);
    for (const Coupling& c : J) {
        f.add(&c.i, sizeof c.i);
        f.add(&c.j, sizeof c.j);
        f.add(&c.a, sizeof c.a);
        f.add(&c.b, sizeof c.b);
    }
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%s/M%d/cu%d/obs%d/%016" PRIx64, arch.c_str(),
                  prec == SPIN_C64 ? "c64" : "c128", M, prop.multiProcessorCount, observed, f.h);
    *key = buf;
    return SPIN_OK;
}

// Cache file: one JSON object; every entry on its own line, which is also
// how it is read back.
bool read_file(const char* path, std::map<std::string, Tuned>* out) {
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    while (std::getline(in, line)) {
        char key[200];
        Tuned t;
        if (std::sscanf(line.c_str(),
                        " \"%199[^\"]\": {\"tile_bits\": %d, \"reg_bits\": %d, \"coalesce_bits\": %d, "
                        "\"engine\": %d, \"exchange\": %d, \"ms_per_step\": %lf}",
                        key, &t.tile_bits, &t.reg_bits, &t.coalesce_bits, &t.engine, &t.exchange,
                        &t.ms_per_step) == 7)
            (*out)[key] = t;
    }
    return true;
}

int write_file(const char* path, const std::map<std::string, Tuned>& entries) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return fail(SPIN_EINVAL, std::string("cannot write ") + tmp);
        out << "{\n \"format\": \"spinqp-autotune-2\",\n \"entries\": {\n";
        size_t n = 0;
        for (const auto& kv : entries) {
            char line[400];
            std::snprintf(line, sizeof line,
                          "  \"%s\": {\"tile_bits\": %d, \"reg_bits\": %d, \"coalesce_bits\": %d, "
                          "\"engine\": %d, \"exchange\": %d, \"ms_per_step\": %.6f}%s\n",
                          kv.first.c_str(), kv.second.tile_bits, kv.second.reg_bits,
                          kv.second.coalesce_bits, kv.second.engine, kv.second.exchange,
                          kv.second.ms_per_step, ++n < entries.size() ? "," : "");
            out << line;
        }
        out << " }\n}\n";
        if (!out) return fail(SPIN_EINVAL, std::string("cannot write ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(SPIN_EINVAL, std::string("cannot replace ") + path);
    return SPIN_OK;
}

spin_options to_options(const Tuned& t) {
    spin_options o;
    std::memset(&o, 0, sizeof o);
    o.tile_bits = t.tile_bits;
    o.reg_bits = t.reg_bits;
    o.coalesce_bits = t.coalesce_bits;
    o.engine = t.engine;
    o.exchange = t.exchange;
    return o;
}

// Candidate launch shapes; the first is the library default.  The MFMA
// matrix engine is not among them: a dense stage matrix costs about 20x the
// flops of the butterflies it replaces and it removes no LDS exchange, so it
// never wins on these workloads (it stays selectable through spin_options).
// Exchange 2 = half tiles (two workgroups per CU; one for complex128 tiles
// of 2^14), 1 = whole tiles.
std::vector<Tuned> candidates(int32_t prec) {
    if (prec == SPIN_C64)
        return {{14, 5, 4, 0, 2, 0}, {14, 5, 5, 0, 2, 0}, {14, 5, 6, 0, 2, 0}, {14, 6, 4, 0, 2, 0},
                {14, 5, 4, 0, 1, 0}, {14, 5, 6, 0, 1, 0}, {14, 4, 4, 0, 1, 0}, {13, 5, 5, 0, 1, 0},
                {13, 4, 4, 0, 1, 0}};
    return {{13, 4, 4, 0, 2, 0}, {13, 5, 4, 0, 2, 0}, {14, 5, 4, 0, 2, 0}, {13, 4, 4, 0, 1, 0},
            {13, 5, 4, 0, 1, 0}, {12, 4, 4, 0, 1, 0}};
}

struct DeviceBuffers {
    void* psi = nullptr;
    double* P = nullptr;
    double* N = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~DeviceBuffers() {
        if (psi) (void)hipFree(psi);
        if (P) (void)hipFree(P);
        if (N) (void)hipFree(N);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

void release_tune_cache() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

}  // namespace spinqp

using namespace spinqp;

extern "C" int spin_autotune(int32_t prec, int32_t M, const spin_coupling* J, int32_t K, double dt,
                             int32_t observed_site, int64_t trial_steps, const char* cache_path,
                             spin_options* best, spin_tune_result* results, int32_t cap,
                             int32_t* n_results, void* stream) {
    try {
        if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "prec must be SPIN_C64 or SPIN_C128");
        const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
        if (M < 1 || M > maxM) return fail(SPIN_EINVAL, "M out of range");
        if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
        if (observed_site < 0 || observed_site >= M) return fail(SPIN_EINVAL, "observed_site out of range");
        if (trial_steps < 1) return fail(SPIN_EINVAL, "trial_steps < 1");
        if (cap < 0 || (cap > 0 && !results)) return fail(SPIN_EINVAL, "results is NULL with cap > 0");
        std::vector<Coupling> Jv;
        int rc = validate_couplings(M, J, K, &Jv);
        if (rc) return rc;
        std::string key;
        if ((rc = tune_key(prec, M, Jv, dt, observed_site, &key))) return rc;
        hipStream_t st = static_cast<hipStream_t>(stream);

        std::vector<Tuned> cand = candidates(prec);
        if (choose_shape(prec, M, nullptr).resident) cand.resize(1);   // one workgroup: nothing to tune
        DeviceBuffers b;
        const size_t elem = prec == SPIN_C64 ? 8 : 16;
        if (hipMalloc(&b.psi, elem << M) != hipSuccess) return fail(SPIN_ENOMEM, "autotune state allocation failed");
        if (hipMalloc(reinterpret_cast<void**>(&b.P), sizeof(double) * size_t(trial_steps + 1)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&b.N), sizeof(double) * size_t(trial_steps + 1)) != hipSuccess)
            return fail(SPIN_ENOMEM, "autotune buffer allocation failed");
        if (hipEventCreate(&b.e0) != hipSuccess || hipEventCreate(&b.e1) != hipSuccess)
            return fail(SPIN_EHIP, "hipEventCreate failed");

        // A short trial measures the time of one pass launch of each shape;
        // the ranking scales it by the passes per step of a long run's plan
        // (host planning only), whose repeating block a short trial's plan
        // does not reach.
        const int64_t long_steps = std::max<int64_t>(trial_steps, kTuneLongSteps);
        // 1) every candidate: a timed trial of trial_steps steps
        struct Trial {
            int status = SPIN_OK;
            double trial = -1.0;       // ms per step of the trial
            double per_launch = -1.0;  // ms per pass launch of the trial (tiled path)
            double pps = 0.0;          // passes per step reported
        };
        std::vector<Trial> tr(cand.size());
        for (size_t ci = 0; ci < cand.size(); ++ci) {
            spin_options o = to_options(cand[ci]);
            spin_plan_info info;
            std::memset(&info, 0, sizeof info);
            int crc = spin_prepare_plan(prec, M, J, K, dt, trial_steps, observed_site, &o);
            if (crc == SPIN_OK) crc = spin_describe_plan(prec, M, J, K, dt, trial_steps, observed_site, &o, &info);
            if (crc == SPIN_OK) crc = spin_init_random_phase(b.psi, prec, M, 0, 1, st);
            if (crc == SPIN_OK)   // warm-up
                crc = spin_trotter_evolve_ex(b.psi, prec, M, J, K, dt, trial_steps, observed_site, b.P, b.N, &o, st);
            float ms = -1.0f;
            if (crc == SPIN_OK) {
                if (hipEventRecord(b.e0, st) != hipSuccess) return fail(SPIN_EHIP, "hipEventRecord failed");
                crc = spin_trotter_evolve_ex(b.psi, prec, M, J, K, dt, trial_steps, observed_site, b.P, b.N, &o, st);
                if (hipEventRecord(b.e1, st) != hipSuccess || hipEventSynchronize(b.e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, b.e0, b.e1) != hipSuccess)
                    return fail(SPIN_EHIP, "autotune timing failed");
            }
            tr[ci].status = crc;
            tr[ci].pps = info.passes_per_step;
            if (crc == SPIN_OK) {
                tr[ci].trial = double(ms) / double(trial_steps);
                // one workgroup holds the state: one launch, nothing to scale
                if (info.path == 2 && info.launches > 0) tr[ci].per_launch = double(ms) / double(info.launches);
            }
            cand[ci].ms_per_step = tr[ci].trial;
        }
        // 2) the candidates within 20% of the fastest trial (at most five):
        //    time per launch x passes per step of their long-run plan
        //    (host planning only)
        std::vector<int> order;
        for (size_t ci = 0; ci < cand.size(); ++ci)
            if (tr[ci].status == SPIN_OK) order.push_back(int(ci));
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return tr[a].trial < tr[c].trial; });
        int ibest = order.empty() ? -1 : order[0];
        double best_pred = order.empty() ? 0.0 : tr[order[0]].trial;
        for (size_t n = 0; n < order.size() && n < 5; ++n) {
            const int ci = order[n];
            if (tr[ci].trial > 1.2 * tr[order[0]].trial || tr[ci].per_launch < 0) continue;
            spin_options o = to_options(cand[ci]);
            spin_plan_info linfo;
            std::memset(&linfo, 0, sizeof linfo);
            if (spin_describe_plan(prec, M, J, K, dt, long_steps, observed_site, &o, &linfo) != SPIN_OK) continue;
            tr[ci].pps = linfo.passes_per_step;
            cand[ci].ms_per_step = tr[ci].per_launch * linfo.passes_per_step;
            if (n == 0 || cand[ci].ms_per_step < best_pred) {
                best_pred = cand[ci].ms_per_step;
                ibest = ci;
            }
        }
        int nres = 0;
        for (size_t ci = 0; ci < cand.size(); ++ci, ++nres) {
            if (nres >= cap) continue;
            spin_tune_result& r = results[nres];
            std::memset(&r, 0, sizeof r);
            r.opt = to_options(cand[ci]);
            r.ms_per_step = cand[ci].ms_per_step;
            r.trial_ms_per_step = tr[ci].trial;
            r.passes_per_step = tr[ci].pps;
            r.status = tr[ci].status;
        }
        if (n_results) *n_results = nres;
        if (hipStreamSynchronize(st) != hipSuccess) return fail(SPIN_EHIP, "hipStreamSynchronize failed");
        if (ibest < 0) return fail(SPIN_EUNSUPPORTED, "no candidate shape ran");
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[key] = cand[ibest];
        }
        if (cache_path) {
            std::map<std::string, Tuned> entries;
            read_file(cache_path, &entries);
            entries[key] = cand[ibest];
            if ((rc = write_file(cache_path, entries))) return rc;
        }
        if (best) *best = to_options(cand[ibest]);
        return fail(SPIN_OK, "");
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}

extern "C" int spin_tuned_options(int32_t prec, int32_t M, const spin_coupling* J, int32_t K, double dt,
                                  int32_t observed_site, const char* cache_path, spin_options* best) {
    try {
        if (!best) return fail(SPIN_EINVAL, "best is NULL");
        if (prec != SPIN_C64 && prec != SPIN_C128) return fail(SPIN_EINVAL, "prec must be SPIN_C64 or SPIN_C128");
        const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
        if (M < 1 || M > maxM) return fail(SPIN_EINVAL, "M out of range");
        if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
        if (observed_site < 0 || observed_site >= M) return fail(SPIN_EINVAL, "observed_site out of range");
        std::vector<Coupling> Jv;
        int rc = validate_couplings(M, J, K, &Jv);
        if (rc) return rc;
        std::string key;
        if ((rc = tune_key(prec, M, Jv, dt, observed_site, &key))) return rc;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                *best = to_options(it->second);
                return fail(SPIN_OK, "");
            }
        }
        if (cache_path) {
            std::map<std::string, Tuned> entries;
            read_file(cache_path, &entries);
            auto it = entries.find(key);
            if (it != entries.end()) {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tuned[key] = it->second;
                *best = to_options(it->second);
                return fail(SPIN_OK, "");
            }
        }
        return fail(SPIN_ENOTFOUND, "no autotuned entry for these arguments (key " + key + ")");
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
