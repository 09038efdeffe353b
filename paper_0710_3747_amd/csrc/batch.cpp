// batch.cpp -- spin_trotter_evolve_batch: many independent problems of
// uneven size in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <sstream>
#include <vector>

#include "../../include/spin.h"
#include "abi_internal.hpp"
#include "kernels.hpp"
#include "planner.hpp"

namespace spinqp {

template <typename T>
static int batch_resident(const spin_problem* probs, int32_t n, const std::vector<std::vector<Coupling>>& Js,
                          double dt, int64_t n_steps, int init, hipStream_t st) {
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
        for (int p : idx) {
            const spin_problem& pr = probs[p];
            ResidentPlan rp;
            try {
                rp = plan_resident(pr.M, Js[p], dt, pr.observed_site, true, g.first.first);
            } catch (const std::exception& e) {
                return fail(SPIN_EUNSUPPORTED, std::string("planning failed: ") + e.what());
            }
            ResidentJob j{};
            j.psi = pr.psi;
            j.P = pr.P_dev;
            j.N = pr.N_dev;
            j.seed = pr.seed;
            j.M = pr.M;
            j.polarized = pr.polarized_site;
            j.init = init ? 1 : 0;
            const int nthreads = 1 << std::max(0, pr.M - g.first.first);
            j.pro_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.prologue, pr.M, pr.observed_site, g.first.first, nthreads, 1, tb, true);
            j.pro_nstage = int(tb.stages.size()) - j.pro_stage0;
            j.step_stage0 = int(tb.stages.size());
            encode_pass<T>(rp.step, pr.M, pr.observed_site, g.first.first, nthreads, 1, tb, true);
            j.step_nstage = int(tb.stages.size()) - j.step_stage0;
            jobs.push_back(j);
        }
        // tables live until the launch has run: allocate, copy, launch, free
        // after synchronising the stream (batch calls are not on hot loops)
        void *d_jobs = nullptr, *d_st = nullptr, *d_ops = nullptr;
        auto cleanup = [&]() {
            if (d_jobs) (void)hipFree(d_jobs);
            if (d_st) (void)hipFree(d_st);
            if (d_ops) (void)hipFree(d_ops);
        };
        if (hipMalloc(&d_jobs, jobs.size() * sizeof(ResidentJob)) != hipSuccess ||
            hipMalloc(&d_st, std::max<size_t>(16, tb.stages.size() * sizeof(DevStage))) != hipSuccess ||
            hipMalloc(&d_ops, std::max<size_t>(16, tb.ops.size() * sizeof(DevOp<T>))) != hipSuccess) {
            cleanup();
            return fail(SPIN_ENOMEM, "batch table allocation failed");
        }
        hipError_t e = hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(ResidentJob),
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !tb.stages.empty())
            e = hipMemcpyAsync(d_st, tb.stages.data(), tb.stages.size() * sizeof(DevStage),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !tb.ops.empty())
            e = hipMemcpyAsync(d_ops, tb.ops.data(), tb.ops.size() * sizeof(DevOp<T>),
                               hipMemcpyHostToDevice, st);
        ResidentJob none{};
        if (e == hipSuccess)
            e = launch_resident<T>(g.first.first, g.first.second, none,
                                   static_cast<const ResidentJob*>(d_jobs), int(jobs.size()),
                                   static_cast<const DevStage*>(d_st),
                                   static_cast<const DevOp<T>*>(d_ops), n_steps, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        cleanup();
        if (e != hipSuccess) return fail(SPIN_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    return SPIN_OK;
}

}  // namespace spinqp

using namespace spinqp;

extern "C" int spin_trotter_evolve_batch(const spin_problem* probs, int32_t n,
                                         const spin_coupling* J_all, int64_t K_total,
                                         int32_t prec, double dt, int64_t n_steps,
                                         int32_t init_random_phase, void* stream) {
    try {
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
            if (init_random_phase && (pr.polarized_site < 0 || pr.polarized_site >= pr.M))
                return fail(SPIN_EINVAL, os.str() + "polarized_site out of range");
            if (pr.K < 0 || pr.coupling_offset < 0 || pr.coupling_offset + pr.K > K_total)
                return fail(SPIN_EINVAL, os.str() + "coupling range outside J_all");
            rc = validate_couplings(pr.M, J_all + pr.coupling_offset, pr.K, &Js[p]);
            if (rc) return fail(rc, os.str() + spin_last_error());
            if (pr.M > cap) return fail(SPIN_EUNSUPPORTED, os.str() + "M above the one-workgroup capacity");
        }
        if (n == 0) return SPIN_OK;
        hipStream_t st = static_cast<hipStream_t>(stream);
        int rc = prec == SPIN_C64 ? batch_resident<float>(probs, n, Js, dt, n_steps, init_random_phase, st)
                                  : batch_resident<double>(probs, n, Js, dt, n_steps, init_random_phase, st);
        return rc;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
