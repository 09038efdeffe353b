// ensemble.cpp -- spin_ensemble_evolve: the ensemble average of Eq. (1)
// by brute force, every basis-state member evolved on its own.
//
// Members are independent evolutions under one Hamiltonian, so 2^c of them
// are stacked as one state of M + c sites: the member index sits on the top
// c address bits, which no coupling touches.  One fused evolution of that
// state applies every factor to every member, and its observable, summed
// over the whole state, is the sum of the members' polarizations.  The
// evolutions run one after another over the member range, and their sums
// are accumulated on the device in member order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/spin.h"
#include "abi_internal.hpp"
#include "kernels.hpp"

using namespace spinqp;

namespace {

int ensemble_args(int32_t prec, int32_t M, const spin_coupling* J, int32_t K, double dt,
                  int64_t n_steps, int32_t polarized_site, int32_t observed_site,
                  int64_t first_member, int64_t n_members, void* work, int64_t work_amplitudes,
                  double* P_dev) {
    int rc = validate_common(work, prec, M);
    if (rc) return rc;
    if (!P_dev) return fail(SPIN_EINVAL, "P_dev is NULL");
    if (!std::isfinite(dt)) return fail(SPIN_EINVAL, "dt is not finite");
    if (n_steps < 0) return fail(SPIN_EINVAL, "n_steps < 0");
    if (polarized_site < 0 || polarized_site >= M) return fail(SPIN_EINVAL, "polarized_site out of range");
    if (observed_site < 0 || observed_site >= M) return fail(SPIN_EINVAL, "observed_site out of range");
    const int64_t members = int64_t(1) << (M - 1);
    if (n_members < 1) return fail(SPIN_EINVAL, "n_members < 1");
    if (first_member < 0 || first_member > members - n_members) {
        std::ostringstream os;
        os << "member range [" << first_member << ", +" << n_members << ") outside 0.." << members - 1;
        return fail(SPIN_EINVAL, os.str());
    }
    if (work_amplitudes < (int64_t(1) << M)) return fail(SPIN_EINVAL, "work holds fewer than 2^M amplitudes");
    std::vector<Coupling> Jv;
    return validate_couplings(M, J, K, &Jv);
}

// log2 of the members per evolution (see spin_ensemble_evolve).
int member_bits(int32_t prec, int32_t M, int64_t n_members, int64_t work_amplitudes) {
    const int maxM = prec == SPIN_C64 ? SPIN_MAX_M_C64 : SPIN_MAX_M_C128;
    int c = 0;
    while (M + c + 1 <= maxM && (int64_t(1) << (M + c + 1)) <= work_amplitudes &&
           (int64_t(1) << c) < n_members)
        ++c;
    return c;
}

}  // namespace

extern "C" int spin_ensemble_evolve(int32_t prec, int32_t M, const spin_coupling* J, int32_t K,
                                    double dt, int64_t n_steps, int32_t polarized_site,
                                    int32_t observed_site, int64_t first_member, int64_t n_members,
                                    void* work, int64_t work_amplitudes, double* P_dev,
                                    double* N_dev, const spin_options* opt, void* stream) {
    try {
        int rc = ensemble_args(prec, M, J, K, dt, n_steps, polarized_site, observed_site,
                               first_member, n_members, work, work_amplitudes, P_dev);
        if (rc) return rc;
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int c = member_bits(prec, M, n_members, work_amplitudes);
        const int64_t per = int64_t(1) << c;
        const int64_t chunks = (n_members + per - 1) / per;
        const int64_t len = n_steps + 1;
        double* tmp = nullptr;
        if (chunks > 1) {
            void* p = nullptr;
            if ((rc = scratch_get_slot(st, 1, size_t(2 * len) * sizeof(double), &p))) return rc;
            tmp = static_cast<double*>(p);
        }
        const double inv = 1.0 / double(n_members);
        for (int64_t q = 0; q < chunks; ++q) {
            const int64_t first = first_member + q * per;
            const int64_t count = std::min(per, n_members - q * per);
            hipError_t e = prec == SPIN_C64
                               ? launch_init_members<float>(work, M, c, polarized_site, uint64_t(first),
                                                            uint64_t(count), st)
                               : launch_init_members<double>(work, M, c, polarized_site, uint64_t(first),
                                                             uint64_t(count), st);
            if (e != hipSuccess) return fail(SPIN_EHIP, std::string("member init: ") + hipGetErrorString(e));
            double* Pq = q == 0 ? P_dev : tmp;
            double* Nq = N_dev ? (q == 0 ? N_dev : tmp + len) : nullptr;
            rc = spin_trotter_evolve_ex(work, prec, M + c, J, K, dt, n_steps, observed_site, Pq, Nq, opt,
                                        stream);
            if (rc) return rc;
            const double scale = q + 1 == chunks ? inv : 1.0;
            if (q > 0 || chunks == 1) {
                e = launch_accumulate(P_dev, q > 0 ? tmp : nullptr, len, scale, st);
                if (e == hipSuccess && N_dev) e = launch_accumulate(N_dev, q > 0 ? tmp + len : nullptr, len, scale, st);
                if (e != hipSuccess) return fail(SPIN_EHIP, std::string("member sum: ") + hipGetErrorString(e));
            }
        }
        fail(SPIN_OK, "");
        return SPIN_OK;
    } catch (const std::exception& e) {
        return fail(SPIN_EUNSUPPORTED, std::string("internal error: ") + e.what());
    }
}
