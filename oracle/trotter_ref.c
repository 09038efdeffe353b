/*
 * Plain C FP64 oracle of the random-phase Trotter loop (test infrastructure
 * only: called by the tests and by the CPU-baseline leg of the benchmark).
 *
 * Same algorithm, conventions and order as oracle/trotter.py:
 *  - initial state: the random-phase superposition of the section
 *    "Ensemble vs. pure entangled state" (alpha_i = sqrt(p_i) exp(i phi_i),
 *    p_i = 1/2^(M-1)), phases from the SplitMix64 counter generator
 *    (Steele, Lea & Flood, OOPSLA 2014), written here from its definition;
 *  - Hamiltonian of the section "Spin systems with different coupling
 *    networks"; each factor is exp(-i tau H_ij) applied exactly;
 *  - symmetric Strang step: couplings in list order, then reversed, each
 *    with tau = dt/2 (the paper names the Trotter-Suzuki decomposition but
 *    no scheme; this is the reading fixed for parity);
 *  - P[k] = sum_x (1 - 2 bit_n'(x)) |psi_x|^2, N[k] = sum_x |psi_x|^2.
 * One full pass over the state per factor; OpenMP over amplitude pairs;
 * no blocking, no fusion, no intrinsics.  psi is interleaved (re, im).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void oracle_init_random_phase(double *psi, int M, int n, uint64_t seed) {
    const int64_t dim = (int64_t)1 << M;
    const double amp = 1.0 / sqrt(ldexp(1.0, M - 1));
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; ++x) {
        if ((x >> n) & 1) { psi[2 * x] = 0.0; psi[2 * x + 1] = 0.0; continue; }
        uint64_t r = ((uint64_t)x & ((1ULL << n) - 1)) | (((uint64_t)x >> (n + 1)) << n);
        uint64_t z = sm64_mix(seed + (r + 1) * 0x9E3779B97F4A7C15ULL);
        double phi = two_pi * ((double)(z >> 11) * 0x1.0p-53);
        psi[2 * x] = amp * cos(phi);
        psi[2 * x + 1] = amp * sin(phi);
    }
}

static void apply_factor(double *psi, int M, int i, int j, double a, double b, double tau) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int64_t npairs = (int64_t)1 << (M - 2);
    const double t = 0.5 * b * tau, c = cos(t), s = sin(t);
    const double par = cos(0.25 * a * tau), pai = sin(0.25 * a * tau);  /* exp(+i a tau/4) */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npairs; ++p) {
        /* insert zero bits at positions lo and hi */
        int64_t x = p;
        x = ((x >> lo) << (lo + 1)) | (x & (((int64_t)1 << lo) - 1));
        x = ((x >> hi) << (hi + 1)) | (x & (((int64_t)1 << hi) - 1));
        const int64_t xa = x | ((int64_t)1 << j);   /* bit_i = 0, bit_j = 1 */
        const int64_t xb = x | ((int64_t)1 << i);   /* bit_i = 1, bit_j = 0 */
        const double ar = psi[2 * xa], ai = psi[2 * xa + 1];
        const double br = psi[2 * xb], bi = psi[2 * xb + 1];
        /* (c a - i s b, -i s a + c b) */
        double nar = c * ar + s * bi, nai = c * ai - s * br;
        double nbr = c * br + s * ai, nbi = c * bi - s * ar;
        if (a != 0.0) {
            double tr, ti;
            tr = par * nar - pai * nai; ti = par * nai + pai * nar; nar = tr; nai = ti;
            tr = par * nbr - pai * nbi; ti = par * nbi + pai * nbr; nbr = tr; nbi = ti;
            /* aligned configurations: exp(-i a tau/4) */
            const int64_t x0 = x, x1 = x | ((int64_t)1 << i) | ((int64_t)1 << j);
            double r0 = psi[2 * x0], i0 = psi[2 * x0 + 1];
            psi[2 * x0] = par * r0 + pai * i0; psi[2 * x0 + 1] = par * i0 - pai * r0;
            double r1 = psi[2 * x1], i1 = psi[2 * x1 + 1];
            psi[2 * x1] = par * r1 + pai * i1; psi[2 * x1 + 1] = par * i1 - pai * r1;
        }
        psi[2 * xa] = nar; psi[2 * xa + 1] = nai;
        psi[2 * xb] = nbr; psi[2 * xb + 1] = nbi;
    }
}

static void observe(const double *psi, int M, int site, double *P, double *N) {
    const int64_t dim = (int64_t)1 << M;
    double p = 0.0, nn = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : p, nn)
    for (int64_t x = 0; x < dim; ++x) {
        const double w = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
        nn += w;
        p += ((x >> site) & 1) ? -w : w;
    }
    *P = p; *N = nn;
}

void oracle_observe(const double *psi, int M, int site, double *P, double *N) {
    observe(psi, M, site, P, N);
}

/* Evolve psi in place for n_steps Strang steps; P, N have n_steps+1 entries. */
void oracle_trotter_run(double *psi, int M, int K, const int *ci, const int *cj,
                        const double *ca, const double *cb, double dt, int64_t n_steps,
                        int observed, double *P, double *N) {
    const double tau = 0.5 * dt;
    observe(psi, M, observed, &P[0], &N[0]);
    for (int64_t k = 1; k <= n_steps; ++k) {
        for (int g = 0; g < K; ++g) apply_factor(psi, M, ci[g], cj[g], ca[g], cb[g], tau);
        for (int g = K - 1; g >= 0; --g) apply_factor(psi, M, ci[g], cj[g], ca[g], cb[g], tau);
        observe(psi, M, observed, &P[k], &N[k]);
    }
}
