// Host check of the tiled-pass tables (test program; links the planner).
//
// Reads "M prec k r c n_steps observed plant half" and then K lines
// "i j a b" on stdin,
// plans the call as the library does (plan_stream_best), encodes every pass
// and checks, by emulating the kernel's address arithmetic, the invariants
// that let a stage exchange or a tile boundary go without a workgroup
// barrier:
//  * an exchange marked wave-local (xnext = 0): every wave scatters to
//    exactly the LDS slots it gathers from next;
//  * a pass without the tile-end barrier: every wave's LDS slots in the last
//    stage are its slots in the first stage;
//  * a multi-stage pass with no barrier in any exchange: every wave stores
//    exactly the global offsets it loaded (no wave's store can overtake
//    another wave's load of the same tile);
//  * every stage's LDS map is a bijection onto the tile, or for half-tile
//    exchanges (half = 1) onto half a tile, with the split position (the top
//    register bit) mapped to no offset.
// Prints one summary line; exit status 0 when every check holds.  With a
// non-zero 8th header value every exchange is marked wave-local before the
// checks (a planted mistake the checks must report).
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../../paper_0710_3747_amd/csrc/planner.hpp"

using namespace spinqp;

static uint32_t lds_addr(const DevStage& S, int ntb, int rr, uint32_t tid, uint32_t j) {
    uint32_t a = 0;
    for (int q = 0; q < ntb; ++q)
        if ((tid >> q) & 1u) a ^= S.tmask[q];
    for (int b = 0; b < rr; ++b)
        if ((j >> b) & 1u) a ^= S.rbit[b];
    return a;
}

static int64_t gl_off(const int64_t* gt, const int64_t* gr, int ntb, int rr, uint32_t tid, uint32_t j) {
    int64_t o = 0;
    for (int q = 0; q < ntb; ++q)
        if ((tid >> q) & 1u) o ^= gt[q];
    for (int b = 0; b < rr; ++b)
        if ((j >> b) & 1u) o ^= gr[b];
    return o;
}

template <typename T>
static int check(int M, const std::vector<Coupling>& J, int k, int r, int c, int64_t steps, int observed,
                 bool plant, bool half, long* n_pass, long* n_cross, long* n_ex, long* n_tile) {
    PassParams pp;
    pp.k = k;
    pp.r = r;
    pp.c = c;
    pp.half = half;
    StreamPlan sp = plan_stream_best(M, J, 0.05, steps, observed, true, pp);
    int bad = 0;
    for (const HostPass& hp : sp.passes) {
        DevTables<T> tb;
        encode_pass<T>(hp, M, observed, tb);
        if (plant)
            for (DevStage& st : tb.stages) st.xnext = 0;
        const DevPass& P = tb.passes.back();
        const int ns = P.nstage;
        const int rr = int(hp.stages[0].regs.size());
        const int ntb = P.k - rr;
        const uint32_t nt = 1u << ntb, nr = 1u << rr, nwave = nt >= 64 ? nt / 64 : 1;
        const uint32_t lanes_per_wave = nt >= 64 ? 64 : nt;
        auto wave_set = [&](const DevStage& S, uint32_t w) {
            std::set<uint32_t> s;
            for (uint32_t t = w * lanes_per_wave; t < (w + 1) * lanes_per_wave; ++t)
                for (uint32_t j = 0; j < nr; ++j) s.insert(lds_addr(S, ntb, rr, t, j));
            return s;
        };
        ++*n_pass;
        bool any_cross = false;
        for (int si = 0; si < ns; ++si) {
            const DevStage& S = tb.stages[P.stage0 + si];
            const int kk = P.half ? P.k - 1 : P.k;
            const uint32_t nj = P.half ? nr / 2 : nr;
            if (bool(P.half) != half || (P.half && (ns > 1 && S.rbit[rr - 1] != 0))) {
                std::printf("half-tile pass without the split position on the top register bit\n");
                ++bad;
            }
            std::set<uint32_t> all;
            for (uint32_t t = 0; t < nt; ++t)
                for (uint32_t j = 0; j < nj; ++j) all.insert(lds_addr(S, ntb, rr, t, j));
            if (all.size() != (size_t(1) << kk) || *all.rbegin() >= (uint32_t(1) << kk) * sizeof(T) * 2) {
                std::printf("stage map is not a bijection onto the exchange buffer\n");
                ++bad;
            }
            if (si + 1 == ns) break;
            ++*n_ex;
            const DevStage& S2 = tb.stages[P.stage0 + si + 1];
            if (S.xnext) {
                any_cross = true;
                ++*n_cross;
                continue;
            }
            for (uint32_t w = 0; w < nwave; ++w)
                if (wave_set(S, w) != wave_set(S2, w)) {
                    std::printf("wave-local exchange moves amplitudes between waves\n");
                    ++bad;
                    break;
                }
        }
        // data flow of one tile: every amplitude loaded by the first stage
        // reaches the last stage's store of the same tile-local index
        // (input layout -> output layout), through every exchange
        {
            auto local_of = [&](int64_t off, const int32_t* tbit) {
                uint32_t x = 0;
                for (int p = 0; p < P.k; ++p)
                    if ((off >> tbit[p]) & 1) x |= 1u << p;
                return x;
            };
            const DevStage& S0 = tb.stages[P.stage0];
            std::vector<uint32_t> cur(size_t(nt) * nr);   // tile-local index held by (tid, j)
            for (uint32_t t = 0; t < nt; ++t)
                for (uint32_t j = 0; j < nr; ++j)
                    cur[size_t(t) * nr + j] = local_of(gl_off(S0.gt_in, S0.gr_in, ntb, rr, t, j), P.tbit);
            for (int si = 0; si + 1 < ns; ++si) {
                const DevStage& A = tb.stages[P.stage0 + si];
                const DevStage& B2 = tb.stages[P.stage0 + si + 1];
                std::vector<uint32_t> nxt(cur.size(), ~0u);
                const uint32_t halves = P.half ? 2 : 1, hn = nr / halves;
                for (uint32_t hv = 0; hv < halves; ++hv) {
                    std::vector<uint32_t> slot(size_t(1) << P.k, ~0u);
                    for (uint32_t t = 0; t < nt; ++t)
                        for (uint32_t j = hv * hn; j < (hv + 1) * hn; ++j)
                            slot[lds_addr(A, ntb, rr, t, j) / (sizeof(T) * 2)] = cur[size_t(t) * nr + j];
                    for (uint32_t t = 0; t < nt; ++t)
                        for (uint32_t j = hv * hn; j < (hv + 1) * hn; ++j)
                            nxt[size_t(t) * nr + j] = slot[lds_addr(B2, ntb, rr, t, j) / (sizeof(T) * 2)];
                }
                cur.swap(nxt);
            }
            const DevStage& SL = tb.stages[P.stage0 + ns - 1];
            bool ok = true;
            for (uint32_t t = 0; t < nt && ok; ++t)
                for (uint32_t j = 0; j < nr && ok; ++j)
                    ok = cur[size_t(t) * nr + j] == local_of(gl_off(SL.gt_out, SL.gr_out, ntb, rr, t, j), P.tbit_out);
            if (!ok) {
                std::printf("data flow: an amplitude is stored at another tile position\n");
                ++bad;
            }
        }
        if (ns > 1 && P.tile_barrier) ++*n_tile;
        if (ns > 1) {
            const DevStage& S0 = tb.stages[P.stage0];
            const DevStage& SL = tb.stages[P.stage0 + ns - 1];
            if (!P.tile_barrier)
                for (uint32_t w = 0; w < nwave; ++w)
                    if (wave_set(S0, w) != wave_set(SL, w)) {
                        std::printf("tile boundary without barrier: wave slots differ\n");
                        ++bad;
                        break;
                    }
            if (!any_cross)
                for (uint32_t w = 0; w < nwave; ++w) {
                    std::set<int64_t> ld, st;
                    for (uint32_t t = w * lanes_per_wave; t < (w + 1) * lanes_per_wave; ++t)
                        for (uint32_t j = 0; j < nr; ++j) {
                            ld.insert(gl_off(S0.gt_in, S0.gr_in, ntb, rr, t, j));
                            st.insert(gl_off(SL.gt_out, SL.gr_out, ntb, rr, t, j));
                        }
                    if (ld != st) {
                        std::printf("pass without barriers: a wave stores offsets it did not load\n");
                        ++bad;
                        break;
                    }
                }
        }
    }
    return bad;
}

int main() {
    int M, prec, k, r, c, observed;
    long long steps;
    int plant = 0, half = 0;
    if (std::scanf("%d %d %d %d %d %lld %d %d %d", &M, &prec, &k, &r, &c, &steps, &observed, &plant, &half) != 9)
        return 2;
    std::vector<Coupling> J;
    Coupling x;
    while (std::scanf("%d %d %lf %lf", &x.i, &x.j, &x.a, &x.b) == 4) J.push_back(x);
    long np = 0, ncross = 0, nex = 0, ntile = 0;
    const int bad = prec == 1
                        ? check<float>(M, J, k, r, c, steps, observed, plant != 0, half != 0, &np, &ncross, &nex, &ntile)
                        : check<double>(M, J, k, r, c, steps, observed, plant != 0, half != 0, &np, &ncross, &nex, &ntile);
    std::printf("templates %ld exchanges %ld cross-wave %ld tile-barriers %ld failures %d\n", np, nex, ncross,
                ntile, bad);
    return bad ? 1 : 0;
}
