// planner.cpp -- Strang op sequence, pass scheduling, stage scheduling and
// encoding of the device tables.  Host only.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <functional>
#include <map>
#include <sstream>
#include <stdexcept>

namespace spinqp {

// ------------------------------------------------------------------ sequence
SeqBuilder::SeqBuilder(int M, const std::vector<Coupling>& J, double dt, int observed, bool merge,
                       bool profile)
    : observed_(observed), merge_(merge), profile_(profile), dt_(dt), J_(J), last_(M, -1) {}

void SeqBuilder::emit_factor(const Coupling& c, double tau, int64_t step) {
    int i = std::min(c.i, c.j), j = std::max(c.i, c.j);
    int idx = idx_++;
    if (merge_) {
        int li = last_[i], lj = last_[j];
        // An op absorbs factors of its own step and of the next one only, so
        // the merged sequence repeats with a period of at most two steps.
        if (li >= 0 && li == lj && ops[li].kind == 0 && ops[li].i == i && ops[li].j == j &&
            ops[li].step >= step - 1) {
            ops[li].A += c.a * tau;
            ops[li].B += c.b * tau;
            return;
        }
    }
    ops.push_back(Op{0, i, j, c.a * tau, c.b * tau, step, idx});
    last_[i] = last_[j] = int(ops.size()) - 1;
}

void SeqBuilder::emit_observable(int64_t step) {
    if (step != cur_step_) { cur_step_ = step; idx_ = 0; }
    if (!profile_) {
        ops.push_back(Op{1, observed_, observed_, 0.0, 0.0, step, 1 << 30});
        last_[observed_] = int(ops.size()) - 1;
        return;
    }
    for (int s = 0; s < int(last_.size()); ++s) {
        ops.push_back(Op{1, s, s, 0.0, 0.0, step, (1 << 30) + s});
        last_[s] = int(ops.size()) - 1;
    }
}

void SeqBuilder::emit_step(int64_t step) {
    cur_step_ = step;
    idx_ = 0;
    const double tau = 0.5 * dt_;
    for (size_t g = 0; g < J_.size(); ++g) emit_factor(J_[g], tau, step);
    for (size_t g = J_.size(); g-- > 0;) emit_factor(J_[g], tau, step);
    emit_observable(step);
}

// ----------------------------------------------------------------- scheduler
namespace {

using Mask = uint64_t;
inline Mask bit(int s) { return Mask(1) << s; }
inline int popc(Mask m) { return __builtin_popcountll(m); }

struct Sched {
    int M, observed, k, max_meas;
    bool all_sites = false;    // observables on every site (profile)
    const std::vector<Op>& ops;
    std::vector<std::vector<int>> site_ops;
    std::vector<int> pos_i, pos_j;     // index of op in site_ops of its sites
    std::vector<int> head;
    std::vector<char> done;
    size_t first_pending = 0;
    // A pass may not run further ahead than `window` steps past the oldest
    // pending op; keeps passes bounded and the frontier comparable.
    int64_t window = 3;
    int64_t limit = INT64_MAX;

    int rotate = 0;    // start offset of the local search's site loops

    Sched(int M_, int obs, int k_, int mm, const std::vector<Op>& o)
        : M(M_), observed(obs), k(k_), max_meas(mm), ops(o), site_ops(M_),
          pos_i(o.size()), pos_j(o.size()), head(M_, 0), done(o.size(), 0) {
        for (size_t n = 0; n < ops.size(); ++n) {
            const Op& op = ops[n];
            pos_i[n] = int(site_ops[op.i].size());
            site_ops[op.i].push_back(int(n));
            if (op.j != op.i) {
                pos_j[n] = int(site_ops[op.j].size());
                site_ops[op.j].push_back(int(n));
            } else {
                pos_j[n] = pos_i[n];
            }
        }
    }

    void mark_done(int n) {
        done[n] = 1;
        head[ops[n].i] = std::max(head[ops[n].i], pos_i[n] + 1);
        head[ops[n].j] = std::max(head[ops[n].j], pos_j[n] + 1);
    }

    bool ready(int n, const std::vector<int>& h) const {
        const Op& op = ops[n];
        return h[op.i] == pos_i[n] && h[op.j] == pos_j[n];
    }
    bool eligible(int n, Mask T) const {
        const Op& op = ops[n];
        if (op.step > limit) return false;
        if (op.kind == 1) return true;
        return (T & bit(op.i)) && (T & bit(op.j));
    }

    // Number of ops (factors weigh 1, observables a little) a pass over tile
    // T can apply from the current frontier; optionally the applied list.
    double closure(Mask T, std::vector<int>* applied) const {
        std::vector<int> h = head;
        std::vector<int> work;
        int nmeas = 0, nnorm = 0;
        double score = 0;
        auto consider = [&](int s) {
            if (h[s] < int(site_ops[s].size())) {
                int n = site_ops[s][h[s]];
                if (eligible(n, T) && ready(n, h)) work.push_back(n);
            }
        };
        for (int s = 0; s < M; ++s)
            if ((T & bit(s)) || s == observed || all_sites) consider(s);
        while (!work.empty()) {
            int n = work.back();
            work.pop_back();
            if (!ready(n, h)) continue;
            const Op& op = ops[n];
            if (op.kind == 1) {
                if (nmeas >= max_meas) continue;
                // with every site observed, the observed site's op also
                // carries the step's norm: at most kMaxMeas norm slots
                if (all_sites && op.i == observed) {
                    if (nnorm >= kMaxMeas) continue;
                    ++nnorm;
                }
                ++nmeas;
                score += 1e-3;
            } else {
                score += 1.0;
            }
            if (applied) applied->push_back(n);
            h[op.i] = pos_i[n] + 1;
            h[op.j] = pos_j[n] + 1;
            consider(op.i);
            if (op.j != op.i) consider(op.j);
        }
        if (applied) std::sort(applied->begin(), applied->end());
        return score;
    }

    bool all_done() {
        while (first_pending < ops.size() && done[first_pending]) ++first_pending;
        return first_pending >= ops.size();
    }

    // Seed of the tile search grown breadth-first over the coupling graph
    // of the pending factors, from the sites of the earliest pending one:
    // a connected cluster, which the sequence-order seed misses when the
    // list runs along one part of the graph first (a ladder's legs).
    Mask cluster_seed(Mask forced) const {
        Mask T = forced;
        size_t n0 = first_pending;
        while (n0 < ops.size() && (done[n0] || ops[n0].kind == 1)) ++n0;
        if (n0 == ops.size()) return T;
        std::vector<int> queue{ops[n0].i, ops[n0].j};
        Mask seen = bit(ops[n0].i) | bit(ops[n0].j);
        for (size_t q = 0; q < queue.size() && popc(T) < k; ++q) {
            const int s = queue[q];
            if (popc(T | bit(s)) > k) break;
            T |= bit(s);
            for (int n : site_ops[s]) {
                const Op& op = ops[n];
                if (done[n] || op.kind == 1 || op.step > limit) continue;
                const int o = op.i == s ? op.j : op.i;
                if (!(seen & bit(o))) {
                    seen |= bit(o);
                    queue.push_back(o);
                }
            }
        }
        return T;
    }

    Mask choose_tile(Mask forced) {
        // Seeds: sites of the earliest pending ops in sequence order, and a
        // connected cluster around the earliest one; the local search runs
        // from each and the better result is kept.
        Mask T = forced;
        for (size_t n = first_pending; n < ops.size() && popc(T) < k; ++n) {
            if (done[n] || ops[n].kind == 1) continue;
            Mask add = bit(ops[n].i) | bit(ops[n].j);
            if (popc(T | add) <= k) T |= add;
            if (n - first_pending > 4096) break;
        }
        for (int s = 0; s < M && popc(T) < k; ++s) T |= bit(s);
        double best = 0;
        T = improve_tile(T, forced, &best);
        Mask C = cluster_seed(forced);
        for (int s = 0; s < M && popc(C) < k; ++s) C |= bit(s);
        if (C != T) {
            double v = 0;
            C = improve_tile(C, forced, &v);
            if (v > best + 1e-9) T = C;
        }
        return T;
    }

    // First-improvement local search over single-site swaps from T.
    Mask improve_tile(Mask T, Mask forced, double* score) const {
        double best = closure(T, nullptr);
        for (int round = 0; round < 64; ++round) {
            bool improved = false;
            for (int o2 = 0; o2 < M && !improved; ++o2) {
                const int out = (o2 + rotate) % M;
                if (!(T & bit(out)) || (forced & bit(out))) continue;
                for (int i2 = 0; i2 < M; ++i2) {
                    const int in = (i2 + rotate) % M;
                    if (T & bit(in)) continue;
                    Mask T2 = (T & ~bit(out)) | bit(in);
                    double v = closure(T2, nullptr);
                    if (v > best + 1e-9) {
                        best = v;
                        T = T2;
                        improved = true;
                        break;
                    }
                }
            }
            if (!improved) break;
        }
        *score = best;
        return T;
    }

    // The tile the next pass would take with no forced sites (lookahead).
    // next_pass reuses it when it holds the forced sites.
    Mask peeked = 0;
    Mask peek_tile() {
        peeked = 0;
        if (all_done()) return 0;
        limit = ops[first_pending].step + window;
        peeked = choose_tile(0);
        return peeked;
    }

    // Schedules one pass; returns the applied op indices (sorted) and T.
    std::vector<int> next_pass(Mask forced, Mask* Tout) {
        all_done();
        limit = ops[first_pending].step + window;
        Mask T = peeked && !(forced & ~peeked) ? peeked : choose_tile(forced);
        peeked = 0;
        std::vector<int> applied;
        closure(T, &applied);
        if (applied.empty()) throw std::runtime_error("planner: no progress");
        for (int n : applied) mark_done(n);
        *Tout = T;
        return applied;
    }

    // Frontier signature relative to the lowest pending step.
    bool signature(std::vector<int64_t>* sig, int64_t* base) const {
        int64_t b = INT64_MAX;
        for (int s = 0; s < M; ++s)
            if (head[s] < int(site_ops[s].size())) b = std::min(b, ops[site_ops[s][head[s]]].step);
        if (b == INT64_MAX) return false;
        sig->assign(2 * M, -1);
        for (int s = 0; s < M; ++s) {
            if (head[s] < int(site_ops[s].size())) {
                const Op& op = ops[site_ops[s][head[s]]];
                (*sig)[2 * s] = op.step - b;
                (*sig)[2 * s + 1] = op.idx;
            }
        }
        *base = b;
        return true;
    }
};

HostPass make_pass(const std::vector<Op>& ops, const std::vector<int>& applied, Mask T, int M) {
    HostPass hp;
    for (int s = 0; s < M; ++s)
        if (T & bit(s)) hp.sites.push_back(s);
    hp.bit_in = hp.sites;        // canonical layout: site s is bit s
    hp.bit_out = hp.sites;
    hp.layout.resize(M);
    for (int s = 0; s < M; ++s) hp.layout[s] = s;
    bool any_factor = false;
    for (int n : applied) {
        hp.ops.push_back(ops[n]);
        any_factor |= ops[n].kind == 0;
    }
    hp.writes = any_factor;
    return hp;
}

// Site -> address-bit layout carried from pass to pass.  Every tile keeps
// the c lowest address bits (contiguous runs of 2^c amplitudes); which
// sites sit there changes: each pass stores its tile with the sites the
// next pass will use placed on the low bits (a permutation of the tile's own
// bits, so the store covers the same addresses it loaded).
struct Relabel {
    int M, c;
    std::vector<int> pi;       // site -> bit
    Relabel(int M_, int c_) : M(M_), c(c_), pi(M_) {
        for (int s = 0; s < M; ++s) pi[s] = s;
    }
    Mask low_sites() const {
        Mask m = 0;
        for (int s = 0; s < M; ++s)
            if (pi[s] < c) m |= bit(s);
        return m;
    }
    bool identity() const {
        for (int s = 0; s < M; ++s)
            if (pi[s] != s) return false;
        return true;
    }
    // Fills the layout fields of hp for tile T (hp.sites set in site order),
    // choosing the next low-bit sites from T_next, preferably outside
    // `avoid` (the registers of the pass's last stage, which could not be
    // stored straight to the low bits), and advances pi.
    void apply(HostPass& hp, Mask T, Mask T_next, Mask avoid, Mask avoid_soft = 0) {
        std::vector<int> sites;
        for (int s = 0; s < M; ++s)
            if (T & bit(s)) sites.push_back(s);
        std::sort(sites.begin(), sites.end(), [&](int a, int b) { return pi[a] < pi[b]; });
        hp.sites = sites;
        hp.layout = pi;
        hp.bit_in.clear();
        for (int s : sites) hp.bit_in.push_back(pi[s]);
        // next low-bit sites: in T and in the next tile; keep current ones first
        const Mask old_low = low_sites();
        std::vector<int> cand_keep, cand_new, cand_soft, cand_avoid, fill;
        for (int s = 0; s < M; ++s) {
            if (!(T & bit(s))) continue;
            const bool nxt = T_next & bit(s), low = old_low & bit(s);
            if (nxt && (avoid & bit(s))) cand_avoid.push_back(s);
            else if (nxt && (avoid_soft & bit(s))) cand_soft.push_back(s);
            else if (nxt && low) cand_keep.push_back(s);
            else if (nxt) cand_new.push_back(s);
            else fill.push_back(s);
        }
        std::vector<int> lows = cand_keep;
        for (int s : cand_new) lows.push_back(s);
        for (int s : cand_soft) lows.push_back(s);
        for (int s : cand_avoid) lows.push_back(s);
        // too few shared sites: keep current low sites, then any tile site
        std::vector<int> rest;
        for (int s : fill)
            if (old_low & bit(s)) rest.push_back(s);
        for (int s : fill)
            if (!(old_low & bit(s))) rest.push_back(s);
        for (int s : rest) lows.push_back(s);
        lows.resize(std::min<size_t>(lows.size(), size_t(c)));
        // New layout of the tile's bits B: sites staying on the low bits keep
        // them, entering sites take the freed low bits (both in site order);
        // every other site returns to its own bit when that bit is in B and
        // free, the rest fill the remaining bits of B in order.  Pulling
        // sites home keeps the layout a function of the recent passes, so a
        // repeating schedule also repeats its layouts.
        Mask new_low = 0;
        for (int s : lows) new_low |= bit(s);
        Mask B = 0;
        for (int s : sites) B |= bit(pi[s]);
        Mask used = 0;
        std::vector<int> npi(pi);
        std::vector<int> entering;
        for (int s : sites) {
            if (!(new_low & bit(s))) continue;
            if (pi[s] < c) used |= bit(pi[s]);
            else entering.push_back(s);
        }
        int lb = 0;
        for (int s : entering) {
            while (used & bit(lb)) ++lb;
            npi[s] = lb;
            used |= bit(lb);
        }
        std::vector<int> homeless;
        for (int s : sites) {
            if (new_low & bit(s)) continue;
            if (s >= c && (B & bit(s)) && !(used & bit(s))) {
                npi[s] = s;
                used |= bit(s);
            } else {
                homeless.push_back(s);
            }
        }
        int hb = 0;
        for (int s : homeless) {
            while (hb < M && (!(B & bit(hb)) || (used & bit(hb)) || hb < c)) ++hb;
            if (hb == M) throw std::runtime_error("planner: relabel out of bits");
            npi[s] = hb;
            used |= bit(hb);
        }
        pi = npi;
        hp.bit_out.clear();
        for (int s : sites) hp.bit_out.push_back(pi[s]);
    }
    // Layout fields of a pass that keeps the layout (a read-only pass).
    void keep(HostPass& hp, Mask T) const {
        std::vector<int> sites;
        for (int s = 0; s < M; ++s)
            if (T & bit(s)) sites.push_back(s);
        std::sort(sites.begin(), sites.end(), [&](int a, int b) { return pi[a] < pi[b]; });
        hp.sites = sites;
        hp.layout = pi;
        hp.bit_in.clear();
        for (int s : sites) hp.bit_in.push_back(pi[s]);
        hp.bit_out = hp.bit_in;
    }
    // Permutation-only passes (no ops) that bring pi back to the identity.
    std::vector<HostPass> restore(int k) {
        std::vector<HostPass> out;
        for (int guard = 0; !identity() && guard < 4 * M; ++guard) {
            std::vector<int> pinv(M);
            for (int s = 0; s < M; ++s) pinv[pi[s]] = s;
            Mask T = low_sites();
            for (int s = 0; s < M && popc(T) < k; ++s) {
                if (pi[s] == s) continue;
                const Mask need = bit(s) | bit(pinv[s]);
                if (popc(T | need) <= k) T |= need;
            }
            for (int s = 0; s < M && popc(T) < k; ++s) T |= bit(s);
            HostPass hp;
            std::vector<int> sites;
            for (int s = 0; s < M; ++s)
                if (T & bit(s)) sites.push_back(s);
            std::sort(sites.begin(), sites.end(), [&](int a, int b) { return pi[a] < pi[b]; });
            hp.sites = sites;
            hp.layout = pi;
            for (int s : sites) hp.bit_in.push_back(pi[s]);
            // sites whose home bit is in the tile go home; the rest take the
            // remaining bits in order
            Mask B = 0;
            for (int s : sites) B |= bit(pi[s]);
            std::vector<int> homeless, freebits;
            Mask taken = 0;
            for (int s : sites)
                if (B & bit(s)) taken |= bit(s);
            for (int s : sites)
                if (!(B & bit(s))) homeless.push_back(s);
            for (int s : sites)
                if (!(taken & bit(pi[s]))) freebits.push_back(pi[s]);
            std::sort(freebits.begin(), freebits.end());
            for (int s : sites)
                if (B & bit(s)) pi[s] = s;
            for (size_t n = 0; n < homeless.size(); ++n) pi[homeless[n]] = freebits[n];
            for (int s : sites) hp.bit_out.push_back(pi[s]);
            hp.writes = true;
            out.push_back(std::move(hp));
        }
        if (!identity()) throw std::runtime_error("planner: layout not restored");
        return out;
    }
};

std::vector<Op> gen_sequence(int M, const std::vector<Coupling>& J, double dt, int observed,
                             bool merge, int64_t s_begin, int64_t s_end, bool initial_obs,
                             bool profile) {
    SeqBuilder sb(M, J, dt, observed, merge, profile);
    if (initial_obs) sb.emit_observable(0);
    for (int64_t s = s_begin; s <= s_end; ++s) sb.emit_step(s);
    return sb.ops;
}

}  // namespace

// ----------------------------------------------------------------- stages
void plan_stages_coalesced(HostPass& pass, int r, int c, int beam, bool half) {
    uint32_t af = 0, al = 0;
    const int k = int(pass.sites.size());
    for (int p = 0; p < k; ++p) {
        if (pass.bit_in[p] < c) af |= 1u << p;
        if (pass.bit_out[p] < c) al |= 1u << p;
    }
    pass.split = -1;
    if (!half || k < 2 || r < 2) {
        plan_stages(pass, r, af, al, beam);
        return;
    }
    // split position: the one whose greedy staging is shortest (ties: the
    // position with the most factors), staged again with the requested beam
    std::vector<int> nops(k, 0), local(kMaxSites, -1);
    for (int p = 0; p < k; ++p) local[pass.sites[p]] = p;
    for (const Op& op : pass.ops)
        if (op.kind == 0) {
            ++nops[local[op.i]];
            ++nops[local[op.j]];
        }
    int best = -1;
    size_t best_n = 0;
    for (int h = 0; h < k; ++h) {
        if (((af | al) >> h) & 1u) continue;
        HostPass t = pass;
        try {
            plan_stages(t, r, af, al, 1, 1u << h);
        } catch (const std::runtime_error&) {
            continue;
        }
        if (best < 0 || t.stages.size() < best_n ||
            (t.stages.size() == best_n && nops[h] > nops[best])) {
            best = h;
            best_n = t.stages.size();
        }
    }
    if (best < 0) throw std::runtime_error("planner: no split position for a half-tile pass");
    plan_stages(pass, r, af, al, beam, 1u << best);
    pass.split = best;
    // the split position on the top register bit of every stage
    for (HostStage& st : pass.stages) {
        std::vector<int> regs;
        for (int q : st.regs)
            if (q != best) regs.push_back(q);
        if (int(regs.size()) + 1 != int(st.regs.size())) throw std::runtime_error("planner: split position lost");
        regs.push_back(best);
        st.regs = regs;
    }
}

void plan_stages(HostPass& pass, int r, uint32_t avoid_first, uint32_t avoid_last, int beam,
                 uint32_t force) {
    const int k = int(pass.sites.size());
    const int nops = int(pass.ops.size());
    std::vector<int> local(kMaxSites, -1);
    for (int p = 0; p < k; ++p) local[pass.sites[p]] = p;
    // per local position queue of op indices
    std::vector<std::vector<int>> q(k + 1);
    std::vector<int> pi(nops), pj(nops), li(nops), lj(nops);
    const int OBS = k;   // observables queue on a virtual position
    for (int n = 0; n < nops; ++n) {
        const Op& op = pass.ops[n];
        if (op.kind == 1) {
            int p = local[op.i] >= 0 ? local[op.i] : OBS;
            li[n] = lj[n] = p;
        } else {
            li[n] = local[op.i];
            lj[n] = local[op.j];
            if (li[n] < 0 || lj[n] < 0) throw std::runtime_error("planner: op outside tile");
        }
        pi[n] = int(q[li[n]].size());
        q[li[n]].push_back(n);
        if (lj[n] != li[n]) {
            pj[n] = int(q[lj[n]].size());
            q[lj[n]].push_back(n);
        } else {
            pj[n] = pi[n];
        }
    }
    auto ready = [&](int n, const std::vector<int>& h) {
        return h[li[n]] == pi[n] && h[lj[n]] == pj[n];
    };
    struct State {
        std::vector<int> head;
        std::vector<char> done;
        int ndone = 0;
        std::vector<HostStage> stages;
    };
    struct Cand {
        uint32_t S;
        std::vector<int> ops;
        int cnt;
    };
    // Register sets for the next stage: greedy growth from a few ready ops,
    // best first.  The first stage's registers may not take the avoided
    // positions.
    auto candidates = [&](const State& st, int nseeds) {
        std::vector<int> seeds;
        for (int n = 0; n < nops && int(seeds.size()) < nseeds; ++n)
            if (!st.done[n] && ready(n, st.head) && pass.ops[n].kind == 0) seeds.push_back(n);
        if (seeds.empty()) seeds.push_back(-1);
        const uint32_t avoid = st.stages.empty() ? avoid_first : 0u;
        std::vector<Cand> out;
        for (int seed : seeds) {
            std::vector<int> h = st.head;
            uint32_t S = force;
            if (seed >= 0) S = force | (1u << li[seed]) | (1u << lj[seed]);
            if ((S & avoid) || __builtin_popcount(S) > r) S = force;
            std::vector<int> got;
            std::vector<char> taken(nops, 0);
            int cnt = 0;
            bool changed = true;
            while (changed) {
                changed = false;
                for (int n = 0; n < nops; ++n) {
                    if (st.done[n] || taken[n] || !ready(n, h)) continue;
                    const Op& op = pass.ops[n];
                    if (op.kind == 0) {
                        uint32_t need = (1u << li[n]) | (1u << lj[n]);
                        if (need & avoid) continue;
                        if (__builtin_popcount(S | need) > r) continue;
                        S |= need;
                        ++cnt;
                    }
                    taken[n] = 1;
                    got.push_back(n);
                    h[li[n]] = pi[n] + 1;
                    h[lj[n]] = pj[n] + 1;
                    changed = true;
                }
            }
            bool dup = false;
            for (const Cand& c : out) dup |= c.S == S && c.cnt == cnt;
            if (!dup) out.push_back(Cand{S, got, cnt});
        }
        std::stable_sort(out.begin(), out.end(), [](const Cand& a, const Cand& b) { return a.cnt > b.cnt; });
        return out;
    };
    auto advance = [&](const State& st, const Cand& c) {
        State nx = st;
        uint32_t S = c.S | force;
        const uint32_t avoid = st.stages.empty() ? avoid_first : 0u;
        // Fill the register set up to r positions, highest positions first
        // (keeps the lanes on low positions), never the avoided ones and
        // preferably not the last stage's.
        for (int pass2 = 0; pass2 < 2; ++pass2)
            for (int p = k - 1; p >= 0 && __builtin_popcount(S) < std::min(r, k); --p) {
                if ((avoid >> p) & 1u) continue;
                if (pass2 == 0 && ((avoid_last >> p) & 1u)) continue;
                S |= 1u << p;
            }
        HostStage hs;
        for (int p = 0; p < k; ++p)
            if (S & (1u << p)) hs.regs.push_back(p);
        std::vector<int> ops = c.ops;
        std::sort(ops.begin(), ops.end());
        for (int n : ops) {
            nx.done[n] = 1;
            ++nx.ndone;
            nx.head[li[n]] = std::max(nx.head[li[n]], pi[n] + 1);
            nx.head[lj[n]] = std::max(nx.head[lj[n]], pj[n] + 1);
        }
        hs.ops = ops;
        nx.stages.push_back(std::move(hs));
        return nx;
    };
    // A finished stage list still needs an extra stage when its last stage
    // holds an output low-bit position (or is a lone stage that moves data).
    auto penalty = [&](const State& st) {
        uint32_t m = 0;
        for (int p : st.stages.back().regs) m |= 1u << p;
        if (st.stages.size() == 1) return (m & (avoid_first | avoid_last)) != 0 || pass.bit_in != pass.bit_out;
        return (m & avoid_last) != 0;
    };
    // Beam search over stage sequences (width 1: the greedy choice); a
    // level adds one stage to every kept sequence.
    State init;
    init.head.assign(k + 1, 0);
    init.done.assign(nops, 0);
    std::vector<State> level{init};
    State best;
    bool have = false;
    const int width = std::max(1, beam);
    const int nseeds = width > 1 ? 12 : 6;
    const int per_state = width > 1 ? 3 : 1;
    while (!have) {
        if (level.front().ndone == nops) {   // no ops at all
            best = level.front();
            break;
        }
        std::vector<State> next;
        for (const State& st : level) {
            auto cs = candidates(st, nseeds);
            if (cs.front().ops.empty() && !st.stages.empty())
                throw std::runtime_error("planner: stage made no progress");
            for (int i = 0; i < int(cs.size()) && i < per_state; ++i) next.push_back(advance(st, cs[i]));
        }
        std::stable_sort(next.begin(), next.end(),
                         [](const State& a, const State& b) { return a.ndone > b.ndone; });
        std::vector<State> kept;
        for (State& st : next) {
            bool dup = false;
            for (const State& o : kept) dup |= o.done == st.done;
            if (!dup) kept.push_back(std::move(st));
            if (int(kept.size()) == width) break;
        }
        for (const State& st : kept)
            if (st.ndone == nops && (!have || (penalty(best) && !penalty(st)))) {
                best = st;
                have = true;
            }
        level = std::move(kept);
    }
    pass.stages = std::move(best.stages);
    // a pass always has a stage; the last one must be storable directly
    // A single stage stores from the registers it loaded with no workgroup
    // barrier in between, so each lane must store exactly the addresses it
    // loaded (another wave's loads of the tile may still be in flight): only
    // a pass that keeps its layout can have one stage.
    auto bad_last = [&]() {
        if (pass.stages.empty()) return true;
        uint32_t m = 0;
        for (int p : pass.stages.back().regs) m |= 1u << p;
        if (pass.stages.size() == 1)
            return (m & (avoid_first | avoid_last)) != 0 || pass.bit_in != pass.bit_out;
        return (m & avoid_last) != 0;
    };
    for (int extra = 0; bad_last(); ++extra) {
        if (extra == 2) throw std::runtime_error("planner: cannot place the last stage");
        HostStage st;
        const uint32_t av = pass.stages.empty() ? avoid_first : avoid_last;
        if (force & av) throw std::runtime_error("planner: forced position on a low bit");
        for (int p = 0; p < k; ++p)
            if ((force >> p) & 1u) st.regs.push_back(p);
        for (int p = k - 1; p >= 0 && int(st.regs.size()) < std::min(r, k); --p)
            if (!((av >> p) & 1u) && !((force >> p) & 1u)) st.regs.push_back(p);
        std::sort(st.regs.begin(), st.regs.end());
        if (int(st.regs.size()) < std::min(r, k)) throw std::runtime_error("planner: tile too small");
        pass.stages.push_back(std::move(st));
    }
}

// ----------------------------------------------------------- stream plan
// Fallback: every step planned alone (no merging across the step boundary),
// so one step's passes repeat verbatim.
static StreamPlan plan_stream_per_step(int M, const std::vector<Coupling>& J, double dt,
                                       int64_t n_steps, int observed, bool merge,
                                       const PassParams& pp) {
    StreamPlan plan;
    plan.n_steps = n_steps;
    const int k = std::min(pp.k, M);
    Mask forced = 0;
    for (int s = 0; s < std::min(pp.c, k); ++s) forced |= bit(s);
    // read-only passes for the step-0 observables (one per site with the
    // profile, at most max_meas per pass)
    SeqBuilder sb0(M, J, dt, observed, merge, pp.profile);
    sb0.emit_observable(0);
    int nobs0 = 0;
    for (size_t o = 0; o < sb0.ops.size(); o += size_t(pp.max_meas)) {
        HostPass obs;
        for (int s = 0; s < k; ++s) obs.sites.push_back(s);
        obs.bit_in = obs.sites;
        obs.bit_out = obs.sites;
        obs.layout.resize(M);
        for (int s = 0; s < M; ++s) obs.layout[s] = s;
        for (size_t q = o; q < std::min(sb0.ops.size(), o + size_t(pp.max_meas)); ++q)
            obs.ops.push_back(sb0.ops[q]);
        obs.writes = false;
        plan.passes.push_back(obs);
        ++nobs0;
    }
    SeqBuilder sb(M, J, dt, observed, merge, pp.profile);
    sb.emit_step(1);
    Sched sc(M, observed, k, pp.max_meas, sb.ops);
    sc.all_sites = pp.profile;
    sc.window = pp.window;
    sc.rotate = pp.rotate;
    while (!sc.all_done()) {
        Mask T;
        auto ap = sc.next_pass(forced, &T);
        plan.passes.push_back(make_pass(sb.ops, ap, T, M));
    }
    for (auto& p : plan.passes) plan_stages_coalesced(p, std::min(pp.r, int(p.sites.size())), pp.c, 1, pp.half);
    for (int t = 0; t < nobs0; ++t) {
        plan.launch_tmpl.push_back(t);
        plan.launch_offset.push_back(0);
    }
    for (int64_t st = 0; st < n_steps; ++st)
        for (size_t t = size_t(nobs0); t < plan.passes.size(); ++t) {
            plan.launch_tmpl.push_back(int(t));
            plan.launch_offset.push_back(st);
        }
    plan.period_steps = 1;
    plan.period_passes = int(plan.passes.size()) - nobs0;
    return plan;
}

namespace {

// One pass: the tile must hold the sites now on the low bits; a writing pass
// hands the low bits to sites of the tile the scheduler would take next.
HostPass schedule_one(Sched& sc, Relabel& rl, const std::vector<Op>& ops, int M,
                      const PassParams& pp) {
    Mask T;
    auto ap = sc.next_pass(rl.low_sites(), &T);
    HostPass hp = make_pass(ops, ap, T, M);
    if (!hp.writes) {
        rl.keep(hp, T);
        return hp;
    }
    // stages with the input layout tell which sites the last stage holds in
    // registers; the low output bits go preferably to other sites
    HostPass tmp = hp;
    rl.keep(tmp, T);
    uint32_t af = 0;
    for (size_t p = 0; p < tmp.sites.size(); ++p)
        if (tmp.bit_in[p] < rl.c) af |= 1u << p;
    Mask last_regs = 0;
    try {
        if (pp.low_policy >= 1) plan_stages(tmp, std::min(pp.r, int(tmp.sites.size())), af, 0);
        if (pp.low_policy >= 1)
            for (int q : tmp.stages.back().regs) last_regs |= bit(tmp.sites[q]);
    } catch (const std::runtime_error&) {
        last_regs = 0;
    }
    // the first stage of the next pass cannot hold low-bit sites in
    // registers: avoid, if possible, the sites it would start with
    const Mask T_next = sc.peek_tile();
    Mask next_first = 0;
    if (T_next && pp.low_policy >= 2) {
        std::vector<int> nap;
        sc.closure(T_next, &nap);
        HostPass nx = make_pass(ops, nap, T_next, M);
        rl.keep(nx, T_next);
        try {
            plan_stages(nx, std::min(pp.r, int(nx.sites.size())), 0, 0);
            for (int q : nx.stages.front().regs) next_first |= bit(nx.sites[q]);
        } catch (const std::runtime_error&) {
            next_first = 0;
        }
    }
    rl.apply(hp, T, T_next, last_regs, next_first);
    return hp;
}

// Sites away from their own address bit.
Mask displaced(const Relabel& rl) {
    Mask d = 0;
    for (int s = 0; s < rl.M; ++s)
        if (rl.pi[s] != s) d |= bit(s);
    return d;
}

// The last pass of a run, when one pass can be it: a tile holding the
// low-bit sites and every site away from its own bit whose closure is every
// remaining op, stored with every site on its own bit.  A displaced site's
// current bit is the own bit of another displaced site, so such a tile's
// bits are exactly its sites' own bits and the store stays inside the
// tile's addresses.  This saves the permutation-only pass that would
// otherwise restore the layout.  Returns false, changing nothing, when no
// such tile is found.
bool try_finish(Sched& sc, Relabel& rl, const std::vector<Op>& ops, int M, HostPass* out) {
    constexpr size_t kFinishOps = 256;   // only near the end of a run
    if (sc.all_done()) return false;
    size_t remaining = 0;
    for (size_t n = sc.first_pending; n < ops.size() && remaining <= kFinishOps; ++n)
        remaining += !sc.done[n];
    if (remaining > kFinishOps) return false;
    const Mask D = displaced(rl);
    const Mask forced = rl.low_sites() | D;
    if (popc(forced) > sc.k) return false;
    const int64_t lim = sc.limit;
    sc.limit = INT64_MAX;
    const Mask T = sc.choose_tile(forced);
    std::vector<int> applied;
    sc.closure(T, &applied);
    sc.limit = lim;
    if (applied.size() != remaining) return false;
    for (int n : applied) sc.mark_done(n);
    HostPass hp = make_pass(ops, applied, T, M);
    rl.keep(hp, T);
    hp.bit_out = hp.sites;           // every site on its own bit
    hp.writes = hp.writes || D != 0;
    for (int s = 0; s < M; ++s) rl.pi[s] = s;
    *out = std::move(hp);
    return true;
}

// Schedules the remaining ops of `sc` and leaves the canonical layout.
void schedule_to_end(Sched& sc, Relabel& rl, const std::vector<Op>& ops, int M, const PassParams& pp,
                     int k, std::vector<HostPass>& out) {
    while (!sc.all_done()) {
        HostPass fin;
        if (try_finish(sc, rl, ops, M, &fin)) {
            out.push_back(std::move(fin));
            break;
        }
        out.push_back(schedule_one(sc, rl, ops, M, pp));
    }
    for (HostPass& hp : rl.restore(k)) out.push_back(std::move(hp));
}

// Templates [t0, t0 + n) launched in order with observable labels shifted
// by `offset`.
void add_launches(StreamPlan& plan, int t0, int n, int64_t offset) {
    for (int t = t0; t < t0 + n; ++t) {
        plan.launch_tmpl.push_back(t);
        plan.launch_offset.push_back(offset);
    }
}

// Appends passes as templates; returns the index of the first.
int add_templates(StreamPlan& plan, std::vector<HostPass>&& passes) {
    const int t0 = int(plan.passes.size());
    for (HostPass& hp : passes) plan.passes.push_back(std::move(hp));
    return t0;
}

// Self-contained block: steps 1..n (and the step-0 observable if asked),
// from the canonical layout back to it.
std::vector<HostPass> plan_block(int M, const std::vector<Coupling>& J, double dt, int observed,
                                 bool merge, const PassParams& pp, int64_t n, bool initial_obs) {
    const int k = std::min(pp.k, M), c = std::min(pp.c, k);
    std::vector<Op> ops = gen_sequence(M, J, dt, observed, merge, 1, n, initial_obs, pp.profile);
    Sched sc(M, observed, k, pp.max_meas, ops);
    sc.all_sites = pp.profile;
    sc.window = pp.window;
    sc.rotate = pp.rotate;
    Relabel rl(M, c);
    std::vector<HostPass> out;
    schedule_to_end(sc, rl, ops, M, pp, k, out);
    return out;
}

void finish_stages(StreamPlan& plan, const PassParams& pp) {
    for (auto& p : plan.passes)
        plan_stages_coalesced(p, std::min(pp.r, int(p.sites.size())), pp.c, 1, pp.half);
}

// Blocks of `W` steps repeated verbatim: the first carries the step-0
// observable, the last the remainder.  Each block drains the pipeline and
// restores the layout, which costs a few passes per block.
StreamPlan plan_stream_blocks(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                              int observed, bool merge, const PassParams& pp, int64_t W) {
    StreamPlan plan;
    plan.n_steps = n_steps;
    const int64_t first = std::min(W, n_steps);
    auto b0 = plan_block(M, J, dt, observed, merge, pp, first, true);
    const int nb0 = int(b0.size());
    add_launches(plan, add_templates(plan, std::move(b0)), nb0, 0);
    const int64_t reps = n_steps / W, rem = n_steps - std::max<int64_t>(reps, 1) * W;
    if (reps > 1) {
        auto mid = plan_block(M, J, dt, observed, merge, pp, W, false);
        const int nm = int(mid.size());
        const int t0 = add_templates(plan, std::move(mid));
        for (int64_t r = 1; r < reps; ++r) add_launches(plan, t0, nm, r * W);
        plan.period_steps = int(W);
        plan.period_passes = nm;
    }
    if (rem > 0) {
        auto last = plan_block(M, J, dt, observed, merge, pp, rem, false);
        const int nl = int(last.size());
        add_launches(plan, add_templates(plan, std::move(last)), nl, std::max<int64_t>(reps, 1) * W);
    }
    finish_stages(plan, pp);
    return plan;
}

// Pipelined long run: schedule kGen steps continuously and look for a
// repeating state (frontier and layout); the passes between two
// occurrences are a period template repeated to the end, then a tail.
StreamPlan plan_stream_periodic(int M, const std::vector<Coupling>& J, double dt,
                                int64_t n_steps, int observed, bool merge,
                                const PassParams& pp, int64_t kGen) {
    StreamPlan plan;
    plan.n_steps = n_steps;
    const int k = std::min(pp.k, M);
    const int c = std::min(pp.c, k);
    const int64_t kSafe = 8;     // steps kept between the frontier and the end
    std::vector<Op> ops = gen_sequence(M, J, dt, observed, merge, 1, kGen, true, pp.profile);
    Sched sc(M, observed, k, pp.max_meas, ops);
    sc.all_sites = pp.profile;
    sc.window = pp.window;
    sc.rotate = pp.rotate;
    Relabel rl(M, c);
    std::map<std::vector<int64_t>, std::pair<int, int64_t>> seen;
    std::vector<HostPass> passes;
    int p1 = -1, p2 = -1;
    int64_t s1 = 0, s2 = 0;
    std::vector<int64_t> sig;
    int64_t base = 0;
    while (!sc.all_done()) {
        if (sc.signature(&sig, &base)) {
            if (base > kGen - kSafe) break;
            sig.insert(sig.end(), rl.pi.begin(), rl.pi.end());   // the layout is state too
            auto it = seen.find(sig);
            // the merged sequence has period two: only even shifts are exact
            if (it != seen.end() && base > it->second.second &&
                (base - it->second.second) % 2 == 0) {
                p1 = it->second.first;
                s1 = it->second.second;
                p2 = int(passes.size());
                s2 = base;
                break;
            }
            if (it == seen.end()) seen[sig] = {int(passes.size()), base};
        }
        passes.push_back(schedule_one(sc, rl, ops, M, pp));
    }
    if (p1 < 0) throw std::runtime_error("planner: no periodic schedule found");
    const int64_t delta = s2 - s1;
    int64_t max_rel = 0;   // largest step touched by the period at shift 0
    for (int p = p1; p < p2; ++p)
        for (const Op& op : passes[p].ops) max_rel = std::max(max_rel, op.step);
    // the prefix must also stay clear of the last two steps
    int64_t max_pre = 0;
    for (int p = 0; p < p1; ++p)
        for (const Op& op : passes[p].ops) max_pre = std::max(max_pre, op.step);
    if (max_pre > n_steps - 2 || max_rel > n_steps - 2)
        throw std::runtime_error("planner: run too short for the periodic plan");
    const int64_t reps = (n_steps - 2 - max_rel) / delta + 1;

    plan.passes.assign(passes.begin(), passes.begin() + p2);
    for (int p = 0; p < p1; ++p) {
        plan.launch_tmpl.push_back(p);
        plan.launch_offset.push_back(0);
    }
    for (int64_t r = 0; r < reps; ++r)
        for (int p = p1; p < p2; ++p) {
            plan.launch_tmpl.push_back(p);
            plan.launch_offset.push_back(r * delta);
        }
    plan.period_steps = int(delta);
    plan.period_passes = p2 - p1;

    // Tail: the frontier after `reps` periods is the signature at p1
    // shifted by reps*delta.  Regenerate the real sequence from there on.
    std::vector<int64_t> sig1;
    {
        // recompute the signature at p1 by replaying: it is the key stored
        for (auto& kv : seen)
            if (kv.second.first == p1) { sig1 = kv.first; break; }
    }
    const int64_t base_t = s1 + reps * delta;
    // regenerate from an odd step so merged ops keep their identities
    int64_t gen_from = std::max<int64_t>(1, base_t - 2);
    if (gen_from % 2 == 0) --gen_from;
    std::vector<Op> tops = gen_sequence(M, J, dt, observed, merge, gen_from, n_steps, false, pp.profile);
    Sched tc(M, observed, k, pp.max_meas, tops);
    tc.all_sites = pp.profile;
    tc.window = pp.window;
    tc.rotate = pp.rotate;
    Relabel tl(M, c);
    tl.pi.assign(sig1.begin() + 2 * M, sig1.end());
    for (size_t n = 0; n < tops.size(); ++n) {
        const Op& op = tops[n];
        auto before = [&](int s) {
            if (sig1[2 * s] < 0) return true;    // site had nothing pending: all done
            int64_t hs = sig1[2 * s] + base_t;
            int64_t hi = sig1[2 * s + 1];
            return op.step < hs || (op.step == hs && op.idx < hi);
        };
        bool d1 = before(op.i), d2 = before(op.j);
        if (d1 != d2) throw std::runtime_error("planner: inconsistent tail frontier");
        if (d1) tc.mark_done(int(n));
    }
    std::vector<HostPass> tail;
    schedule_to_end(tc, tl, tops, M, pp, k, tail);
    const int nt = int(tail.size());
    add_launches(plan, add_templates(plan, std::move(tail)), nt, 0);
    finish_stages(plan, pp);
    return plan;
}

}  // namespace

StreamPlan plan_stream(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                       int observed, bool merge, const PassParams& pp) {
    if (M > 63) throw std::runtime_error("planner: M too large");
    const int64_t kGen = 48;     // steps scheduled when searching for a period
    if (n_steps <= 2 * kGen)
        return plan_stream_blocks(M, J, dt, n_steps, observed, merge, pp, std::max<int64_t>(n_steps, 1));
    StreamPlan best;
    bool have = false;
    try {
        best = plan_stream_periodic(M, J, dt, n_steps, observed, merge, pp, kGen);
        have = true;
    } catch (const std::runtime_error&) {
    }
    try {
        StreamPlan blocks = plan_stream_blocks(M, J, dt, n_steps, observed, merge, pp, kGen);
        if (!have || blocks.launch_tmpl.size() < best.launch_tmpl.size()) best = std::move(blocks);
        have = true;
    } catch (const std::runtime_error&) {
    }
    if (have) return best;
    return plan_stream_per_step(M, J, dt, n_steps, observed, merge, pp);
}

double plan_cost(const StreamPlan& plan, const PlanCostModel& cm) {
    std::vector<double> tcost(plan.passes.size());
    for (size_t t = 0; t < plan.passes.size(); ++t) {
        const HostPass& hp = plan.passes[t];
        int nf = 0;
        for (const Op& op : hp.ops) nf += op.kind == 0;
        tcost[t] = cm.pass + cm.stage * double(hp.stages.size()) + cm.op * nf;
    }
    double c = 0;
    for (int t : plan.launch_tmpl) c += tcost[t];
    return c;
}

StreamPlan plan_stream_best(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                            int observed, bool merge, const PassParams& pp,
                            const PlanCostModel& cm) {
    // The schedule reacts strongly to small changes (which sites a tile
    // keeps, tie-breaks), so variants differ by 10-20 % in cost.  The number
    // tried grows with the work of the call (amplitude-steps), keeping the
    // planning time small against the run.
    // A window of 5 steps pays when few low bits are pinned (c = 4 on the
    // ladders: 6 % fewer passes); it is tried with policy 2 only.
    // Variants are ranked on whole-tile staging (cheaper to plan); the chosen
    // plan is staged again below, with the split positions of half-tile
    // exchanges when asked for.
    std::vector<PassParams> vs;
    for (int rotate : {0, 3, 6, 9, 12, 15})
        for (int window : {3, 4, 5})
            for (int policy : {2, 1}) {
                if (window == 5 && policy != 2) continue;
                PassParams v = pp;
                v.half = false;
                v.window = window;
                v.low_policy = policy;
                v.rotate = rotate % std::max(M, 1);
                vs.push_back(v);
            }
    const double work = std::ldexp(double(std::max<int64_t>(n_steps, 1)), M);
    const size_t nv = work < std::ldexp(1.0, 28) ? 1 : work < std::ldexp(1.0, 33) ? 4 : vs.size();
    StreamPlan best;
    double best_cost = 0;
    for (size_t i = 0; i < nv; ++i) {
        StreamPlan sp = plan_stream(M, J, dt, n_steps, observed, merge, vs[i]);
        const double c = plan_cost(sp, cm);
        if (i == 0 || c < best_cost) {
            best = std::move(sp);
            best_cost = c;
        }
    }
    // The chosen plan's register stages again, with a beam search (too slow
    // for every variant); a pass keeps whichever staging is shorter.  For
    // half-tile exchanges every pass is staged again around its split
    // position.
    if (pp.half) {
        for (HostPass& hp : best.passes)
            plan_stages_coalesced(hp, std::min(pp.r, int(hp.sites.size())), pp.c, nv > 1 ? 32 : 1, true);
    } else if (nv > 1) {
        for (HostPass& hp : best.passes) {
            HostPass alt = hp;
            plan_stages_coalesced(alt, std::min(pp.r, int(alt.sites.size())), pp.c, 32);
            if (alt.stages.size() < hp.stages.size()) hp.stages = std::move(alt.stages);
        }
    }
    return best;
}

// --------------------------------------------------------------- resident
ResidentPlan plan_resident(int M, const std::vector<Coupling>& J, double dt, int observed,
                           bool merge, int r, bool profile) {
    ResidentPlan rp;
    rp.prologue.sites.resize(M);
    rp.step.sites.resize(M);
    for (int s = 0; s < M; ++s) rp.prologue.sites[s] = rp.step.sites[s] = s;
    for (HostPass* hp : {&rp.prologue, &rp.step}) {
        hp->bit_in = hp->bit_out = hp->sites;
        hp->layout = hp->sites;
    }
    SeqBuilder sb0(M, J, dt, observed, merge, profile);
    sb0.emit_observable(0);
    rp.prologue.ops = sb0.ops;
    rp.prologue.writes = false;
    SeqBuilder sb(M, J, dt, observed, merge, profile);
    sb.emit_step(1);
    rp.step.ops = sb.ops;
    rp.step.writes = true;
    plan_stages(rp.prologue, std::min(r, M));
    plan_stages(rp.step, std::min(r, M));
    return rp;
}

// ----------------------------------------------------------------- encode
namespace {

// Rank over GF(2) of a small set of bit vectors.
int gf2_rank(std::vector<uint32_t> v) {
    int rank = 0;
    for (int bitp = 31; bitp >= 0; --bitp) {
        int piv = -1;
        for (size_t i = rank; i < v.size(); ++i)
            if (v[i] >> bitp & 1u) { piv = int(i); break; }
        if (piv < 0) continue;
        std::swap(v[rank], v[piv]);
        for (size_t i = 0; i < v.size(); ++i)
            if (int(i) != rank && (v[i] >> bitp & 1u)) v[i] ^= v[rank];
        ++rank;
    }
    return rank;
}

// LDS layout of one tiled pass: element index image of each tile-local
// position p (phys(l) = xor of img[p] over the set bits of l).  Every
// position flips its own index bit and a searched set of the nb lowest index
// bits; the nb x nb block of the lowest positions is kept invertible, so the
// whole map is.  gfx950 serves an LDS access in groups of lanes: a 64-bit
// write by 16 lanes at a time, which must hit distinct 8-byte slots modulo
// 128 bytes, a 64-bit read by 16 lanes (distinct modulo 256 bytes); a
// 128-bit write by 8 lanes (distinct 16-byte slots modulo 128 bytes) and a
// 128-bit read by 16 lanes (modulo 256 bytes).  With lane bits on the lowest
// thread bits, a group is conflict-free when the slot images of its lane
// bits are linearly independent.  Each stage's scatter (every stage but the
// last) and gather (every stage but the first) is checked.
std::vector<uint32_t> search_layout(int k, int elem_bytes, const std::vector<std::vector<int>>& patterns,
                                    uint64_t seed) {
    std::vector<uint32_t> img(k), best;
    int best_def = 1 << 30;
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 1;
    auto rnd = [&]() {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        return st;
    };
    // (lane bits, slot bits) of a write and of a read
    const std::pair<int, int> wr = elem_bytes == 8 ? std::make_pair(4, 4) : std::make_pair(3, 3);
    const std::pair<int, int> rd = elem_bytes == 8 ? std::make_pair(4, 5) : std::make_pair(4, 4);
    const int nb = std::min(k, elem_bytes == 8 ? 5 : 4);
    const uint32_t slot_mask = (1u << nb) - 1;
    auto deficiency = [&](const std::vector<int>& pat, std::pair<int, int> chk) {
        std::vector<uint32_t> v;
        for (int q = 0; q < chk.first && q < int(pat.size()); ++q)
            v.push_back(img[pat[q]] & ((1u << chk.second) - 1));
        return int(v.size()) - gf2_rank(v);
    };
    // the first stage's lanes (input coalescing) and the last stage's (output
    // coalescing) are fixed; the lanes of the stages in between are chosen
    // afterwards (choose_lanes)
    const int ns = int(patterns.size());
    for (int attempt = 0; attempt < 4000; ++attempt) {
        // even attempts keep the lowest positions on themselves
        for (int p = 0; p < k; ++p) {
            const bool keep = attempt == 0 || (attempt % 2 == 0 && p < nb);
            img[p] = (1u << p) ^ (keep ? 0u : uint32_t(rnd()) & slot_mask);
        }
        std::vector<uint32_t> low(img.begin(), img.begin() + nb);
        if (gf2_rank(low) < nb) continue;
        int def = 0;
        if (ns > 1) def += deficiency(patterns[0], wr) + deficiency(patterns[ns - 1], rd);
        for (int si = 1; si + 1 < ns; ++si) {
            // some choice of lanes must satisfy both checks: the thread
            // positions' slot images must span enough
            std::vector<uint32_t> w, r;
            for (int p : patterns[si]) {
                w.push_back(img[p] & ((1u << wr.second) - 1));
                r.push_back(img[p] & ((1u << rd.second) - 1));
            }
            def += std::max(0, wr.first - gf2_rank(w)) + std::max(0, rd.first - gf2_rank(r));
        }
        if (def < best_def) {
            best_def = def;
            best = img;
            if (def == 0) break;
        }
    }
    return best;
}

// Orders the thread positions of a stage between the first and the last so
// that its lowest lane bits take positions whose LDS slot images are
// independent (conflict-free scatter and gather); the rest keep their order.
void choose_lanes(std::vector<int>& tp, const std::vector<uint32_t>& img, int elem_bytes) {
    const int lanes = 4, wbits = elem_bytes == 8 ? 4 : 3, wl = elem_bytes == 8 ? 4 : 3;
    const int rbits = elem_bytes == 8 ? 5 : 4;
    if (int(tp.size()) < lanes) return;
    auto ok = [&](const std::vector<int>& pick) {
        std::vector<uint32_t> w, r;
        for (int q = 0; q < int(pick.size()); ++q) {
            if (q < wl) w.push_back(img[pick[q]] & ((1u << wbits) - 1));
            r.push_back(img[pick[q]] & ((1u << rbits) - 1));
        }
        return gf2_rank(w) == int(w.size()) && gf2_rank(r) == int(r.size());
    };
    // depth-first over ordered picks, pruned by the rank conditions
    std::vector<int> pick, best;
    std::function<bool()> dfs = [&]() {
        if (int(pick.size()) == lanes) return true;
        for (int p : tp) {
            if (std::find(pick.begin(), pick.end(), p) != pick.end()) continue;
            pick.push_back(p);
            if (ok(pick) && dfs()) return true;
            pick.pop_back();
        }
        return false;
    };
    if (!dfs()) return;
    std::vector<int> out = pick;
    for (int p : tp)
        if (std::find(pick.begin(), pick.end(), p) == pick.end()) out.push_back(p);
    tp = out;
}

// Positions on the wave bits of every stage of a multi-stage pass (as
// masks of tile-local positions; zero where the workgroup is one wave).
// The stages are cut into maximal runs whose register positions leave at
// least `nw` positions free; a run's wave positions are free in all its
// stages.  The first stage keeps its 6 lowest-input-bit thread positions on
// the lane bits and the last stage its 6 lowest-output-bit ones, so global
// accesses keep their contiguous runs.  The first run's wave positions are
// also the last run's when both allow it (no barrier at the tile end), and
// positions that keep their address bit are preferred.
std::vector<uint32_t> wave_bits_plan(const HostPass& hp) {
    const int k = int(hp.sites.size()), nst = int(hp.stages.size());
    std::vector<uint32_t> w(nst, 0);
    if (nst == 0) return w;
    const int nw = k - int(hp.stages[0].regs.size()) - 6;
    if (nw <= 0 || nst == 1) return w;
    const uint32_t all = (1u << k) - 1;
    std::vector<uint32_t> forbid(nst, 0);
    for (int si = 0; si < nst; ++si)
        for (int p : hp.stages[si].regs) forbid[si] |= 1u << p;
    auto low6 = [&](int si, const std::vector<int>& bit) {
        std::vector<int> tp;
        for (int p = 0; p < k; ++p)
            if (!((forbid[si] >> p) & 1u)) tp.push_back(p);
        std::stable_sort(tp.begin(), tp.end(), [&](int a, int b) { return bit[a] < bit[b]; });
        uint32_t m = 0;
        for (int q = 0; q < 6 && q < int(tp.size()); ++q) m |= 1u << tp[q];
        return m;
    };
    const uint32_t lo_first = low6(0, hp.bit_in), lo_last = low6(nst - 1, hp.bit_out);
    forbid[0] |= lo_first;
    forbid[nst - 1] |= lo_last;
    // maximal runs
    std::vector<std::pair<int, int>> runs;
    std::vector<uint32_t> avail;
    for (int s0 = 0; s0 < nst;) {
        uint32_t used = forbid[s0];
        if (__builtin_popcount(all & ~used) < nw) throw std::runtime_error("encode: no room for wave bits");
        int e = s0 + 1;
        while (e < nst && __builtin_popcount(all & ~(used | forbid[e])) >= nw) used |= forbid[e++];
        runs.push_back({s0, e});
        avail.push_back(all & ~used);
        s0 = e;
    }
    auto pick = [&](uint32_t cand) {
        uint32_t m = 0;
        int n = 0;
        for (int pass2 = 0; pass2 < 2 && n < nw; ++pass2)
            for (int p = k - 1; p >= 0 && n < nw; --p) {
                if (!((cand >> p) & 1u) || ((m >> p) & 1u)) continue;
                if (pass2 == 0 && hp.bit_in[p] != hp.bit_out[p]) continue;
                m |= 1u << p;
                ++n;
            }
        return m;
    };
    const size_t nr = runs.size();
    std::vector<uint32_t> rw(nr);
    for (size_t r = 0; r < nr; ++r) rw[r] = pick(avail[r]);
    if (nr > 1 && __builtin_popcount(avail[0] & avail[nr - 1]) >= nw)
        rw[0] = rw[nr - 1] = pick(avail[0] & avail[nr - 1]);
    for (size_t r = 0; r < nr; ++r)
        for (int si = runs[r].first; si < runs[r].second; ++si) w[si] = rw[r];
    return w;
}

uint32_t apply_layout(const std::vector<uint32_t>& img, uint32_t l) {
    uint32_t o = 0;
    for (size_t p = 0; p < img.size(); ++p)
        if (l >> p & 1u) o ^= img[p];
    return o;
}

}  // namespace

namespace {

// Dense product of consecutive factors on 5 register bits (32 x 32 complex,
// FP64), applied as each factor's exact two-spin propagator: on register
// index j with bits (qa, qb) anti-aligned, partner j' = j ^ bit qa ^ bit qb,
//   psi_j <- e^{+iA/4} (cos(B/2) psi_j - i sin(B/2) psi_j'),
// aligned: psi_j <- e^{-iA/4} psi_j.
struct StageMatrix {
    std::vector<std::complex<double>> u;   // row-major 32 x 32
    bool any = false;
    StageMatrix() { reset(); }
    void reset() {
        u.assign(32 * 32, 0.0);
        for (int i = 0; i < 32; ++i) u[i * 32 + i] = 1.0;
        any = false;
    }
    void apply(int qa, int qb, double A, double B) {
        const double c = std::cos(0.5 * B), s = std::sin(0.5 * B);
        const std::complex<double> pa = std::polar(1.0, 0.25 * A), pal = std::polar(1.0, -0.25 * A);
        const std::complex<double> mis(0.0, -s);
        std::vector<std::complex<double>> v(u);
        for (int j = 0; j < 32; ++j) {
            const bool anti = ((j >> qa) & 1) != ((j >> qb) & 1);
            const int jp = j ^ (1 << qa) ^ (1 << qb);
            for (int col = 0; col < 32; ++col)
                v[j * 32 + col] = anti ? pa * (c * u[j * 32 + col] + mis * u[jp * 32 + col])
                                       : pal * u[j * 32 + col];
        }
        u.swap(v);
        any = true;
    }
    // Appends the real 64 x 64 form in MFMA A-operand order.
    void emit(std::vector<float>& mats) const {
        auto W = [&](int row, int col) {
            const bool im_out = row >= 32, im_in = col >= 32;
            const std::complex<double> z = u[(row & 31) * 32 + (col & 31)];
            if (!im_out && !im_in) return z.real();
            if (!im_out && im_in) return -z.imag();
            if (im_out && !im_in) return z.imag();
            return z.real();
        };
        for (int b = 0; b < 2; ++b)
            for (int p = 0; p < 32; ++p)
                for (int l = 0; l < 64; ++l) mats.push_back(float(W(32 * b + l % 32, 2 * p + l / 32)));
    }
};

}  // namespace

template <typename T>
void encode_pass(const HostPass& hp, int M, int observed, DevTables<T>& out, bool fixed_swizzle,
                 int engine, bool profile) {
    const int k = int(hp.sites.size());
    constexpr int eb = sizeof(T) * 2;
    DevPass dp{};
    dp.k = k;
    dp.stage0 = int(out.stages.size());
    dp.nstage = int(hp.stages.size());
    dp.writes = hp.writes ? 1 : 0;
    dp.half = hp.split >= 0 ? 1 : 0;
    if (hp.stages.empty()) throw std::runtime_error("encode: pass without stages");
    std::vector<int> local(kMaxSites, -1);
    int64_t tile_bits = 0;
    for (int p = 0; p < k; ++p) {
        dp.tbit[p] = hp.bit_in[p];
        dp.tbit_out[p] = hp.bit_out[p];
        local[hp.sites[p]] = p;
        tile_bits |= int64_t(1) << hp.bit_in[p];
    }
    int nf = 0;
    for (int b = 0; b < M; ++b)
        if (!((tile_bits >> b) & 1)) {
            dp.free_mask |= int64_t(1) << b;
            ++nf;
        }
    dp.nfree = nf;
    dp.obs_free_bit = local[observed] < 0 ? hp.layout[observed] : -1;

    // thread positions of every stage, and the LDS layout
    // Thread bit q of a stage is position tq[q].  The lanes of the last stage
    // of a multi-stage pass take positions in order of output bit, so that
    // consecutive lanes store consecutive addresses; elsewhere position
    // order, which is input-bit order.
    //
    // Wave bits: thread bits 6 and up select the wave.  A stage exchange
    // that keeps the same positions on the wave bits (in the same order)
    // moves every amplitude within its wave, so the wave's LDS slots are its
    // own and no workgroup barrier is needed (wave_bits_plan).
    for (int p = 1; p < k; ++p)
        if (hp.bit_in[p] <= hp.bit_in[p - 1]) throw std::runtime_error("encode: input bits not increasing");
    if (hp.stages.size() == 1 && hp.bit_in != hp.bit_out)
        throw std::runtime_error("encode: one-stage pass that moves amplitudes");
    const int nst = int(hp.stages.size());
    std::vector<uint32_t> wmask(nst, 0);
    if (!fixed_swizzle) wmask = wave_bits_plan(hp);
    std::vector<std::vector<int>> tpos_all, lanes_all;
    for (int si = 0; si < nst; ++si) {
        uint32_t rmask = 0;
        for (int p : hp.stages[si].regs) rmask |= 1u << p;
        std::vector<int> tp, wv;
        for (int p = 0; p < k; ++p)
            if (!(rmask & (1u << p))) ((wmask[si] >> p) & 1u ? wv : tp).push_back(p);
        if (si + 1 == nst && si > 0)
            std::stable_sort(tp.begin(), tp.end(),
                             [&](int a, int b) { return hp.bit_out[a] < hp.bit_out[b]; });
        lanes_all.push_back(tp);
        tp.insert(tp.end(), wv.begin(), wv.end());
        tpos_all.push_back(tp);
    }
    std::vector<uint32_t> img(k);
    if (fixed_swizzle) {
        for (int p = 0; p < k; ++p) img[p] = lds_swizzle<eb>(1u << p);
    } else if (hp.split >= 0) {
        // half-tile exchange: the LDS holds one half at a time, addressed by
        // the other k - 1 positions; the split position has no image (both
        // halves use the same slots)
        const int h = hp.split;
        for (const HostStage& st : hp.stages)
            if (st.regs.empty() || st.regs.back() != h)
                throw std::runtime_error("encode: split position not on the top register bit");
        auto comp = [&](int p) { return p < h ? p : p - 1; };
        std::vector<std::vector<int>> pat;
        for (const auto& lv : lanes_all) {
            std::vector<int> q;
            for (int p : lv) q.push_back(comp(p));
            pat.push_back(q);
        }
        const std::vector<uint32_t> im = search_layout(k - 1, eb, pat, uint64_t(k) * 131 + hp.ops.size());
        for (int p = 0; p < k; ++p) img[p] = p == h ? 0u : im[comp(p)];
        for (int si = 1; si + 1 < nst; ++si) {
            std::vector<int> tp = lanes_all[si];
            choose_lanes(tp, img, eb);
            for (size_t q = 0; q < tp.size(); ++q) tpos_all[si][q] = tp[q];
        }
    } else {
        img = search_layout(k, eb, lanes_all, uint64_t(k) * 131 + hp.ops.size());
        for (int si = 1; si + 1 < nst; ++si) {
            // reorder the lane positions only; the wave positions stay last
            std::vector<int> tp = lanes_all[si];
            choose_lanes(tp, img, eb);
            for (size_t q = 0; q < tp.size(); ++q) tpos_all[si][q] = tp[q];
        }
    }
    // The exchange after stage si crosses waves (workgroup barrier) when the
    // wave positions change.  A wave's stores of a tile may overlap another
    // wave's loads of it unless both keep the same wave positions on the
    // same address bits; then some exchange of the tile must have a
    // workgroup barrier (every wave has consumed its loads once it has made
    // its first exchange), and the first one gets it.  The tile-end barrier
    // is needed when the last stage's waves differ from the first stage's
    // (the next tile's first scatters would land in slots other waves still
    // read).
    std::vector<int> xnext(std::max(nst - 1, 0), 0);
    bool any_cross = false;
    for (int si = 0; si + 1 < nst; ++si) {
        xnext[si] = (fixed_swizzle || wmask[si] != wmask[si + 1]) ? 1 : 0;
        any_cross |= xnext[si] != 0;
    }
    if (nst > 1) {
        bool keep_bits = true;
        for (int p = 0; p < k; ++p)
            if ((wmask[0] >> p) & 1u) keep_bits &= hp.bit_in[p] == hp.bit_out[p];
        if (!any_cross && !(wmask[0] == wmask[nst - 1] && keep_bits)) xnext[0] = 1;
        dp.tile_barrier = (fixed_swizzle || wmask[0] != wmask[nst - 1]) ? 1 : 0;
    }
    auto byte_off = [&](uint32_t l) { return apply_layout(img, l) * uint32_t(eb); };

    int nmeas = 0;
    for (size_t si = 0; si < hp.stages.size(); ++si) {
        const HostStage& hs = hp.stages[si];
        DevStage ds{};
        ds.op0 = int(out.ops.size());
        const int rr = int(hs.regs.size());
        ds.ntb = k - rr;
        ds.xnext = (int(si) + 1 < nst) ? xnext[si] : 1;
        const std::vector<int>& tq = tpos_all[si];
        for (int q = 0; q < ds.ntb; ++q) {
            ds.tmask[q] = byte_off(1u << tq[q]);
            ds.gt_in[q] = int64_t(1) << hp.bit_in[tq[q]];
            ds.gt_out[q] = int64_t(1) << hp.bit_out[tq[q]];
        }
        for (int b = 0; b < rr; ++b) {
            ds.rbit[b] = byte_off(1u << hs.regs[b]);
            ds.gr_in[b] = int64_t(1) << hp.bit_in[hs.regs[b]];
            ds.gr_out[b] = int64_t(1) << hp.bit_out[hs.regs[b]];
        }
        ds.obs_tq = -1;
        ds.obs_mask = 0;
        const int pobs = local[observed];
        if (pobs >= 0) {
            bool in_reg = false;
            for (int b = 0; b < rr; ++b)
                if (hs.regs[b] == pobs) { ds.obs_mask = 1 << b; in_reg = true; }
            if (!in_reg)
                for (int t = 0; t < ds.ntb; ++t)
                    if (tq[t] == pobs) ds.obs_tq = t;
        }
        auto regbit = [&](int p) {
            for (int b = 0; b < rr; ++b)
                if (hs.regs[b] == p) return b;
            throw std::runtime_error("encode: factor site not in registers");
        };
        if (engine == 1 && rr != 5) throw std::runtime_error("encode: matrix engine needs 5 register bits");
        StageMatrix sm;
        auto flush = [&]() {
            if (!sm.any) return;
            DevOp<T> d{};
            d.code = kOpMat;
            d.aux = int32_t(out.mats.size() / kMatFloats);
            sm.emit(out.mats);
            out.ops.push_back(d);
            sm.reset();
        };
        for (int n : hs.ops) {
            const Op& op = hp.ops[n];
            if (op.kind == 1 && profile) {
                flush();
                if (dp.pmeas >= kMaxMeasProfile) throw std::runtime_error("encode: too many observables");
                const int site = op.i, slot = dp.pmeas++;
                int kind = 2, index = hp.layout[site];
                if (local[site] >= 0) {
                    kind = 0;
                    for (int t = 0; t < ds.ntb; ++t)
                        if (tq[t] == local[site]) index = t;
                    for (int b = 0; b < rr; ++b)
                        if (hs.regs[b] == local[site]) {
                            kind = 1;
                            index = b;
                        }
                }
                int nslot = -1;
                if (site == observed) {
                    if (dp.pnorm >= kMaxMeas) throw std::runtime_error("encode: too many norms");
                    nslot = dp.pnorm++;
                    dp.pnorm_meas[nslot] = slot;
                }
                DevOp<T> d{};
                d.code = kOpMeas;
                d.aux = slot | (kind << 6) | (index << 8) | ((nslot + 1) << 14) | (site << 17);
                dp.pmeas_step[slot] = op.step;
                dp.pmeas_site[slot] = int8_t(site);
                out.ops.push_back(d);
                continue;
            }
            if (op.kind == 1) {
                flush();
                if (nmeas >= kMaxMeas) throw std::runtime_error("encode: too many observables");
                DevOp<T> d{};
                d.code = kOpMeas;
                d.aux = nmeas;
                dp.meas_step[nmeas] = op.step;
                ++nmeas;
                out.ops.push_back(d);
                continue;
            }
            int qa = regbit(local[op.i]), qb = regbit(local[op.j]);
            if (qa > qb) std::swap(qa, qb);
            if (engine == 1) {
                sm.apply(qa, qb, op.A, op.B);
                continue;
            }
            // rotation angle theta = B/2; split until |theta| <= pi/2 so the
            // three-shear form stays well conditioned.
            double theta = 0.5 * op.B;
            int pieces = 1;
            while (std::fabs(theta / pieces) > 1.5707963267948966) pieces *= 2;
            for (int pc = 0; pc < pieces; ++pc) {
                DevOp<T> d{};
                const double th = theta / pieces;
                d.code = qa * 8 + qb;
                d.aux = 0;
                d.t = T(std::tan(0.5 * th));
                d.s = T(std::sin(th));
                const double A = pc == 0 ? op.A : 0.0;
                if (A != 0.0) d.code |= kOpZZ;
                d.pr = T(std::cos(0.25 * A));
                d.pi = T(std::sin(0.25 * A));
                out.ops.push_back(d);
            }
        }
        flush();
        ds.nop = int(out.ops.size()) - ds.op0;
        out.stages.push_back(ds);
    }
    dp.nmeas = nmeas;
    out.passes.push_back(dp);
}

template void encode_pass<float>(const HostPass&, int, int, DevTables<float>&, bool, int, bool);
template void encode_pass<double>(const HostPass&, int, int, DevTables<double>&, bool, int, bool);

std::string describe_plan(const StreamPlan& plan) {
    std::ostringstream os;
    os << "launches=" << plan.launch_tmpl.size() << " templates=" << plan.passes.size()
       << " steps=" << plan.n_steps << " passes/step=" << plan.passes_per_step()
       << " period=" << plan.period_passes << "/" << plan.period_steps;
    size_t nst = 0, nop = 0;
    for (auto& p : plan.passes) {
        nst += p.stages.size();
        nop += p.ops.size();
    }
    os << " stages/template=" << (plan.passes.empty() ? 0.0 : double(nst) / plan.passes.size())
       << " ops/template=" << (plan.passes.empty() ? 0.0 : double(nop) / plan.passes.size());
    return os.str();
}

}  // namespace spinqp
