// planner.cpp -- Strang op sequence, pass scheduling, stage scheduling and
// encoding of the device tables.  Host only.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <sstream>
#include <stdexcept>

namespace spinqp {

// ------------------------------------------------------------------ sequence
SeqBuilder::SeqBuilder(int M, const std::vector<Coupling>& J, double dt, int observed, bool merge)
    : observed_(observed), merge_(merge), dt_(dt), J_(J), last_(M, -1) {}

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
    ops.push_back(Op{1, observed_, observed_, 0.0, 0.0, step, 1 << 30});
    last_[observed_] = int(ops.size()) - 1;
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
        int nmeas = 0;
        double score = 0;
        auto consider = [&](int s) {
            if (h[s] < int(site_ops[s].size())) {
                int n = site_ops[s][h[s]];
                if (eligible(n, T) && ready(n, h)) work.push_back(n);
            }
        };
        for (int s = 0; s < M; ++s)
            if ((T & bit(s)) || s == observed) consider(s);
        while (!work.empty()) {
            int n = work.back();
            work.pop_back();
            if (!ready(n, h)) continue;
            const Op& op = ops[n];
            if (op.kind == 1) {
                if (nmeas >= max_meas) continue;
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

    Mask choose_tile(Mask forced) {
        // Seed: sites of the earliest pending ops, in sequence order.
        Mask T = forced;
        for (size_t n = first_pending; n < ops.size() && popc(T) < k; ++n) {
            if (done[n] || ops[n].kind == 1) continue;
            Mask add = bit(ops[n].i) | bit(ops[n].j);
            if (popc(T | add) <= k) T |= add;
            if (n - first_pending > 4096) break;
        }
        for (int s = 0; s < M && popc(T) < k; ++s) T |= bit(s);
        double best = closure(T, nullptr);
        // First-improvement local search over single-site swaps.
        for (int round = 0; round < 64; ++round) {
            bool improved = false;
            for (int out = 0; out < M && !improved; ++out) {
                if (!(T & bit(out)) || (forced & bit(out))) continue;
                for (int in = 0; in < M; ++in) {
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
        return T;
    }

    // Schedules one pass; returns the applied op indices (sorted) and T.
    std::vector<int> next_pass(Mask forced, Mask* Tout) {
        all_done();
        limit = ops[first_pending].step + window;
        Mask T = choose_tile(forced);
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
    bool any_factor = false;
    for (int n : applied) {
        hp.ops.push_back(ops[n]);
        any_factor |= ops[n].kind == 0;
    }
    hp.writes = any_factor;
    return hp;
}

std::vector<Op> gen_sequence(int M, const std::vector<Coupling>& J, double dt, int observed,
                             bool merge, int64_t s_begin, int64_t s_end, bool initial_obs,
                             bool barrier) {
    // barrier: the observable is made to depend on every site (encoded by
    // emitting it as an op on each site in turn is not possible), so the
    // caller asks for no merging and the scheduler treats steps separately.
    (void)barrier;
    SeqBuilder sb(M, J, dt, observed, merge);
    if (initial_obs) sb.emit_observable(0);
    for (int64_t s = s_begin; s <= s_end; ++s) sb.emit_step(s);
    return sb.ops;
}

}  // namespace

// ----------------------------------------------------------------- stages
void plan_stages(HostPass& pass, int r) {
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
    std::vector<int> head(k + 1, 0);
    std::vector<char> done(nops, 0);
    int ndone = 0;
    auto ready = [&](int n, const std::vector<int>& h) {
        return h[li[n]] == pi[n] && h[lj[n]] == pj[n];
    };
    while (ndone < nops) {
        // Greedy growth from the earliest ready ops; try a few seeds.
        int best_cnt = -1;
        std::vector<int> best_ops;
        uint32_t best_S = 0;
        std::vector<int> seeds;
        for (int n = 0; n < nops && int(seeds.size()) < 6; ++n)
            if (!done[n] && ready(n, head) && pass.ops[n].kind == 0) seeds.push_back(n);
        if (seeds.empty()) seeds.push_back(-1);
        for (int seed : seeds) {
            std::vector<int> h = head;
            uint32_t S = 0;
            if (seed >= 0) S = (1u << li[seed]) | (1u << lj[seed]);
            std::vector<int> got;
            std::vector<char> taken(nops, 0);
            int cnt = 0;
            bool changed = true;
            while (changed) {
                changed = false;
                for (int n = 0; n < nops; ++n) {
                    if (done[n] || taken[n] || !ready(n, h)) continue;
                    const Op& op = pass.ops[n];
                    if (op.kind == 0) {
                        uint32_t need = (1u << li[n]) | (1u << lj[n]);
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
            if (cnt > best_cnt) {
                best_cnt = cnt;
                best_ops = got;
                best_S = S;
            }
        }
        if (best_ops.empty()) throw std::runtime_error("planner: stage made no progress");
        // Fill the register set up to r positions, highest positions first
        // (keeps the lanes on low positions: contiguous LDS addresses).
        for (int p = k - 1; p >= 0 && __builtin_popcount(best_S) < std::min(r, k); --p)
            best_S |= 1u << p;
        HostStage st;
        for (int p = 0; p < k; ++p)
            if (best_S & (1u << p)) st.regs.push_back(p);
        std::sort(best_ops.begin(), best_ops.end());
        for (int n : best_ops) {
            done[n] = 1;
            ++ndone;
            head[li[n]] = std::max(head[li[n]], pi[n] + 1);
            head[lj[n]] = std::max(head[lj[n]], pj[n] + 1);
        }
        st.ops = best_ops;
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
    HostPass obs;
    for (int s = 0; s < k; ++s) obs.sites.push_back(s);
    obs.ops.push_back(Op{1, observed, observed, 0, 0, 0, 1 << 30});
    obs.writes = false;
    plan.passes.push_back(obs);
    SeqBuilder sb(M, J, dt, observed, merge);
    sb.emit_step(1);
    Sched sc(M, observed, k, pp.max_meas, sb.ops);
    while (!sc.all_done()) {
        Mask T;
        auto ap = sc.next_pass(forced, &T);
        plan.passes.push_back(make_pass(sb.ops, ap, T, M));
    }
    for (auto& p : plan.passes) plan_stages(p, std::min(pp.r, int(p.sites.size())));
    plan.launch_tmpl.push_back(0);
    plan.launch_offset.push_back(0);
    for (int64_t st = 0; st < n_steps; ++st)
        for (size_t t = 1; t < plan.passes.size(); ++t) {
            plan.launch_tmpl.push_back(int(t));
            plan.launch_offset.push_back(st);
        }
    plan.period_steps = 1;
    plan.period_passes = int(plan.passes.size()) - 1;
    return plan;
}

static StreamPlan plan_stream_pipelined(int M, const std::vector<Coupling>& J, double dt,
                                        int64_t n_steps, int observed, bool merge,
                                        const PassParams& pp);

StreamPlan plan_stream(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                       int observed, bool merge, const PassParams& pp) {
    try {
        return plan_stream_pipelined(M, J, dt, n_steps, observed, merge, pp);
    } catch (const std::runtime_error&) {
        return plan_stream_per_step(M, J, dt, n_steps, observed, merge, pp);
    }
}

static StreamPlan plan_stream_pipelined(int M, const std::vector<Coupling>& J, double dt,
                                        int64_t n_steps, int observed, bool merge,
                                        const PassParams& pp) {
    StreamPlan plan;
    plan.n_steps = n_steps;
    if (M > 63) throw std::runtime_error("planner: M too large");
    const int k = std::min(pp.k, M);
    Mask forced = 0;
    for (int s = 0; s < std::min(pp.c, k); ++s) forced |= bit(s);

    const int64_t kGen = 48;     // steps generated when searching for a period
    const int64_t kSafe = 8;     // steps kept between the frontier and the end
    auto finish = [&](std::vector<HostPass>& passes) {
        for (auto& p : passes) plan_stages(p, std::min(pp.r, int(p.sites.size())));
    };

    if (n_steps <= 2 * kGen) {
        std::vector<Op> ops = gen_sequence(M, J, dt, observed, merge, 1, n_steps, true, false);
        Sched sc(M, observed, k, pp.max_meas, ops);
        while (!sc.all_done()) {
            Mask T;
            auto ap = sc.next_pass(forced, &T);
            plan.passes.push_back(make_pass(ops, ap, T, M));
        }
        finish(plan.passes);
        for (size_t t = 0; t < plan.passes.size(); ++t) {
            plan.launch_tmpl.push_back(int(t));
            plan.launch_offset.push_back(0);
        }
        return plan;
    }

    // Long run: schedule the first kGen steps, look for a repeating frontier.
    std::vector<Op> ops = gen_sequence(M, J, dt, observed, merge, 1, kGen, true, false);
    Sched sc(M, observed, k, pp.max_meas, ops);
    std::map<std::vector<int64_t>, std::pair<int, int64_t>> seen;
    std::vector<HostPass> passes;
    int p1 = -1, p2 = -1;
    int64_t s1 = 0, s2 = 0;
    std::vector<int64_t> sig;
    int64_t base = 0;
    while (!sc.all_done()) {
        if (sc.signature(&sig, &base)) {
            if (base > kGen - kSafe) break;
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
        Mask T;
        auto ap = sc.next_pass(forced, &T);
        passes.push_back(make_pass(ops, ap, T, M));
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
    std::vector<Op> tops = gen_sequence(M, J, dt, observed, merge, gen_from, n_steps, false, false);
    Sched tc(M, observed, k, pp.max_meas, tops);
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
    while (!tc.all_done()) {
        Mask T;
        auto ap = tc.next_pass(forced, &T);
        tail.push_back(make_pass(tops, ap, T, M));
    }
    for (auto& tp : tail) {
        plan.launch_tmpl.push_back(int(plan.passes.size()));
        plan.launch_offset.push_back(0);
        plan.passes.push_back(std::move(tp));
    }
    finish(plan.passes);
    return plan;
}

// --------------------------------------------------------------- resident
ResidentPlan plan_resident(int M, const std::vector<Coupling>& J, double dt, int observed,
                           bool merge, int r) {
    ResidentPlan rp;
    rp.prologue.sites.resize(M);
    rp.step.sites.resize(M);
    for (int s = 0; s < M; ++s) rp.prologue.sites[s] = rp.step.sites[s] = s;
    rp.prologue.ops.push_back(Op{1, observed, observed, 0, 0, 0, 0});
    rp.prologue.writes = false;
    SeqBuilder sb(M, J, dt, observed, merge);
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
// position p (phys(l) = xor of img[p] over the set bits of l).  Positions
// below `nb` (the bank-slot bits: 32 slots of 8 bytes or 16 of 16 bytes in a
// 256-byte bank row) map to themselves; higher positions also flip a
// searched set of slot bits.  The search makes every access pattern of the
// pass -- the load/store layout and each stage's gather -- map the lanes of
// a 2^nb-lane group onto distinct slots (no bank conflicts).
std::vector<uint32_t> search_layout(int k, int nb, const std::vector<std::vector<int>>& patterns,
                                    uint64_t seed) {
    std::vector<uint32_t> img(k), best;
    int best_def = 1 << 30;
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 1;
    auto rnd = [&]() {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        return st;
    };
    const uint32_t slot_mask = (1u << nb) - 1;
    for (int attempt = 0; attempt < 4000; ++attempt) {
        for (int p = 0; p < k; ++p)
            img[p] = (1u << p) | (p >= nb && attempt > 0 ? uint32_t(rnd()) & slot_mask : 0u);
        int def = 0;
        for (const auto& pat : patterns) {
            std::vector<uint32_t> v;
            for (size_t q = 0; q < pat.size() && int(q) < nb; ++q) v.push_back(img[pat[q]] & slot_mask);
            def += int(v.size()) - gf2_rank(v);
        }
        if (def < best_def) {
            best_def = def;
            best = img;
            if (def == 0) break;
        }
    }
    return best;
}

uint32_t apply_layout(const std::vector<uint32_t>& img, uint32_t l) {
    uint32_t o = 0;
    for (size_t p = 0; p < img.size(); ++p)
        if (l >> p & 1u) o ^= img[p];
    return o;
}

}  // namespace

template <typename T>
void encode_pass(const HostPass& hp, int M, int observed, int r, int nthreads, int vec,
                 DevTables<T>& out, bool fixed_swizzle) {
    const int k = int(hp.sites.size());
    constexpr int eb = sizeof(T) * 2;
    DevPass dp{};
    dp.k = k;
    dp.stage0 = int(out.stages.size());
    dp.nstage = int(hp.stages.size());
    dp.writes = hp.writes ? 1 : 0;
    int nf = 0;
    std::vector<int> local(kMaxSites, -1);
    for (int p = 0; p < k; ++p) {
        dp.tbit[p] = hp.sites[p];
        local[hp.sites[p]] = p;
    }
    for (int s = 0; s < M; ++s)
        if (local[s] < 0) {
            dp.fbit[nf++] = s;
            dp.free_mask |= int64_t(1) << s;
        }
    dp.nfree = nf;
    dp.obs_free_bit = local[observed] < 0 ? observed : -1;
    // load/store iterations: element e = it*nthreads*vec + t*vec + v
    const int per_thread = (1 << k) / nthreads;     // amplitudes per lane
    const int nit = per_thread / vec;
    if (nit > 64 || nit < 1 || (nit & (nit - 1))) throw std::runtime_error("encode: bad iteration count");
    const int lo = __builtin_ctz(unsigned(nthreads * vec));
    const int vb = __builtin_ctz(unsigned(vec));

    // thread positions of every stage, and the LDS layout
    std::vector<std::vector<int>> tpos_all;
    for (const HostStage& hs : hp.stages) {
        uint32_t rmask = 0;
        for (int p : hs.regs) rmask |= 1u << p;
        std::vector<int> tp;
        for (int p = 0; p < k; ++p)
            if (!(rmask & (1u << p))) tp.push_back(p);
        tpos_all.push_back(tp);
    }
    std::vector<uint32_t> img(k);
    if (fixed_swizzle) {
        for (int p = 0; p < k; ++p) img[p] = lds_swizzle<eb>(1u << p);
    } else {
        std::vector<std::vector<int>> patterns = tpos_all;
        std::vector<int> ld;
        for (int q = 0; vb + q < lo; ++q) ld.push_back(vb + q);
        patterns.push_back(ld);
        img = search_layout(k, eb == 8 ? 5 : 4, patterns, uint64_t(k) * 131 + hp.ops.size());
    }
    auto byte_off = [&](uint32_t l) { return apply_layout(img, l) * uint32_t(eb); };
    for (int b = 0; (1 << b) < nit; ++b) {
        dp.it_gbit[b] = int64_t(1) << hp.sites[lo + b];
        dp.it_lbit[b] = byte_off(1u << (lo + b));
    }
    for (int q = 0; vb + q < lo && q < 16; ++q) dp.ld_tmask[q] = byte_off(1u << (vb + q));

    int nmeas = 0;
    for (size_t si = 0; si < hp.stages.size(); ++si) {
        const HostStage& hs = hp.stages[si];
        DevStage ds{};
        ds.op0 = int(out.ops.size());
        const int rr = int(hs.regs.size());
        ds.ntb = k - rr;
        const std::vector<int>& tq = tpos_all[si];
        for (int q = 0; q < ds.ntb; ++q) ds.tmask[q] = byte_off(1u << tq[q]);
        for (int b = 0; b < rr; ++b) ds.rbit[b] = byte_off(1u << hs.regs[b]);
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
        for (int n : hs.ops) {
            const Op& op = hp.ops[n];
            if (op.kind == 1) {
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
        ds.nop = int(out.ops.size()) - ds.op0;
        out.stages.push_back(ds);
    }
    dp.nmeas = nmeas;
    out.passes.push_back(dp);
}

template void encode_pass<float>(const HostPass&, int, int, int, int, int, DevTables<float>&, bool);
template void encode_pass<double>(const HostPass&, int, int, int, int, int, DevTables<double>&, bool);

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
