// planner.hpp -- host-side planning of the Strang product into tiled passes.
//
// The symmetric Trotter step (couplings in list order with tau = dt/2, then
// in reverse order with tau = dt/2) is expanded into an op sequence with an
// observable op after every step.  Adjacent factors on the same pair with
// no op in between touching either site are merged (exact: the two-spin
// propagators of one pair commute and add their strengths).  The sequence is
// then cut into passes: each pass owns a set of k sites (its tile bits) and
// applies a down-set-closed run of ops whose sites all lie in that set, so
// every pass is one read + write sweep of the state.  Inside a pass, ops are
// grouped into stages whose sites fit the r register bits of a lane.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "device_plan.hpp"

namespace spinqp {

struct Coupling {
    int i, j;
    double a, b;
};

struct Op {
    int kind;          // 0 = factor, 1 = observable
    int i, j;          // factor sites (i < j); observable: i = j = observed site
    double A, B;       // integrated strengths sum(a*tau), sum(b*tau)
    int64_t step;      // observable: its step index; factor: step of first occurrence
    int idx;           // emission index inside that step (identity for period search)
};

// Emits the merged op sequence step by step.
class SeqBuilder {
  public:
    // profile: the observable of a step is one op per site (site s, step k:
    // the polarisation of site s), each ordered only against that site's
    // factors.
    SeqBuilder(int M, const std::vector<Coupling>& J, double dt, int observed, bool merge,
               bool profile = false);
    void emit_observable(int64_t step);
    void emit_step(int64_t step);   // forward + reverse factors, then observable(step)
    std::vector<Op> ops;

  private:
    void emit_factor(const Coupling& c, double tau, int64_t step);
    int observed_;
    bool merge_;
    bool profile_;
    double dt_;
    std::vector<Coupling> J_;
    std::vector<int> last_;    // per site: index of the last op touching it, or -1
    int idx_ = 0;
    int64_t cur_step_ = -1;
};

struct HostStage {
    std::vector<int> regs;     // register bit q -> tile-local position
    std::vector<int> ops;      // indices into HostPass::ops
};

struct HostPass {
    int split = -1;            // tile-local position held in registers by every stage (the
                               // top register bit), or -1; see PassParams::half
    std::vector<int> sites;    // tile-local position p -> site
    std::vector<int> bit_in;   // tile-local position p -> global bit before the pass (increasing)
    std::vector<int> bit_out;  // tile-local position p -> global bit after the pass
    std::vector<int> layout;   // site -> global bit before the pass (all M sites)
    std::vector<Op> ops;       // execution order
    std::vector<HostStage> stages;
    bool writes = true;
};

struct PassParams {
    int k = 14;                // tile bits
    int r = 5;                 // register bits
    int c = 4;                 // low global bits every tile must contain
    int max_meas = kMaxMeas;
    bool profile = false;      // observables of every site (max_meas kMaxMeasProfile)
    // Half-tile exchanges: one tile position (chosen per pass) is a register
    // position of every stage, on the top register bit, so a stage exchange
    // can move the tile through LDS in two halves (the position's two
    // values), each half through the same LDS slots.
    bool half = false;
    // Scheduling variant (plan_stream tries several and keeps the cheapest
    // by the cost model below):
    int window = 3;            // steps a pass may run ahead of the oldest pending op
    int low_policy = 2;        // next low-bit sites avoid: 0 nothing, 1 the last stage's
                               // registers, 2 also the next pass's first stage
    int rotate = 0;            // start offset of the tile local search (tie-breaking)
};

// Modelled cost of a plan in units of one memory-bound pass: a pass costs
// its sweep plus a share per register stage (an LDS exchange) and per
// factor op (VALU), fitted to measured pass-kernel durations.
struct PlanCostModel {
    double pass = 1.0, stage = 0.26, op = 0.032;
};

// Plan of one evolve call on the tiled (streaming) path.  Launch l runs
// pass template tmpl[l] with its observable step labels shifted by
// offset[l].
struct StreamPlan {
    std::vector<HostPass> passes;      // templates
    std::vector<int> launch_tmpl;
    std::vector<int64_t> launch_offset;
    int64_t n_steps = 0;
    int period_steps = 0;              // 0 if no period was used
    int period_passes = 0;
    double passes_per_step() const {
        return n_steps ? double(launch_tmpl.size()) / double(n_steps) : 0.0;
    }
};

// Stages for one pass.  The first stage is loaded straight from HBM and
// the last stored straight back, so their register sets must avoid the
// positions holding the coalescing address bits (avoid_first / avoid_last,
// masks of tile-local positions); empty stages are added where needed.
// beam: width of the search over stage sequences (1 = greedy).
// force: positions in the register set of every stage.
void plan_stages(HostPass& pass, int r, uint32_t avoid_first = 0, uint32_t avoid_last = 0,
                 int beam = 1, uint32_t force = 0);
// Same, with the masks taken from the pass's layouts: positions whose input
// (output) global bit is below c.  half: also choose the pass's split
// position (HostPass::split) and keep it on the top register bit of every
// stage.
void plan_stages_coalesced(HostPass& pass, int r, int c, int beam = 1, bool half = false);

// Full streaming plan for one scheduling variant: sequence, passes, period
// search, stages.
StreamPlan plan_stream(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                       int observed, bool merge, const PassParams& pp);

// Modelled cost of a plan (whole call).
double plan_cost(const StreamPlan& plan, const PlanCostModel& cm = PlanCostModel());

// Tries a set of scheduling variants of pp and returns the plan of least
// modelled cost.
StreamPlan plan_stream_best(int M, const std::vector<Coupling>& J, double dt, int64_t n_steps,
                            int observed, bool merge, const PassParams& pp,
                            const PlanCostModel& cm = PlanCostModel());

// Plan for a state that fits one workgroup: stages over all M sites for the
// prologue (observable of step 0) and for one periodic step (factors, then
// the observable).  No merging across step boundaries, so every step is
// identical.
struct ResidentPlan {
    HostPass prologue;
    HostPass step;
};
ResidentPlan plan_resident(int M, const std::vector<Coupling>& J, double dt, int observed,
                           bool merge, int r, bool profile = false);

// Encoded device tables.
template <typename T>
struct DevTables {
    std::vector<DevPass> passes;
    std::vector<DevStage> stages;
    std::vector<DevOp<T>> ops;
    std::vector<float> mats;           // matrix engine: kMatFloats per kOpMat
};

// Encodes one pass (or the stages of a one-workgroup plan) into the device
// tables.  fixed_swizzle: use the one-workgroup kernel's fixed LDS swizzle
// instead of a layout searched for this pass.  engine 1: the factors of each
// stage (between observables) become one kOpMat (needs 5 register bits).
// profile: observables of every site, each with its own slot (see kOpMeas).
template <typename T>
void encode_pass(const HostPass& hp, int M, int observed, DevTables<T>& out,
                 bool fixed_swizzle = false, int engine = 0, bool profile = false);

std::string describe_plan(const StreamPlan& plan);

}  // namespace spinqp
