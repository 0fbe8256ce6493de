// Device-side executor interface: plan upload, workspace layout, and the
// launch sequence of one factor + solve (Algorithm 1, Steps 2-6).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rcr.h"
#include "plan.hpp"

namespace rcr {

// Phase flag: the factor and the solve of one rcr_solve share its first
// right-hand side, so the wide local factor may initialise that solve.
constexpr int RCR_PHASE_FIRST_RHS = 4;

// Device copy of a plan's integer arrays.
// The residual kernel sums a node's child terms in one team; a node with more
// children than this is summed by a workgroup of its own (k_residual_hub).
constexpr int RES_HUB = 64;

struct PlanDev {
  int device = -1;
  char *base = nullptr;  // one allocation holding every array below
  OpRec *ops = nullptr;
  Op4 *exp_ops = nullptr, *tc_ops = nullptr, *sx_ops = nullptr;
  int32_t *parent = nullptr;
  int32_t *child_off = nullptr, *child_idx = nullptr;  // children in increasing id (residual)
  int32_t *hubs = nullptr;  // nodes with more than RES_HUB children, increasing id (residual)
  int64_t n_hubs = 0;
  int64_t *koff = nullptr, *exp_off = nullptr, *tc_off = nullptr, *sx_off = nullptr;  // level offsets
  int32_t *lift_plus = nullptr;  // lifted plans: decision node of each native non-leaf
  size_t bytes = 0;
};

// Element offsets (in units of the working type) of the solver's scratch arrays.
struct WsLayout {
  size_t U, EA, EC, EP, CT, PW, Finv, W, Ginv, Acl, Tm, Kw;  // matrices
  size_t h, cv, z, p, kff, b, xw, uw, yw;                     // vectors
  size_t rq, rr, rc;                                          // right-hand side copies (mixed)
  size_t total_bytes;
};

// The first WS_HEADER_BYTES of a workspace hold the solve's status words
// (bytes 0..255) and its residual accumulator (bytes 256..263), so that one
// plan can serve concurrent solves on different streams with distinct workspaces.
constexpr size_t WS_HEADER_BYTES = 512;

WsLayout workspace_layout(const PlanHost &ph, int precision);

// Whole device scratch of a solve with this plan: the solver's workspace and,
// for a lifted plan, the float64 lifted problem and solution that follow it.
size_t total_workspace_bytes(const PlanHost &ph, int precision);

struct GraphKey {
  const void *p[16];
  bool operator<(const GraphKey &o) const {
    for (int i = 0; i < 16; ++i)
      if (p[i] != o.p[i]) return p[i] < o.p[i];
    return false;
  }
};

// Launch mapping of the narrow levels (rcr_launch_config; 0 = default).
struct LaunchCfg {
  int quad_tail_rounds = 0, vec_tail_rounds = 0, vec_tail_waves = 0;
};

// The launch sequence captured for timing: one graph per run of same-class
// launches (cls[i] = -1 for a run of untimed launches), replayed one after the
// other with a HIP event recorded on the stream between them (events[i] before
// graph i, events[n] after the last).
struct TimedGraph {
  std::vector<hipGraphExec_t> execs;
  std::vector<int> cls;
  std::vector<hipEvent_t> events;
  int launches[RCR_NUM_KERNEL_CLASSES] = {};
};

struct PlanObj {
  PlanHost host;
  LaunchCfg cfg;
  PlanDev dev;
  std::mutex mu;
  void *ws[2] = {nullptr, nullptr};  // plan-owned workspace per precision
  size_t ws_bytes[2] = {0, 0};
  hipEvent_t last_done = nullptr;    // completion of the latest solve (stream-ordered release)
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::map<GraphKey, TimedGraph> timed;  // the per-class-run graphs used for timing
  std::vector<hipEvent_t> events;
};

int plan_upload(PlanObj &P, hipStream_t st);
void plan_release_device(PlanObj &P);

int solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
          hipStream_t stream);

void drop_graphs(PlanObj &P);

int tune(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt, hipStream_t stream,
         LaunchCfg &best, float &best_ms);

int lift_solve(PlanObj &P, const rcr_native_problem &in, rcr_native_solution &out, const rcr_solve_options &opt,
               hipStream_t stream);

}  // namespace rcr
