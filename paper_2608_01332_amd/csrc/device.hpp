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
// Phase flag (with RCR_PHASE_FIRST_RHS): that right-hand side is the factor's
// only one (a float64 rcr_solve), so the local factor does not store A^cl,
// which only the initialisation of later right-hand sides reads.
constexpr int RCR_PHASE_ONE_RHS = 8;

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
  int32_t *uabs = nullptr;  // per node: 1 when it is absorbed into (its U is kept in U)
  int32_t *rest = nullptr;  // edge slots that no level-1 primitive consumes (condensed on their own)
  int64_t n_rest = 0;
  bool l1_fusable = false;  // level 1 holds only rakes and compresses of original edge slots
  int32_t *rg_n = nullptr, *rg_m = nullptr;  // ragged plans: per-node dimensions
  int64_t *rg_off = nullptr;                 // ragged plans: block offsets of the packed arrays
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

// Cache key of a captured launch sequence: the buffer addresses it was
// captured with and a tag for the entry point and its options.
using GraphKey = std::vector<uintptr_t>;

// At most this many captured sequences are kept per plan (least recently used
// evicted); an evicted or dropped graph is destroyed only after its own latest
// replay has completed.
constexpr size_t GRAPH_CACHE_CAP = 8;

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after every replay of exec
  uint64_t tick = 0;          // last use
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
  uint64_t tick = 0;
};

struct PlanObj {
  PlanHost host;
  LaunchCfg cfg;
  PlanDev dev;
  std::mutex mu;
  void *ws[2] = {nullptr, nullptr};  // plan-owned workspace per precision
  bool ws_factor[2] = {false, false};  // it holds a factor made by rcr_factor
  size_t ws_bytes[2] = {0, 0};
  hipEvent_t last_done = nullptr;    // completion of the latest solve (stream-ordered release)
  std::map<GraphKey, GraphEntry> graphs;
  std::map<GraphKey, TimedGraph> timed;  // the per-class-run graphs used for timing
  uint64_t tick = 0;                     // use counter of the graph caches
  std::vector<hipEvent_t> events;
  double *resid_buf = nullptr;           // device scratch of rcr_kkt_residual (status words + accumulator)
  uint64_t serial = 0;                   // unique id of the plan (never reused)
};

// One right-hand side (q, r, c) and the buffers of its solution (x, u, lam):
// caller-owned float64 device arrays in the layouts of rcr.h.
struct RhsIO {
  const double *q, *r, *c;
  double *x, *u, *lam;
};

int plan_upload(PlanObj &P, hipStream_t st);

// Device memory of the library, from the calling GPU's stream-ordered pool
// (released with hipFreeAsync).
hipError_t dev_alloc(void **p, size_t bytes, hipStream_t st);

// The plan of build_plan with the list-rank selection, computed on the device
// from a device parent array (dplan.hip); the schedules are copied back into P.
int device_plan(const int64_t *parent, int64_t N, int n, int m, hipStream_t st, PlanHost &P);
// Bytes of a plan's device copy (its integer arrays), made by plan_upload.
size_t plan_device_bytes(const PlanHost &h);
void plan_release_device(PlanObj &P);

int solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
          hipStream_t stream);

void drop_graphs(PlanObj &P);
size_t graph_cache_size(const PlanObj &P);

// Algorithm 1, Steps 2-3 (factor into the workspace and K, P) and Steps 4-6
// for k right-hand sides on that factor.
int factor(PlanObj &P, const rcr_problem &in, double *K, double *Pm, const rcr_solve_options &opt,
           hipStream_t stream);
int solve_rhs(PlanObj &P, const rcr_problem &in, const double *K, const double *Pm, int32_t k, const RhsIO *ios,
              const rcr_solve_options &opt, hipStream_t stream);
// Gradients of a scalar loss through the solve, from its seeds dL/dx, dL/du, dL/dy.
int adjoint(PlanObj &P, const rcr_problem &in, const rcr_solution &fwd, const double *gx, const double *gu,
            const double *gy, const rcr_gradient &g, const rcr_solve_options &opt, hipStream_t stream);
// Max-abs residual of eq. (kkt) of a given iterate into *opt.kkt_residual.
int kkt_residual(PlanObj &P, const rcr_problem &in, const rcr_solution &sol, const rcr_solve_options &opt,
                 hipStream_t stream);
// k trees with their own buffers through the merged plan B of their forest.
int batch_solve(PlanObj &B, int32_t k, const rcr_problem *in, rcr_solution *out, const rcr_solve_options &opt,
                hipStream_t stream);
size_t batch_workspace_bytes(const PlanHost &B, int precision);
// rcr_solve on the per-device static scratch array (no allocation).
int solve_noalloc(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
                  hipStream_t stream);
size_t noalloc_scratch_bytes();

int tune(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt, hipStream_t stream,
         LaunchCfg &best, float &best_ms);

// Non-uniform dimensions: pack into the padded uniform problem, solve, unpack.
int ragged_solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
                 hipStream_t stream);

int lift_solve(PlanObj &P, const rcr_native_problem &in, rcr_native_solution &out, const rcr_solve_options &opt,
               hipStream_t stream);

}  // namespace rcr
