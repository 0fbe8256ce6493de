// Host-side topology plan of the rake-compress contraction (Sec. VII).
//
// The plan is built once from the parent array and reused by every solve on
// that topology (Algorithm 1, Step 1).  It records, for each primitive
// operation, the static slot indices of its inputs and outputs and its
// earliest-start dependency level (eq. (earliest-level)), so the executor can
// launch all operations of one level together with no write conflicts
// (unique writer per datum, reads only of data produced at earlier levels).
#pragma once

#include <cstdint>
#include <vector>

namespace rcr {

enum OpKind : int32_t { OP_RAKE = 0, OP_COMBINE = 1, OP_ABSORB = 2, OP_COMPRESS = 3 };

// One primitive operation; field meaning depends on kind (see rcr.h, rcr_plan_export).
struct OpRec {
  int32_t kind, round, level, a, b, c, d, e;
};

// Flags carried, on the device, in the `round` word of an op record (the
// host plan keeps the round): OPF_U_LIVE, node a's U is kept in U (the node
// is absorbed into before it is raked or compressed), else U_a = Q_a;
// OPF_FIRST_ABSORB, the first absorb of node a, which starts from Q_a.  In the
// expansion records the flag OPF_U_LIVE of node j is the fourth word.
enum : int32_t { OPF_U_LIVE = 1, OPF_FIRST_ABSORB = 2 };

// Four int32 words: the records of the expansion and state passes.
struct Op4 {
  int32_t a, b, c, d;
};

struct PlanHost {
  int64_t N = 0;
  int n = 0, m = 0;
  int64_t root = -1;
  int selection = 0;
  // statistics
  int64_t height = 0, leaves = 0, max_degree = 0, rounds = 0;
  int64_t n_rake = 0, n_compress = 0, n_combine = 0, n_absorb = 0;
  int64_t n_contrib = 0;     // rake + combine output slots
  int64_t n_edge_slots = 0;  // N original slots + one per compression
  // CREW check of the level schedule (verify_crew), run on the first request
  // for the plan's statistics: -1 not yet run, else 0 / 1
  mutable int crew = -1;

  // contraction (quadratic and affine passes): ops sorted by (level, kind);
  // ops of level t (1-based) are [lvl_off[t-1], lvl_off[t]).
  std::vector<OpRec> ops;
  std::vector<int64_t> lvl_off;
  // kind_off[5 t + s]: first op of kind s in level t + 1 (s = 0..3), kind_off[5 t + 4] its end
  std::vector<int64_t> kind_off;

  // expansion of compressions: {j, r slot, child k, 0}; level-major like ops.
  // Raked nodes and the root need no expansion op (their value is final when
  // the node leaves the contraction).
  std::vector<Op4> exp_ops;
  std::vector<int64_t> exp_off;

  // composition of edge maps along compressions only (composite transition
  // matrices and state offsets): {l slot, r slot, new slot, j}.
  std::vector<Op4> tc_ops;
  std::vector<int64_t> tc_off;

  // state expansion: {j, edge slot into j at removal, parent at removal, 0}.
  std::vector<Op4> sx_ops;
  std::vector<int64_t> sx_off;

  std::vector<int32_t> parent32;  // original parent array (root: -1)

  // batched plans: a forest of independent trees; tree t owns nodes
  // [tree_off[t], tree_off[t + 1])
  std::vector<int64_t> tree_off;

  // lifted plans of node-control problems (Sec. II-B): the native tree has
  // lift_N nodes of state dimension lift_n; native non-leaf i has the decision
  // node lift_plus[i] (-1 for leaves).  lift_N == 0 for ordinary plans.
  int64_t lift_N = 0;
  int lift_n = 0;
  std::vector<int32_t> lift_plus;

  // ragged plans: node v has state dimension rg_n[v] and the edge into it
  // control dimension rg_m[v] (0 at the root), all padded to n and m for the
  // solve; rg_off[f * (N + 1) + v] is the element offset of v's block of field
  // f (RG_FIELDS, in the order of rcr_ragged_offsets) in the caller's packed
  // arrays, rg_off[f * (N + 1) + N] the field's length.  Empty otherwise.
  std::vector<int32_t> rg_n, rg_m;
  std::vector<int64_t> rg_off;

  int64_t levels() const { return (int64_t)lvl_off.size() - 1; }
  int64_t expand_levels() const { return (int64_t)exp_off.size() - 1; }
  int64_t state_levels() const { return (int64_t)tc_off.size() - 1; }
  int64_t sexp_levels() const { return (int64_t)sx_off.size() - 1; }
};

// Returns 0 or a negative RCR_* status.
// Independent check that every pass schedule is CREW (one writer per datum,
// reads only of data written at a lower level): the contraction, the
// expansion of compressions, the composition of edge maps (with its pairing
// with the affine contraction) and the state expansion (verify_crew in plan.cpp).
bool verify_crew(const PlanHost &P);
// While set on a thread, the plans and merges it builds use no helper threads.
extern thread_local bool build_on_caller_only;

int build_plan(const int64_t *parent, int64_t N, int n, int m, int selection, PlanHost &out);

// Plan of the lifted edge-control tree of a node-control problem (Sec. II-B,
// Prop. 2) on the native tree `parent` with state dimension n and control
// dimension m: the lifted state has dimension n + m.  Returns 0 or a negative
// RCR_* status.
int build_lift_plan(const int64_t *parent, int64_t N, int n, int m, int selection, PlanHost &out);

// Fields of a ragged problem and solution, in the order of rcr_ragged_offsets.
constexpr int RG_FIELDS = 14;

// Plan of a tree whose node v has state dimension n_node[v] and whose edge into
// v has control dimension m_edge[v] (ignored at the root): the topology plan
// of build_plan for the largest dimensions, plus the block offsets of the
// packed (ragged) arrays.  Returns 0 or a negative RCR_* status.
int build_ragged_plan(const int64_t *parent, int64_t N, const int32_t *n_node, const int32_t *m_edge, int selection,
                      PlanHost &out);

// Merge the plans of independent trees into one plan of their forest: node,
// edge and contribution slots are offset per tree, and dependency level t of
// the merged plan is the union of every tree's level t (trees are disjoint, so
// the union keeps a unique writer per datum).  Returns 0 or a negative RCR_* status.
int merge_plans(const std::vector<const PlanHost *> &parts, PlanHost &out);

// D_N of Lemma 4 (eq. (dependency-level-bound)).
int64_t depth_bound(int64_t N);

}  // namespace rcr
