// C-ABI entry points (include/rcr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rcr.h"
#include "device.hpp"
#include "plan.hpp"

struct rcr_plan {
  rcr::PlanObj obj;
};

namespace {
// Plans get a serial id that is never reused, so a cache keyed by ids cannot
// confuse a destroyed plan with a new one at the same address.
std::atomic<uint64_t> next_serial{1};

// Sets rcr::build_on_caller_only for the duration of one plan construction.
struct CallerOnly {
  explicit CallerOnly(const rcr_plan_options *opt) { rcr::build_on_caller_only = opt && opt->single_thread; }
  ~CallerOnly() { rcr::build_on_caller_only = false; }
};

rcr_plan *new_plan() {
  rcr_plan *p = new (std::nothrow) rcr_plan();
  if (p) p->obj.serial = next_serial.fetch_add(1);
  return p;
}

// Merged plans of rcr_batch_solve, keyed by the serial ids of their parts in
// order; least recently used dropped beyond the cap.  An entry is held by
// shared_ptr while a call uses it, so dropping it never frees a plan in use.
struct MergedEntry {
  std::vector<uint64_t> key;
  std::shared_ptr<rcr_plan> plan;
  uint64_t tick = 0;
};
constexpr size_t MERGED_CAP = 32;
std::mutex merged_mu;
uint64_t merged_tick = 0;
std::vector<MergedEntry> &merged_cache() {
  static std::vector<MergedEntry> *c = new std::vector<MergedEntry>();
  return *c;
}

void destroy_plan(rcr_plan *p);

// The cached merged plan of `plans` (built on a miss).
int merged_plan(const rcr_plan *const *plans, int32_t k, std::shared_ptr<rcr_plan> &out) {
  if (!plans || k < 1) return RCR_NULL_ARG;
  std::vector<uint64_t> key((size_t)k);
  for (int32_t t = 0; t < k; ++t) {
    if (!plans[t]) return RCR_NULL_ARG;
    key[(size_t)t] = plans[t]->obj.serial;
  }
  {
    std::lock_guard<std::mutex> lock(merged_mu);
    for (auto &e : merged_cache())
      if (e.key == key) {
        e.tick = ++merged_tick;
        out = e.plan;
        return RCR_OK;
      }
  }
  std::vector<const rcr::PlanHost *> parts;
  for (int32_t t = 0; t < k; ++t) parts.push_back(&plans[t]->obj.host);
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    rc = rcr::merge_plans(parts, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  std::shared_ptr<rcr_plan> sp(p, destroy_plan);
  std::vector<std::shared_ptr<rcr_plan>> dropped;  // released outside the lock
  {
    std::lock_guard<std::mutex> lock(merged_mu);
    auto &c = merged_cache();
    for (auto &e : c)
      if (e.key == key) {  // built meanwhile by another thread
        e.tick = ++merged_tick;
        out = e.plan;
        dropped.push_back(sp);
        return RCR_OK;
      }
    while (c.size() >= MERGED_CAP) {
      auto victim = std::min_element(c.begin(), c.end(),
                                     [](const MergedEntry &a, const MergedEntry &b) { return a.tick < b.tick; });
      dropped.push_back(victim->plan);
      c.erase(victim);
    }
    c.push_back(MergedEntry{key, sp, ++merged_tick});
  }
  out = sp;
  return RCR_OK;
}

// Drop the cached merged plans that hold the plan with this serial id.
void forget_part(uint64_t serial) {
  std::vector<std::shared_ptr<rcr_plan>> dropped;
  {
    std::lock_guard<std::mutex> lock(merged_mu);
    auto &c = merged_cache();
    for (size_t i = 0; i < c.size();) {
      if (std::find(c[i].key.begin(), c[i].key.end(), serial) != c[i].key.end()) {
        dropped.push_back(c[i].plan);
        c.erase(c.begin() + (long)i);
      } else {
        ++i;
      }
    }
  }
}

void destroy_plan(rcr_plan *p) {
  if (!p) return;
  forget_part(p->obj.serial);
  rcr::plan_release_device(p->obj);
  delete p;
}

int has_device() {
  int ndev = 0;
  return hipGetDeviceCount(&ndev) == hipSuccess && ndev >= 1;
}

// Options with defaults filled in, or RCR_BAD_OPTION.
int read_options(const rcr_solve_options *opt, rcr_solve_options &o) {
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.precision != RCR_FP64 && o.precision != RCR_MIXED32) return RCR_BAD_OPTION;
  if (o.executor != RCR_EXEC_LEVELS && o.executor != RCR_EXEC_GRAPH) return RCR_BAD_OPTION;
  if (o.refine_steps < 0) o.refine_steps = 1;
  return RCR_OK;
}
}  // namespace

extern "C" {

int rcr_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m, const rcr_plan_options *opt,
                    rcr_plan **out) {
  if (!parent || !out) return RCR_NULL_ARG;
  *out = nullptr;
  int selection = opt ? opt->selection : RCR_SELECT_GREEDY_INDEX;
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    CallerOnly only(opt);
    rc = rcr::build_plan(parent, N, n, m, selection, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return RCR_OK;
}

int rcr_plan_create_device(const int64_t *parent, int64_t N, int32_t n, int32_t m, const rcr_plan_options *opt,
                           void *stream, rcr_plan **out) {
  if (!parent || !out) return RCR_NULL_ARG;
  *out = nullptr;
  if (opt && opt->selection != RCR_SELECT_LIST_RANK) return RCR_BAD_OPTION;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    rc = rcr::device_plan(parent, N, n, m, (hipStream_t)stream, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return RCR_OK;
}

int rcr_plan_digest(const rcr_plan *plan, uint64_t *digest) {
  if (!plan || !digest) return RCR_NULL_ARG;
  const rcr::PlanHost &h = plan->obj.host;
  uint64_t x = 1469598103934665603ull;
  auto bytes = [&x](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
      x ^= c[i];
      x *= 1099511628211ull;
    }
  };
  auto word = [&](int64_t v) { bytes(&v, sizeof v); };
  auto vec = [&](const auto &v) {
    word((int64_t)v.size());
    if (!v.empty()) bytes(v.data(), v.size() * sizeof(v[0]));
  };
  for (int64_t v : {h.N, (int64_t)h.n, (int64_t)h.m, h.root, (int64_t)h.selection, h.height, h.leaves, h.max_degree,
                    h.rounds, h.n_rake, h.n_compress, h.n_combine, h.n_absorb, h.n_contrib, h.n_edge_slots, h.lift_N,
                    (int64_t)h.lift_n})
    word(v);
  vec(h.ops);
  vec(h.lvl_off);
  vec(h.kind_off);
  vec(h.exp_ops);
  vec(h.exp_off);
  vec(h.tc_ops);
  vec(h.tc_off);
  vec(h.sx_ops);
  vec(h.sx_off);
  vec(h.parent32);
  vec(h.tree_off);
  vec(h.lift_plus);
  vec(h.rg_n);
  vec(h.rg_m);
  vec(h.rg_off);
  *digest = x;
  return RCR_OK;
}

int rcr_lift_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m, const rcr_plan_options *opt,
                         rcr_plan **out) {
  if (!parent || !out) return RCR_NULL_ARG;
  *out = nullptr;
  int selection = opt ? opt->selection : RCR_SELECT_GREEDY_INDEX;
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    CallerOnly only(opt);
    rc = rcr::build_lift_plan(parent, N, n, m, selection, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return RCR_OK;
}

int rcr_lift_solve(const rcr_plan *plan, const rcr_native_problem *in, rcr_native_solution *out,
                   const rcr_solve_options *opt, void *stream) {
  if (!plan || !in || !out) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->q, in->c, in->Delta, in->M, in->R, in->r, in->A, in->B,
                          out->x, out->v, out->lam};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!plan->obj.host.lift_N) return RCR_BAD_OPTION;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::lift_solve(pl->obj, *in, *out, o, (hipStream_t)stream);
}

int rcr_ragged_plan_create(const int64_t *parent, int64_t N, const int32_t *n_node, const int32_t *m_edge,
                           const rcr_plan_options *opt, rcr_plan **out) {
  if (!parent || !n_node || !m_edge || !out) return RCR_NULL_ARG;
  *out = nullptr;
  int selection = opt ? opt->selection : RCR_SELECT_GREEDY_INDEX;
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    CallerOnly only(opt);
    rc = rcr::build_ragged_plan(parent, N, n_node, m_edge, selection, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return RCR_OK;
}

int rcr_ragged_offsets(const rcr_plan *plan, int64_t *offsets) {
  if (!plan || !offsets) return RCR_NULL_ARG;
  const rcr::PlanHost &h = plan->obj.host;
  if (h.rg_off.empty()) return RCR_BAD_OPTION;
  memcpy(offsets, h.rg_off.data(), h.rg_off.size() * sizeof(int64_t));
  return RCR_OK;
}

int rcr_ragged_solve(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                     void *stream) {
  if (!plan || !in || !out) return RCR_NULL_ARG;
  const rcr::PlanHost &h = plan->obj.host;
  if (h.rg_n.empty()) return RCR_BAD_OPTION;
  const double *need[] = {in->Q, in->q, in->c, in->Delta, in->R, in->S, in->r, in->A, in->B,
                          out->K, out->P, out->x, out->u, out->lam};
  for (int f = 0; f < rcr::RG_FIELDS; ++f)  // an empty field (a one-node tree's edge arrays) may be NULL
    if (!need[f] && h.rg_off[(size_t)(f * (h.N + 1) + h.N)] > 0) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::ragged_solve(pl->obj, *in, *out, o, (hipStream_t)stream);
}

int rcr_batch_plan_create(const rcr_plan *const *plans, int32_t k, rcr_plan **out) {
  if (!plans || !out || k < 1) return RCR_NULL_ARG;
  *out = nullptr;
  std::vector<const rcr::PlanHost *> parts;
  for (int32_t t = 0; t < k; ++t) {
    if (!plans[t]) return RCR_NULL_ARG;
    parts.push_back(&plans[t]->obj.host);
  }
  rcr_plan *p = new_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
    rc = rcr::merge_plans(parts, p->obj.host);
  } catch (const std::bad_alloc &) {
    rc = RCR_OOM;
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return RCR_OK;
}

int rcr_plan_upload(const rcr_plan *plan, void *stream) {
  if (!plan) return RCR_NULL_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  std::lock_guard<std::mutex> lock(pl->obj.mu);
  return rcr::plan_upload(pl->obj, (hipStream_t)stream);
}

int rcr_plan_set_launch(rcr_plan *plan, const rcr_launch_config *cfg) {
  if (!plan) return RCR_NULL_ARG;
  rcr::LaunchCfg c;
  if (cfg) {
    if (cfg->vec_tail_waves < 0 || cfg->vec_tail_waves > 16) return RCR_BAD_OPTION;
    c.quad_tail_rounds = cfg->quad_tail_rounds;
    c.vec_tail_rounds = cfg->vec_tail_rounds;
    c.vec_tail_waves = cfg->vec_tail_waves;
  }
  std::lock_guard<std::mutex> lock(plan->obj.mu);
  plan->obj.cfg = c;
  rcr::drop_graphs(plan->obj);
  return RCR_OK;
}

int rcr_plan_get_launch(const rcr_plan *plan, rcr_launch_config *cfg) {
  if (!plan || !cfg) return RCR_NULL_ARG;
  memset(cfg, 0, sizeof(*cfg));
  cfg->quad_tail_rounds = plan->obj.cfg.quad_tail_rounds;
  cfg->vec_tail_rounds = plan->obj.cfg.vec_tail_rounds;
  cfg->vec_tail_waves = plan->obj.cfg.vec_tail_waves;
  return RCR_OK;
}

int rcr_plan_tune(rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                  void *stream, rcr_launch_config *best, float *best_ms) {
  if (!plan || !in || !out || !best) return RCR_NULL_ARG;
  rcr_solve_options o;
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.precision != RCR_FP64 && o.precision != RCR_MIXED32) return RCR_BAD_OPTION;
  if (o.refine_steps < 0) o.refine_steps = 1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RCR_NO_DEVICE;
  rcr::LaunchCfg b;
  float ms = 0.f;
  const int rc = rcr::tune(plan->obj, *in, *out, o, (hipStream_t)stream, b, ms);
  if (rc) return rc;
  memset(best, 0, sizeof(*best));
  best->quad_tail_rounds = b.quad_tail_rounds;
  best->vec_tail_rounds = b.vec_tail_rounds;
  best->vec_tail_waves = b.vec_tail_waves;
  if (best_ms) *best_ms = ms;
  return RCR_OK;
}

int rcr_plan_info(const rcr_plan *plan, rcr_plan_stats *out) {
  if (!plan || !out) return RCR_NULL_ARG;
  const rcr::PlanHost &h = plan->obj.host;
  memset(out, 0, sizeof(*out));
  out->N = h.N;
  out->n = h.n;
  out->m = h.m;
  out->root = h.root;
  out->height = h.height;
  out->leaves = h.leaves;
  out->max_degree = h.max_degree;
  out->rounds = h.rounds;
  out->levels = h.levels();
  out->expand_levels = h.expand_levels();
  out->state_levels = h.state_levels();
  out->sexp_levels = h.sexp_levels();
  out->n_rake = h.n_rake;
  out->n_compress = h.n_compress;
  out->n_combine = h.n_combine;
  out->n_absorb = h.n_absorb;
  out->depth_bound = rcr::depth_bound(h.N);
  {  // checked once per plan, on the first request (kept off plan creation)
    std::lock_guard<std::mutex> lock(const_cast<rcr::PlanObj &>(plan->obj).mu);
    if (h.crew < 0) h.crew = rcr::verify_crew(h) ? 1 : 0;
    out->crew_ok = h.crew;
  }
  out->workspace_bytes_fp64 = (int64_t)rcr::total_workspace_bytes(h, RCR_FP64);
  out->workspace_bytes_mixed = (int64_t)rcr::total_workspace_bytes(h, RCR_MIXED32);
  out->n_trees = h.tree_off.empty() ? 1 : (int64_t)h.tree_off.size() - 1;
  out->plan_device_bytes = (int64_t)rcr::plan_device_bytes(h);
  {
    std::lock_guard<std::mutex> lock(const_cast<rcr::PlanObj &>(plan->obj).mu);
    out->graph_cache_entries = (int64_t)rcr::graph_cache_size(plan->obj);
  }
  return RCR_OK;
}

int64_t rcr_plan_device_bytes(const rcr_plan *plan) {
  return plan ? (int64_t)rcr::plan_device_bytes(plan->obj.host) : 0;
}

int rcr_plan_export(const rcr_plan *plan, int32_t *ops, int64_t capacity, int64_t *count) {
  if (!plan || !count) return RCR_NULL_ARG;
  const rcr::PlanHost &h = plan->obj.host;
  *count = (int64_t)h.ops.size();
  if (!ops) return RCR_OK;
  if (capacity < *count) return RCR_SMALL_WORKSPACE;
  memcpy(ops, h.ops.data(), h.ops.size() * sizeof(rcr::OpRec));
  return RCR_OK;
}

void rcr_plan_destroy(rcr_plan *plan) { destroy_plan(plan); }

int64_t rcr_workspace_size(const rcr_plan *plan, int32_t precision) {
  if (!plan || (precision != RCR_FP64 && precision != RCR_MIXED32)) return 0;
  return (int64_t)rcr::total_workspace_bytes(plan->obj.host, precision);
}

int rcr_solve(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
              void *stream) {
  if (!plan || !in || !out) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->q, in->c, in->Delta, in->R, in->S, in->r, in->A, in->B,
                          out->K, out->P, out->x, out->u, out->lam};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::solve(pl->obj, *in, *out, o, (hipStream_t)stream);
}

int rcr_factor(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
               void *stream) {
  if (!plan || !in || !out) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->Delta, in->R, in->S, in->A, in->B, out->K, out->P};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::factor(pl->obj, *in, out->K, out->P, o, (hipStream_t)stream);
}

int rcr_solve_rhs(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *factor, int32_t k,
                  const rcr_rhs *rhs, rcr_rhs_solution *sol, const rcr_solve_options *opt, void *stream) {
  if (!plan || !in || !factor || !rhs || !sol) return RCR_NULL_ARG;
  if (k < 1) return RCR_BAD_OPTION;
  const double *need[] = {in->Q, in->Delta, in->R, in->S, in->A, in->B, factor->K, factor->P};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  std::vector<rcr::RhsIO> ios((size_t)k);
  for (int32_t i = 0; i < k; ++i) {
    if (!rhs[i].q || !rhs[i].r || !rhs[i].c || !sol[i].x || !sol[i].u || !sol[i].lam) return RCR_NULL_ARG;
    ios[(size_t)i] = rcr::RhsIO{rhs[i].q, rhs[i].r, rhs[i].c, sol[i].x, sol[i].u, sol[i].lam};
  }
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::solve_rhs(pl->obj, *in, factor->K, factor->P, k, ios.data(), o, (hipStream_t)stream);
}

int rcr_adjoint(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *fwd, const rcr_rhs *seed,
                rcr_gradient *grad, const rcr_solve_options *opt, void *stream) {
  if (!plan || !in || !fwd || !seed || !grad) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->Delta, in->R, in->S, in->A, in->B, fwd->K, fwd->P, fwd->x, fwd->u, fwd->lam,
                          seed->q, seed->r, seed->c, grad->q, grad->r, grad->c};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::adjoint(pl->obj, *in, *fwd, seed->q, seed->r, seed->c, *grad, o, (hipStream_t)stream);
}

int rcr_kkt_residual(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *sol,
                     const rcr_solve_options *opt, void *stream) {
  if (!plan || !in || !sol || !opt || !opt->kkt_residual) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->q, in->c, in->Delta, in->R, in->S, in->r, in->A, in->B,
                          sol->x, sol->u, sol->lam};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::kkt_residual(pl->obj, *in, *sol, *opt, (hipStream_t)stream);
}

int rcr_batch_solve(const rcr_plan *const *plans, int32_t k, const rcr_problem *in, rcr_solution *out,
                    const rcr_solve_options *opt, void *stream) {
  if (!plans || !in || !out || k < 1) return RCR_NULL_ARG;
  for (int32_t t = 0; t < k; ++t) {
    const double *need[] = {in[t].Q, in[t].q, in[t].c, in[t].Delta, in[t].R, in[t].S, in[t].r, in[t].A, in[t].B,
                            out[t].K, out[t].P, out[t].x, out[t].u, out[t].lam};
    for (const double *p : need)
      if (!p) return RCR_NULL_ARG;
  }
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  std::shared_ptr<rcr_plan> B;
  if ((rc = merged_plan(plans, k, B))) return rc;
  return rcr::batch_solve(B->obj, k, in, out, o, (hipStream_t)stream);
}

int rcr_batch_prepare(const rcr_plan *const *plans, int32_t k, void *stream) {
  std::shared_ptr<rcr_plan> B;
  int rc = merged_plan(plans, k, B);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  std::lock_guard<std::mutex> lock(B->obj.mu);
  return rcr::plan_upload(B->obj, (hipStream_t)stream);
}

void rcr_batch_release(const rcr_plan *const *plans, int32_t k) {
  if (!plans || k < 1) return;
  std::vector<uint64_t> key((size_t)k);
  for (int32_t t = 0; t < k; ++t) {
    if (!plans[t]) return;
    key[(size_t)t] = plans[t]->obj.serial;
  }
  std::shared_ptr<rcr_plan> dropped;  // released outside the lock
  std::lock_guard<std::mutex> lock(merged_mu);
  auto &c = merged_cache();
  for (size_t i = 0; i < c.size(); ++i)
    if (c[i].key == key) {
      dropped = c[i].plan;
      c.erase(c.begin() + (long)i);
      break;
    }
}

int64_t rcr_batch_workspace_size(const rcr_plan *const *plans, int32_t k, int32_t precision) {
  if (precision != RCR_FP64 && precision != RCR_MIXED32) return 0;
  std::shared_ptr<rcr_plan> B;
  if (merged_plan(plans, k, B)) return 0;
  return (int64_t)rcr::batch_workspace_bytes(B->obj.host, precision);
}

int rcr_solve_noalloc(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                      void *stream) {
  if (!plan || !in || !out) return RCR_NULL_ARG;
  const double *need[] = {in->Q, in->q, in->c, in->Delta, in->R, in->S, in->r, in->A, in->B,
                          out->K, out->P, out->x, out->u, out->lam};
  for (const double *p : need)
    if (!p) return RCR_NULL_ARG;
  rcr_solve_options o;
  int rc = read_options(opt, o);
  if (rc) return rc;
  if (!has_device()) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::solve_noalloc(pl->obj, *in, *out, o, (hipStream_t)stream);
}

int64_t rcr_noalloc_scratch_bytes(void) { return (int64_t)rcr::noalloc_scratch_bytes(); }

const char *rcr_status_string(int s) {
  switch (s) {
    case RCR_OK: return "ok";
    case RCR_INVALID_TREE: return "invalid tree (no root, several roots, a cycle, or an index out of range)";
    case RCR_BAD_DIMS: return "bad dimensions";
    case RCR_NULL_ARG: return "null argument";
    case RCR_NOT_PD: return "Cholesky breakdown (R_e or G_e not positive definite)";
    case RCR_SINGULAR: return "zero pivot in a nonsymmetric local solve";
    case RCR_NONFINITE: return "non-finite value in the output";
    case RCR_OOM: return "out of memory";
    case RCR_HIP_ERROR: return "HIP runtime error";
    case RCR_BAD_OPTION: return "option out of range";
    case RCR_SMALL_WORKSPACE: return "workspace or buffer too small";
    case RCR_NO_DEVICE: return "no usable GPU";
    default: return "unknown status";
  }
}

}  // extern "C"
