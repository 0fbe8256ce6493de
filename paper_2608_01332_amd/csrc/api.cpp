// C-ABI entry points (include/rcr.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rcr.h"
#include "device.hpp"
#include "plan.hpp"

struct rcr_plan {
  rcr::PlanObj obj;
};

extern "C" {

int rcr_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m, const rcr_plan_options *opt,
                    rcr_plan **out) {
  if (!parent || !out) return RCR_NULL_ARG;
  *out = nullptr;
  int selection = opt ? opt->selection : RCR_SELECT_GREEDY_INDEX;
  rcr_plan *p = new (std::nothrow) rcr_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
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

int rcr_lift_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m, const rcr_plan_options *opt,
                         rcr_plan **out) {
  if (!parent || !out) return RCR_NULL_ARG;
  *out = nullptr;
  int selection = opt ? opt->selection : RCR_SELECT_GREEDY_INDEX;
  rcr_plan *p = new (std::nothrow) rcr_plan();
  if (!p) return RCR_OOM;
  int rc;
  try {
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
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.precision != RCR_FP64 && o.precision != RCR_MIXED32) return RCR_BAD_OPTION;
  if (o.executor != RCR_EXEC_LEVELS && o.executor != RCR_EXEC_GRAPH) return RCR_BAD_OPTION;
  if (o.refine_steps < 0) o.refine_steps = 1;
  if (!plan->obj.host.lift_N) return RCR_BAD_OPTION;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::lift_solve(pl->obj, *in, *out, o, (hipStream_t)stream);
}

int rcr_batch_plan_create(const rcr_plan *const *plans, int32_t k, rcr_plan **out) {
  if (!plans || !out || k < 1) return RCR_NULL_ARG;
  *out = nullptr;
  std::vector<const rcr::PlanHost *> parts;
  for (int32_t t = 0; t < k; ++t) {
    if (!plans[t]) return RCR_NULL_ARG;
    parts.push_back(&plans[t]->obj.host);
  }
  rcr_plan *p = new (std::nothrow) rcr_plan();
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
  return RCR_OK;
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

void rcr_plan_destroy(rcr_plan *plan) {
  if (!plan) return;
  rcr::plan_release_device(plan->obj);
  delete plan;
}

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
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.precision != RCR_FP64 && o.precision != RCR_MIXED32) return RCR_BAD_OPTION;
  if (o.executor != RCR_EXEC_LEVELS && o.executor != RCR_EXEC_GRAPH) return RCR_BAD_OPTION;
  if (o.refine_steps < 0) o.refine_steps = 1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RCR_NO_DEVICE;
  rcr_plan *pl = const_cast<rcr_plan *>(plan);
  return rcr::solve(pl->obj, *in, *out, o, (hipStream_t)stream);
}

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
