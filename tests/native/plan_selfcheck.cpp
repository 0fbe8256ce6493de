// Host planner self-check, built with g++ by tests/test_planner_native.py
// (plain, then under AddressSanitizer and ThreadSanitizer).
//
// 1. Plans of several tree families and both selections, built on four
//    threads at once (the planner keeps per-thread working arrays and builds
//    large plans' pass schedules on four threads of its own), each passing the
//    independent CREW check of every pass schedule, and equal to the same plan
//    built alone on the main thread.
// 2. A merged (batched) plan passes the check.
// 3. Each pass schedule corrupted in one place fails the check.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "../../include/rcr.h"
#include "../../paper_2608_01332_amd/csrc/plan.hpp"

using namespace rcr;

static std::vector<int64_t> chainprob(int64_t N, double p, uint64_t seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<int64_t> par((size_t)N, -1);
  for (int64_t i = 1; i < N; ++i) par[(size_t)i] = u(g) < p ? i - 1 : (int64_t)(u(g) * (double)i);
  return par;
}
static std::vector<int64_t> star(int64_t N) {
  std::vector<int64_t> par((size_t)N, 0);
  par[0] = -1;
  return par;
}
static std::vector<int64_t> balanced(int64_t N) {
  std::vector<int64_t> par((size_t)N, -1);
  for (int64_t i = 1; i < N; ++i) par[(size_t)i] = (i - 1) / 2;
  return par;
}
static std::vector<int64_t> caterpillar(int64_t trunk, int legs) {
  std::vector<int64_t> par;
  for (int64_t t = 0; t < trunk; ++t) par.push_back(t == 0 ? -1 : t - 1);
  for (int64_t t = 0; t < trunk; ++t)
    for (int l = 0; l < legs; ++l) par.push_back(t);
  return par;
}

static bool same(const PlanHost &a, const PlanHost &b) {
  auto eq = [](const auto &x, const auto &y) {
    if (x.size() != y.size()) return false;
    for (size_t i = 0; i < x.size(); ++i)
      if (memcmp(&x[i], &y[i], sizeof(x[i])) != 0) return false;
    return true;
  };
  return eq(a.ops, b.ops) && eq(a.lvl_off, b.lvl_off) && eq(a.exp_ops, b.exp_ops) && eq(a.tc_ops, b.tc_ops) &&
         eq(a.sx_ops, b.sx_ops) && eq(a.exp_off, b.exp_off) && eq(a.tc_off, b.tc_off) && eq(a.sx_off, b.sx_off);
}

#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");              \
      return 1;                           \
    }                                     \
  } while (0)

int main() {
  std::vector<std::vector<int64_t>> trees = {chainprob(40000, 0.95, 1), chainprob(3000, 0.5, 2), star(2000),
                                             balanced(4095), caterpillar(3000, 3), chainprob(70000, 0.9, 3)};
  const int T = (int)trees.size();
  // 1. concurrent builds
  std::vector<PlanHost> conc((size_t)(2 * T));
  std::vector<int> rcs((size_t)(2 * T), -1);
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      for (int k = w; k < 2 * T; k += 4)
        rcs[(size_t)k] = build_plan(trees[(size_t)(k / 2)].data(), (int64_t)trees[(size_t)(k / 2)].size(), 6, 2,
                                    k % 2, conc[(size_t)k]);
    });
  for (auto &t : th) t.join();
  for (int k = 0; k < 2 * T; ++k) {
    CHECK(rcs[(size_t)k] == 0, "build %d", k);
    CHECK(verify_crew(conc[(size_t)k]), "crew %d", k);
    PlanHost alone;
    CHECK(build_plan(trees[(size_t)(k / 2)].data(), (int64_t)trees[(size_t)(k / 2)].size(), 6, 2, k % 2, alone) == 0,
          "alone %d", k);
    CHECK(same(alone, conc[(size_t)k]), "plan %d differs between threads", k);
  }
  // 2. merged plan
  {
    std::vector<const PlanHost *> parts;
    for (int k = 0; k < 2 * T; k += 2) parts.push_back(&conc[(size_t)k]);
    PlanHost merged;
    CHECK(merge_plans(parts, merged) == 0, "merge");
    CHECK(verify_crew(merged), "crew of the merged plan");
  }
  // 3. corruptions, each caught
  const PlanHost &base = conc[0];
  CHECK(base.n_compress > 0 && base.expand_levels() > 1 && base.state_levels() > 1 && base.sexp_levels() > 1,
        "the test plan needs every schedule");
  {  // an expansion whose child is expanded later moved to the first level
    PlanHost p = base;
    const int64_t last = p.exp_off[p.expand_levels() - 1];
    std::swap(p.exp_ops[0], p.exp_ops[(size_t)last]);
    CHECK(!verify_crew(p), "expansion order corruption not caught");
  }
  {  // a composition reading a slot composed at the same level
    PlanHost p = base;
    const int64_t i = p.tc_off[1];  // first op of composition level 2 ...
    p.tc_ops[0].a = p.tc_ops[(size_t)i].c;  // ... read by level 1
    CHECK(!verify_crew(p), "composition corruption not caught");
  }
  {  // a state expansion from a parent expanded later
    PlanHost p = base;
    const int64_t last = p.sx_off[p.sexp_levels() - 1];
    std::swap(p.sx_ops[0], p.sx_ops[(size_t)last]);
    CHECK(!verify_crew(p), "state expansion corruption not caught");
  }
  {  // a contraction op writing the slot another op of its level writes
    PlanHost p = base;
    int64_t a = -1, b = -1;
    for (int64_t k = p.lvl_off[0]; k < p.lvl_off[1]; ++k)
      if (p.ops[(size_t)k].kind == OP_COMPRESS) {
        if (a < 0) a = k;
        else if (b < 0) b = k;
      }
    CHECK(a >= 0 && b >= 0, "two level-1 compressions");
    p.ops[(size_t)b].d = p.ops[(size_t)a].d;
    CHECK(!verify_crew(p), "contraction corruption not caught");
  }
  printf("plan self-check OK (%d plans)\n", 2 * T);
  return 0;
}
