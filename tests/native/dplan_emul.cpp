// The device planner's program (dplan.hpp) run on the CPU by its sequential
// executor, checked against the host planner (build_plan, list-rank
// selection): every statistic and every schedule must be identical, for
// thread counts 1024 (the GPU's) and others, for three orders of the
// threads inside each phase (a phase whose result depended on that order would
// race on the GPU), and with sibling groups built by one thread or by the
// whole workgroup.  Invalid trees must be rejected with the host's status.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2608_01332_amd/csrc/dplan.hpp"

using namespace rcr;

static int failures = 0;
#define CHECK(cond, what)                                           \
  do {                                                              \
    if (!(cond)) {                                                  \
      fprintf(stderr, "FAIL %s: %s\n", name.c_str(), what);         \
      ++failures;                                                   \
      return;                                                       \
    }                                                               \
  } while (0)

template <class V>
static bool same(const V &a, const V &b) {
  return a.size() == b.size() && (a.empty() || memcmp(a.data(), b.data(), a.size() * sizeof(a[0])) == 0);
}

static void compare(const std::string &name, const std::vector<int64_t> &parent) {
  PlanHost host;
  const int64_t N = (int64_t)parent.size();
  const int rh = build_plan(parent.data(), N, 6, 2, RCR_SELECT_LIST_RANK, host);
  const int Ts[] = {dplan::THREADS, 37, 1};
  // every group through the one-thread build (above the largest group), then
  // every group of two or more through the workgroup-wide build, then the
  // default threshold
  const int32_t bigs[] = {INT32_MAX, 1, dplan::BIG_GROUP};
  for (int32_t big : bigs)
  for (int T : Ts)
    for (int order = 0; order < 3; ++order) {
      if (T == 1 && order) continue;
      PlanHost dev;
      const int rd = dplan::emulate(parent.data(), N, 6, 2, T, order, dev, big);
      CHECK(rd == rh, "status");
      if (rh) continue;
      CHECK(dev.root == host.root && dev.height == host.height && dev.leaves == host.leaves &&
                dev.max_degree == host.max_degree,
            "tree statistics");
      CHECK(dev.rounds == host.rounds && dev.n_rake == host.n_rake && dev.n_compress == host.n_compress &&
                dev.n_combine == host.n_combine && dev.n_absorb == host.n_absorb && dev.n_contrib == host.n_contrib &&
                dev.n_edge_slots == host.n_edge_slots,
            "round statistics");
      CHECK(dev.selection == host.selection && dev.N == host.N && dev.n == host.n && dev.m == host.m, "header");
      CHECK(same(dev.parent32, host.parent32), "parent32");
      CHECK(same(dev.ops, host.ops), "contraction ops");
      CHECK(same(dev.lvl_off, host.lvl_off) && same(dev.kind_off, host.kind_off), "contraction offsets");
      CHECK(same(dev.exp_ops, host.exp_ops) && same(dev.exp_off, host.exp_off), "expansion schedule");
      CHECK(same(dev.tc_ops, host.tc_ops) && same(dev.tc_off, host.tc_off), "composition schedule");
      CHECK(same(dev.sx_ops, host.sx_ops) && same(dev.sx_off, host.sx_off), "state schedule");
    }
}

static std::vector<int64_t> chainprob(int64_t N, double p, std::mt19937_64 &g) {
  std::vector<int64_t> par((size_t)N);
  par[0] = -1;
  std::uniform_real_distribution<double> u(0, 1);
  for (int64_t i = 1; i < N; ++i) par[(size_t)i] = u(g) < p ? i - 1 : (int64_t)(g() % (uint64_t)i);
  return par;
}

// the same tree under a random relabelling (parents no longer precede children)
static std::vector<int64_t> permuted(const std::vector<int64_t> &par, std::mt19937_64 &g) {
  const size_t N = par.size();
  std::vector<int64_t> perm(N), out(N);
  for (size_t i = 0; i < N; ++i) perm[i] = (int64_t)i;
  std::shuffle(perm.begin(), perm.end(), g);
  for (size_t i = 0; i < N; ++i) out[(size_t)perm[i]] = par[i] < 0 ? -1 : perm[(size_t)par[i]];
  return out;
}

int main() {
  std::mt19937_64 g(20260001);
  std::vector<std::pair<std::string, std::vector<int64_t>>> cases;
  cases.push_back({"single", {-1}});
  cases.push_back({"pair", {-1, 0}});
  cases.push_back({"pair-rev", {1, -1}});
  cases.push_back({"cherry", {-1, 0, 0}});
  {
    std::vector<int64_t> chain(3000);
    for (int64_t i = 0; i < 3000; ++i) chain[(size_t)i] = i - 1;
    cases.push_back({"chain3000", chain});
  }
  {
    std::vector<int64_t> star(5000, 0);
    star[0] = -1;
    cases.push_back({"star5000", star});
  }
  {
    std::vector<int64_t> bal(4095);
    bal[0] = -1;
    for (int64_t i = 1; i < 4095; ++i) bal[(size_t)i] = (i - 1) / 2;
    cases.push_back({"balanced4095", bal});
  }
  {  // caterpillar: a spine with two leaves per spine node
    std::vector<int64_t> cat;
    cat.push_back(-1);
    int64_t prev = 0;
    for (int s = 1; s < 2000; ++s) {
      const int64_t v = (int64_t)cat.size();
      cat.push_back(prev);
      cat.push_back(v);
      cat.push_back(v);
      prev = v;
    }
    cases.push_back({"caterpillar", cat});
  }
  {  // comb: spine with a chain of 5 hanging off each spine node
    std::vector<int64_t> comb;
    comb.push_back(-1);
    int64_t prev = 0;
    for (int s = 1; s < 400; ++s) {
      const int64_t v = (int64_t)comb.size();
      comb.push_back(prev);
      int64_t t = v;
      for (int k = 0; k < 5; ++k) {
        comb.push_back(t);
        t = (int64_t)comb.size() - 1;
      }
      prev = v;
    }
    cases.push_back({"comb", comb});
  }
  {  // hubs: a root with 3000 children, some of them with their own chains and stars
    std::vector<int64_t> hub(1, -1);
    for (int k = 0; k < 3000; ++k) hub.push_back(0);
    for (int k = 0; k < 2000; ++k) hub.push_back(1 + (int64_t)(g() % 3000));
    for (int k = 0; k < 2000; ++k) hub.push_back((int64_t)hub.size() - 1);
    cases.push_back({"hubs", hub});
  }
  {  // a root with 700 chains of random lengths: large root groups of mixed levels, round after round
    std::vector<int64_t> sc(1, -1);
    for (int c = 0; c < 700; ++c) {
      int64_t prev = 0;
      const int len = 1 + (int)(g() % 40);
      for (int l = 0; l < len; ++l) {
        sc.push_back(prev);
        prev = (int64_t)sc.size() - 1;
      }
    }
    cases.push_back({"star_of_chains", sc});
  }
  {  // a root with 200 children of 200 leaves each
    std::vector<int64_t> tl(1, -1);
    for (int c = 0; c < 200; ++c) {
      const int64_t v = (int64_t)tl.size();
      tl.push_back(0);
      for (int l = 0; l < 200; ++l) tl.push_back(v);
    }
    cases.push_back({"two_level_hubs", tl});
  }
  for (double p : {0.5, 0.8, 0.9, 0.95, 0.99}) {
    for (int64_t N : {100, 2500, 20000}) {
      auto t = chainprob(N, p, g);
      cases.push_back({"chainprob" + std::to_string(N) + "_" + std::to_string(p), t});
      if (N <= 2500) cases.push_back({"permuted" + std::to_string(N) + "_" + std::to_string(p), permuted(t, g)});
    }
  }
  cases.push_back({"chainprob65536_0.95", chainprob(65536, 0.95, g)});
  // invalid trees
  cases.push_back({"two-roots", {-1, 0, -1}});
  cases.push_back({"no-root", {1, 0}});
  cases.push_back({"self-loop", {-1, 1}});
  cases.push_back({"out-of-range", {-1, 7}});
  cases.push_back({"bad-negative", {-1, -2}});
  cases.push_back({"cycle-off-root", {-1, 0, 3, 2}});
  cases.push_back({"long-cycle", {-1, 0, 5, 2, 3, 4}});

  for (auto &c : cases) compare(c.first, c.second);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("device planner emulation OK (%zu trees)\n", cases.size());
  return 0;
}
