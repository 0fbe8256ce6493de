// Host planner: structural rounds, readiness-weighted sibling reductions,
// earliest-start dependency levels and static slots (Sec. VII).
//
// Round (Sec. VII-A): rake every non-root leaf; then, in the post-rake tree,
// compress a maximal set of pairwise non-adjacent non-root unary nodes
// (greedy in increasing node id as in the paper, or alternate positions along
// each maximal unary path — any maximal set satisfies Lemma 2).
// Sibling reductions (Lemma 3): the order-preserving binary tree given by the
// alphabetic Shannon-Fano-Elias code on the weights 2^{level}
// (eq. (readiness-code-data)), with unary trie vertices suppressed.
// Levels (eq. (earliest-level)): 1 + the largest producer level of the inputs.
//
// Slots: node data U_i is updated in place at slot i; every compression
// appends a new edge slot (original edge into j is slot j), so an edge record
// is never overwritten and the compress "tape" (A_r, C_r, P_r + U_j) of
// eq. (quadratic-compress) is simply the retained records; rake and combine
// outputs each get their own contribution slot.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <system_error>
#include <thread>
#include <utility>

#include "../../include/rcr.h"

namespace rcr {
namespace {

typedef unsigned __int128 u128;

struct Code {  // alphabetic code word: the leading d bits of r
  u128 r;
  int d;
};

// Working arrays of one plan construction.  Each thread keeps its set between
// plans (up to KEEP_NODES nodes, about 160 bytes per node): a serving loop
// plans many topologies on the same threads, and first-touch page faults of
// fresh arrays would otherwise cost a quarter to a third of a construction.
struct Work {
  std::vector<int32_t> cur_par, lvlU, lvlE, edge_slot, sib_key, cnt, one_child;
  std::vector<uint8_t> alive, sel;
  std::vector<int32_t> contrib_level;
  // removal records
  std::vector<int32_t> rem_slot, rem_par, comp_r, comp_k;
  std::vector<uint8_t> rem_kind;  // 0 none, 1 rake, 2 compress
  std::vector<int32_t> removal_seq;
  std::vector<OpRec> raw;  // forward op sequence before level sorting
  // validation, rounds and the pass schedules
  std::vector<int32_t> deg, bfs_start, bfs_kids, bfs_fill, bfs_order, depth;
  std::vector<int32_t> live, leaves, elig, lvl_e, lvl_t, lvl_x;
  std::vector<std::pair<int64_t, int32_t>> keyed;  // (parent << 32 | sibling key, contribution)
  std::vector<Op4> seq;
  std::vector<int64_t> count, fill, fill_e, fill_t, fill_x;
  // one sibling group of a readiness-weighted reduction
  std::vector<Code> codes;
  std::vector<u128> wts;
  std::vector<int32_t> g_slot, g_lvl;
};
constexpr int64_t KEEP_NODES = int64_t(1) << 17;
// Trees from this size on build their four pass schedules on four threads.
constexpr int64_t PAR_NODES = int64_t(1) << 14;
}  // namespace
thread_local bool build_on_caller_only = false;
namespace {

// Runs the tasks, on threads of their own (the first on the caller's) when
// `parallel` is set and threads can be started, else one after the other.  An
// allocation failure in any task is rethrown on the caller's thread.
template <typename F0, typename... F>
void run_concurrently(bool parallel, F0 &first, F &...rest) {
  if (parallel) {
    constexpr int K = sizeof...(F);
    std::atomic<bool> failed{false};
    std::thread th[K];
    int started = 0;
    auto guarded = [&failed](auto &task) {
      try {
        task();
      } catch (...) {
        failed = true;
      }
    };
    try {
      ((th[started] = std::thread([&guarded, &rest] { guarded(rest); }), ++started), ...);
    } catch (const std::system_error &) {
    }
    guarded(first);
    for (int k = 0; k < started; ++k) th[k].join();
    // tasks that did not get a thread run here
    int k = 0;
    ((k++ >= started ? guarded(rest) : void()), ...);
    if (failed) throw std::bad_alloc();
    return;
  }
  first();
  (rest(), ...);
}

struct Builder : Work {
  const int64_t *parent;
  int64_t N;
  PlanHost &P;
  int32_t next_slot = 0, next_contrib = 0;

  explicit Builder(const int64_t *p, int64_t n, PlanHost &out) : parent(p), N(n), P(out) {}

  int32_t new_contrib(int32_t level) {
    contrib_level.push_back(level);
    return next_contrib++;
  }

  // ---- readiness-weighted reduction (Lemma 3) -----------------------------
  int32_t g_parent = 0, g_round = 0;

  int bit(int j, int pos) const { return (int)((codes[j].r >> (codes[j].d - 1 - pos)) & 1); }

  // returns contribution slot of the aggregate of [lo, hi] and sets *lvl
  int32_t build(int lo, int hi, int depth, int32_t *lvl) {
    for (;;) {
      if (lo == hi) {
        *lvl = g_lvl[lo];
        return g_slot[lo];
      }
      int s = -1;
      for (int j = lo; j <= hi; ++j)
        if (bit(j, depth)) {
          s = j;
          break;
        }
      if (s < 0 || s == lo) {  // unary trie vertex: suppressed
        ++depth;
        continue;
      }
      int32_t la, lb;
      int32_t a = build(lo, s - 1, depth + 1, &la);
      int32_t b = build(s, hi, depth + 1, &lb);
      int32_t lv = 1 + std::max(la, lb);
      int32_t out = new_contrib(lv);
      raw.push_back(OpRec{OP_COMBINE, g_round, lv, a, b, out, g_parent, 0});
      *lvl = lv;
      return out;
    }
  }

  int32_t reduce(int32_t *agg_lvl) {
    const int k = (int)g_slot.size();
    if (k == 1) {
      *agg_lvl = g_lvl[0];
      return g_slot[0];
    }
    // Relative weights w_j = 2^{l_j - l_min}; the code is invariant under a common
    // scale.  Differences are capped so that W < 2^62 and all products fit 128 bits;
    // the cap (>= 40 levels for k <= 2^21 siblings) is never reached by trees of
    // practical size, and reaching it only changes the parenthesisation.
    int32_t lmin = *std::min_element(g_lvl.begin(), g_lvl.end());
    int lg = 0;
    while ((1LL << lg) < k) ++lg;
    int cap = 61 - lg;
    codes.resize(k);
    u128 W = 0;
    std::vector<u128> &w = wts;
    w.resize(k);
    for (int j = 0; j < k; ++j) {
      int e = std::min<int>(g_lvl[j] - lmin, cap);
      w[j] = (u128)1 << e;
      W += w[j];
    }
    u128 S = 0;
    for (int j = 0; j < k; ++j) {
      int d = 0;
      while ((w[j] << d) < W) ++d;  // smallest d with 2^d >= W / w_j
      d += 1;                        // d_j^0 = ceil(log2(W / w_j)) + 1
      u128 num = (2 * S + w[j]) << d;
      codes[j].r = num / (2 * W);    // leading d bits of the midpoint F_j + p_j / 2
      codes[j].d = d;
      S += w[j];
    }
    return build(0, k - 1, 0, agg_lvl);
  }

  int run(int selection) {
    // ---- validation and static statistics
    int64_t root = -1;
    for (int64_t i = 0; i < N; ++i) {
      int64_t p = parent[i];
      if (p < 0) {
        if (p != -1 || root >= 0) return RCR_INVALID_TREE;
        root = i;
      } else if (p >= N || p == i) {
        return RCR_INVALID_TREE;
      }
    }
    if (root < 0) return RCR_INVALID_TREE;
    if (N > (int64_t)(INT32_MAX / 2 - 16)) return RCR_BAD_DIMS;
    P.root = root;
    P.parent32.resize(N);
    deg.assign(N, 0);
    bool topo = root == 0;  // every parent precedes its child
    for (int64_t i = 0; i < N; ++i) {
      P.parent32[i] = (int32_t)parent[i];
      if (parent[i] >= 0) deg[parent[i]]++;
      topo &= parent[i] < i;
    }
    if (topo) {  // parents before children: no cycle, and depths in one forward pass
      depth.resize(N);
      depth[0] = 0;
      int32_t h = 0;
      for (int64_t i = 1; i < N; ++i) {
        depth[i] = depth[parent[i]] + 1;
        h = std::max(h, depth[i]);
      }
      P.height = h;
    } else {  // BFS: reachability (rejects cycles) and height
      std::vector<int32_t> &start = bfs_start, &kids = bfs_kids, &fl = bfs_fill, &order = bfs_order;
      start.resize(N + 1);
      start[0] = 0;
      for (int64_t i = 0; i < N; ++i) start[i + 1] = start[i] + deg[i];
      fl.assign(start.begin(), start.end() - 1);
      kids.resize(N);
      for (int64_t i = 0; i < N; ++i)
        if (parent[i] >= 0) kids[fl[parent[i]]++] = (int32_t)i;
      order.resize(N);
      depth.resize(N);
      int64_t tail = 0;
      order[tail++] = (int32_t)root;
      depth[root] = 0;
      int32_t h = 0;
      // a node is queued once, by its parent: on a cycle the queue stops short of N
      for (int64_t q = 0; q < tail; ++q) {
        const int32_t v = order[q], dv = depth[v] + 1;
        for (int32_t c = start[v]; c < start[v + 1]; ++c) {
          depth[kids[c]] = dv;
          order[tail++] = kids[c];
          h = std::max(h, dv);
        }
      }
      if (tail != N) return RCR_INVALID_TREE;
      P.height = h;
    }
    P.leaves = 0;
    P.max_degree = 0;
    for (int64_t i = 0; i < N; ++i) {
      if (deg[i] == 0) P.leaves++;
      P.max_degree = std::max<int64_t>(P.max_degree, deg[i]);
    }

    // ---- rounds
    cur_par.assign(P.parent32.begin(), P.parent32.end());
    lvlU.assign(N, 0);
    lvlE.assign(N, 0);
    edge_slot.resize(N);
    sib_key.resize(N);
    for (int64_t i = 0; i < N; ++i) edge_slot[i] = sib_key[i] = (int32_t)i;
    one_child.assign(N, -1);
    alive.assign(N, 1);
    sel.assign(N, 0);
    rem_slot.assign(N, -1);
    rem_par.assign(N, -1);
    comp_r.assign(N, -1);
    comp_k.assign(N, -1);
    rem_kind.assign(N, 0);
    next_slot = (int32_t)N;
    raw.clear();
    contrib_level.clear();
    removal_seq.clear();
    raw.reserve((size_t)N * 2);
    contrib_level.reserve((size_t)N * 2);
    removal_seq.reserve((size_t)N);
    live.resize(N);
    for (int64_t i = 0; i < N; ++i) live[i] = (int32_t)i;
    int32_t rnd = 0;
    // cnt[v]: live children of v.  Rakes decrement it; a compression leaves the
    // parent's count unchanged (its child j is replaced by j's child), so it is
    // maintained across rounds instead of recounted.
    cnt.assign(deg.begin(), deg.end());
    while (live.size() > 1) {
      ++rnd;
      leaves.clear();
      for (int32_t v : live)
        if (v != root && cnt[v] == 0) leaves.push_back(v);
      // rakes (every non-root leaf of the tree at the start of the round)
      keyed.clear();
      for (int32_t j : leaves) {
        int32_t lv = 1 + std::max(lvlU[j], lvlE[j]);
        int32_t out = new_contrib(lv);
        raw.push_back(OpRec{OP_RAKE, rnd, lv, j, edge_slot[j], out, cur_par[j], 0});
        rem_kind[j] = 1;
        rem_slot[j] = edge_slot[j];
        rem_par[j] = cur_par[j];
        removal_seq.push_back(j);
        keyed.push_back({(int64_t)cur_par[j] << 32 | (uint32_t)sib_key[j], out});
        P.n_rake++;
      }
      std::sort(keyed.begin(), keyed.end());
      for (size_t g0 = 0; g0 < keyed.size();) {
        int32_t i = (int32_t)(keyed[g0].first >> 32);
        size_t g1 = g0;
        g_slot.clear();
        g_lvl.clear();
        while (g1 < keyed.size() && (int32_t)(keyed[g1].first >> 32) == i) {
          g_slot.push_back(keyed[g1].second);
          g_lvl.push_back(contrib_level[keyed[g1].second]);
          ++g1;
        }
        g_parent = i;
        g_round = rnd;
        int32_t agg_lvl;
        int32_t agg = reduce(&agg_lvl);
        int32_t lv = 1 + std::max(lvlU[i], agg_lvl);
        raw.push_back(OpRec{OP_ABSORB, rnd, lv, i, agg, 0, 0, 0});
        lvlU[i] = lv;
        g0 = g1;
      }
      for (int32_t j : leaves) {
        alive[j] = 0;
        cnt[cur_par[j]]--;
      }
      // unary non-root nodes of the post-rake tree (increasing id) and the
      // single child of every unary node
      elig.clear();
      {
        const int32_t *cp = cur_par.data(), *cn = cnt.data();
        const uint8_t *al = alive.data();
        int32_t *oc = one_child.data();
        for (int32_t v : live) {
          if (!al[v] || v == root) continue;
          if (cn[cp[v]] == 1) oc[cp[v]] = v;
          if (cn[v] == 1) elig.push_back(v);
        }
      }
      if (selection == RCR_SELECT_GREEDY_INDEX) {
        for (int32_t v : elig)
          if (!sel[cur_par[v]] && !sel[one_child[v]]) sel[v] = 1;
      } else {
        // alternate positions along each maximal path of eligible nodes, from its top
        for (int32_t v : elig) sel[v] = 2;  // mark eligible
        for (int32_t v : elig) {
          if (sel[cur_par[v]] == 2 || sel[cur_par[v]] == 1 || sel[cur_par[v]] == 3) continue;  // not a head
          int64_t rank = 0;
          for (int32_t u = v; u >= 0 && (sel[u] == 2); u = one_child[u], ++rank) sel[u] = (rank % 2 == 0) ? 1 : 3;
        }
        for (int32_t v : elig)
          if (sel[v] != 1) sel[v] = 0;
      }
      {  // raw pointers: the byte-array stores below would otherwise force reloads of every vector's base
        int32_t *cp = cur_par.data(), *oc = one_child.data(), *lE = lvlE.data(), *lU = lvlU.data();
        int32_t *es = edge_slot.data(), *rs = rem_slot.data(), *rp = rem_par.data(), *cr = comp_r.data();
        int32_t *ck = comp_k.data(), *sk = sib_key.data();
        uint8_t *se = sel.data(), *rk = rem_kind.data(), *al = alive.data();
        int32_t ns = next_slot;
        int64_t ncomp = 0;
        for (int32_t j : elig) {
          if (se[j] != 1) continue;
          const int32_t i = cp[j], k = oc[j];
          const int32_t lv = 1 + std::max(lE[j], std::max(lU[j], lE[k]));
          const int32_t s = ns++;
          raw.push_back(OpRec{OP_COMPRESS, rnd, lv, j, es[j], es[k], s, k});
          rk[j] = 2;
          rs[j] = es[j];
          rp[j] = i;
          cr[j] = es[k];
          ck[j] = k;
          removal_seq.push_back(j);
          es[k] = s;
          lE[k] = lv;
          cp[k] = i;
          sk[k] = sk[j];
          al[j] = 0;
          ++ncomp;
        }
        next_slot = ns;
        P.n_compress += ncomp;
      }
      for (int32_t j : elig) sel[j] = 0;
      size_t w = 0;
      for (int32_t v : live)
        if (alive[v]) live[w++] = v;
      live.resize(w);
    }
    P.rounds = rnd;
    P.n_contrib = next_contrib;
    P.n_edge_slots = next_slot;
    for (const OpRec &o : raw) {
      if (o.kind == OP_COMBINE) P.n_combine++;
      if (o.kind == OP_ABSORB) P.n_absorb++;
    }

    // The four schedules below read only the round records and write disjoint
    // parts of the plan; for large trees they are built on four threads.
    auto levels_task = [&] {  // contraction levels: sort by (level, kind), stable in creation order
      int32_t L = 0;
      for (const OpRec &o : raw) L = std::max(L, o.level);
      count.assign((size_t)L * 4 + 1, 0);
      for (const OpRec &o : raw) count[(size_t)(o.level - 1) * 4 + o.kind + 1]++;
      for (size_t t = 1; t < count.size(); ++t) count[t] += count[t - 1];
      P.ops.resize(raw.size());
      fill.assign(count.begin(), count.end() - 1);
      for (const OpRec &o : raw) P.ops[fill[(size_t)(o.level - 1) * 4 + o.kind]++] = o;
      P.lvl_off.resize(L + 1);
      for (int32_t t = 0; t <= L; ++t) P.lvl_off[t] = count[(size_t)t * 4];
      P.kind_off.resize((size_t)L * 5);
      for (int32_t t = 0; t < L; ++t)
        for (int s = 0; s <= 4; ++s) P.kind_off[(size_t)t * 5 + s] = count[(size_t)t * 4 + s];
    };
    auto expand_task = [&] {  // expansion of compressions (reverse graph): level = 1 + level of the child's value
      std::vector<int32_t> &eP = lvl_e;
      eP.assign(N, 0);
      int32_t LE = 0;
      for (auto it = removal_seq.rbegin(); it != removal_seq.rend(); ++it) {
        int32_t j = *it;
        if (rem_kind[j] == 2) {
          eP[j] = 1 + eP[comp_k[j]];
          LE = std::max(LE, eP[j]);
        }
      }
      // counting sort by level, stable in removal order
      P.exp_off.assign((size_t)LE + 1, 0);
      for (int32_t j : removal_seq)
        if (rem_kind[j] == 2) P.exp_off[eP[j]]++;
      for (int32_t t = 0; t < LE; ++t) P.exp_off[t + 1] += P.exp_off[t];
      P.exp_ops.resize((size_t)P.exp_off[LE]);
      fill_e.assign(P.exp_off.begin(), P.exp_off.end() - 1);
      for (int32_t j : removal_seq)
        if (rem_kind[j] == 2) P.exp_ops[fill_e[eP[j] - 1]++] = Op4{j, comp_r[j], comp_k[j], 0};
    };
    auto compose_task = [&] {  // composition of edge maps over compressions only
      std::vector<int32_t> &lT = lvl_t;
      lT.assign(next_slot, 0);
      int32_t LT = 0;
      seq.clear();
      for (const OpRec &o : raw)
        if (o.kind == OP_COMPRESS) {
          lT[o.d] = 1 + std::max(lT[o.b], lT[o.c]);
          LT = std::max(LT, lT[o.d]);
          seq.push_back(Op4{o.b, o.c, o.d, o.a});
        }
      P.tc_off.assign((size_t)LT + 1, 0);
      for (const Op4 &q : seq) P.tc_off[lT[q.c]]++;
      for (int32_t t = 0; t < LT; ++t) P.tc_off[t + 1] += P.tc_off[t];
      P.tc_ops.resize((size_t)P.tc_off[LT]);
      fill_t.assign(P.tc_off.begin(), P.tc_off.end() - 1);
      for (const Op4 &q : seq) P.tc_ops[fill_t[lT[q.c] - 1]++] = q;
    };
    auto state_task = [&] {  // state expansion: x_j from the state of its parent at removal time
      std::vector<int32_t> &eX = lvl_x;
      eX.assign(N, 0);
      int32_t LX = 0;
      for (auto it = removal_seq.rbegin(); it != removal_seq.rend(); ++it) {
        int32_t j = *it;
        eX[j] = 1 + eX[rem_par[j]];
        LX = std::max(LX, eX[j]);
      }
      P.sx_off.assign((size_t)LX + 1, 0);
      for (int32_t j : removal_seq) P.sx_off[eX[j]]++;
      for (int32_t t = 0; t < LX; ++t) P.sx_off[t + 1] += P.sx_off[t];
      P.sx_ops.resize((size_t)P.sx_off[LX]);
      fill_x.assign(P.sx_off.begin(), P.sx_off.end() - 1);
      for (int32_t j : removal_seq) P.sx_ops[fill_x[eX[j] - 1]++] = Op4{j, rem_slot[j], rem_par[j], 0};
    };
    run_concurrently(N >= PAR_NODES && !build_on_caller_only, levels_task, expand_task, compose_task, state_task);
    return RCR_OK;
  }

};

}  // namespace

// Independent check of the level schedule: replay the levels in order and
// verify that every input was produced at an earlier level, that each datum
// has at most one writer per level, and that no datum written at a level is
// read by another op of that level.
static bool verify_contraction(const PlanHost &P) {
  const int64_t N = P.N;
  // datum ids: U_i -> i; edge slot s -> N + s; contribution c -> N + slots + c
  const int64_t E0 = N, C0 = N + P.n_edge_slots, ND = C0 + P.n_contrib;
  std::vector<int32_t> produced(ND, -1), wstamp(ND, -1), rstamp(ND, -1);
  for (int64_t i = 0; i < N; ++i) produced[i] = 0;
  for (int64_t s = 0; s < N; ++s) produced[E0 + s] = 0;
  std::vector<int64_t> reads, writes;
  for (int64_t t = 1; t <= P.levels(); ++t) {
    reads.clear();
    writes.clear();
    for (int64_t k = P.lvl_off[t - 1]; k < P.lvl_off[t]; ++k) {
      const OpRec &o = P.ops[k];
      if (o.level != t) return false;
      int64_t in[3];
      int nin = 0;
      int64_t outd = -1;
      switch (o.kind) {
        case OP_RAKE: in[0] = o.a; in[1] = E0 + o.b; nin = 2; outd = C0 + o.c; break;
        case OP_COMBINE: in[0] = C0 + o.a; in[1] = C0 + o.b; nin = 2; outd = C0 + o.c; break;
        case OP_ABSORB: in[0] = o.a; in[1] = C0 + o.b; nin = 2; outd = o.a; break;
        case OP_COMPRESS: in[0] = E0 + o.b; in[1] = o.a; in[2] = E0 + o.c; nin = 3; outd = E0 + o.d; break;
        default: return false;
      }
      for (int q = 0; q < nin; ++q) {
        if (in[q] < 0 || in[q] >= ND) return false;
        if (produced[in[q]] < 0 || produced[in[q]] >= t) return false;
        if (!(o.kind == OP_ABSORB && in[q] == outd)) reads.push_back(in[q]);
      }
      if (outd < 0 || outd >= ND) return false;
      if (wstamp[outd] == t) return false;  // two writers at one level
      wstamp[outd] = (int32_t)t;
      writes.push_back(outd);
    }
    for (int64_t r : reads) rstamp[r] = (int32_t)t;
    for (int64_t w : writes) {
      if (rstamp[w] == t) return false;  // read and written at the same level
      produced[w] = (int32_t)t;
    }
  }
  return true;
}

// Expansion of compressions: P_j from the tape of its out-edge slot r (final
// after the contraction), U_j (final) and P_k of its child k, which is a raked
// node (P_k written by the rake) or a compressed node expanded at a lower
// level.  Every compressed node is expanded exactly once.
static bool verify_expansion(const PlanHost &P) {
  const int64_t N = P.N;
  std::vector<char> compressed((size_t)N, 0), raked((size_t)N, 0);
  for (const OpRec &o : P.ops) {
    if (o.kind == OP_COMPRESS) compressed[(size_t)o.a] = 1;
    if (o.kind == OP_RAKE) raked[(size_t)o.a] = 1;
  }
  std::vector<int32_t> done((size_t)N, -1);  // expansion level that wrote P_j
  int64_t count = 0;
  for (int64_t e = 0; e < P.expand_levels(); ++e)
    for (int64_t i = P.exp_off[e]; i < P.exp_off[e + 1]; ++i) {
      const Op4 &q = P.exp_ops[(size_t)i];
      if (q.a < 0 || q.a >= N || q.c < 0 || q.c >= N || q.b < 0 || q.b >= P.n_edge_slots) return false;
      if (!compressed[(size_t)q.a] || done[(size_t)q.a] >= 0) return false;
      const bool child_ready = raked[(size_t)q.c] || (compressed[(size_t)q.c] && done[(size_t)q.c] >= 0 &&
                                                      done[(size_t)q.c] < e);
      if (!child_ready) return false;
      done[(size_t)q.a] = (int32_t)e;
      ++count;
    }
  return count == P.n_compress;
}

// Composition of edge maps over compressions (composite transitions, and the
// same schedule for the state offsets): the new slot from slots l and r, each
// original (ready before the first level) or written at a lower level; every
// compression's slot written once.  The solve launches composition level i
// together with affine contraction level i (1-based), so an affine primitive
// of contraction level t may only read composites of composition levels
// below t + 1; the two halves touch disjoint arrays otherwise (transitions
// against vectors).
static bool verify_composition(const PlanHost &P) {
  const int64_t N = P.N, S = P.n_edge_slots;
  std::vector<int32_t> lvl((size_t)S, -1);  // composition level that wrote the slot (0: original)
  for (int64_t s = 0; s < N; ++s) lvl[(size_t)s] = 0;
  int64_t count = 0;
  for (int64_t t = 0; t < P.state_levels(); ++t)
    for (int64_t i = P.tc_off[t]; i < P.tc_off[t + 1]; ++i) {
      const Op4 &q = P.tc_ops[(size_t)i];
      if (q.a < 0 || q.a >= S || q.b < 0 || q.b >= S || q.c < N || q.c >= S) return false;
      if (lvl[(size_t)q.a] < 0 || lvl[(size_t)q.a] > t || lvl[(size_t)q.b] < 0 || lvl[(size_t)q.b] > t) return false;
      if (lvl[(size_t)q.c] >= 0) return false;
      lvl[(size_t)q.c] = (int32_t)(t + 1);
      ++count;
    }
  if (count != P.n_compress) return false;
  for (int64_t t = 0; t < P.levels(); ++t)
    for (int64_t k = P.lvl_off[t]; k < P.lvl_off[t + 1]; ++k) {
      const OpRec &o = P.ops[(size_t)k];
      if (o.kind != OP_RAKE && o.kind != OP_COMPRESS) continue;
      const int32_t l = lvl[(size_t)o.b];
      if (l < 0 || l > t + 1) return false;
    }
  return true;
}

// State expansion: x_j from the state of its parent at removal time through
// the composite map of its slot; the parent is the root (state from the local
// solve) or a node expanded at a lower level; every removed node once.
static bool verify_state_expansion(const PlanHost &P) {
  const int64_t N = P.N;
  std::vector<int32_t> done((size_t)N, -1);
  for (int64_t v = 0; v < N; ++v)
    if (P.parent32[(size_t)v] < 0) done[(size_t)v] = -2;  // roots: known before the first level
  int64_t count = 0;
  for (int64_t e = 0; e < P.sexp_levels(); ++e)
    for (int64_t i = P.sx_off[e]; i < P.sx_off[e + 1]; ++i) {
      const Op4 &q = P.sx_ops[(size_t)i];
      if (q.a < 0 || q.a >= N || q.c < 0 || q.c >= N || q.b < 0 || q.b >= P.n_edge_slots) return false;
      if (done[(size_t)q.a] != -1) return false;
      const int32_t pd = done[(size_t)q.c];
      if (!(pd == -2 || (pd >= 0 && pd < e))) return false;
      done[(size_t)q.a] = (int32_t)e;
      ++count;
    }
  return count == P.n_rake + P.n_compress;
}

bool verify_crew(const PlanHost &P) {
  return verify_contraction(P) && verify_expansion(P) && verify_composition(P) && verify_state_expansion(P);
}

int build_plan(const int64_t *parent, int64_t N, int n, int m, int selection, PlanHost &out) {
  if (!parent) return RCR_NULL_ARG;
  if (N < 1 || n < 1 || m < 1 || n > RCR_MAX_DIM || m > RCR_MAX_DIM) return RCR_BAD_DIMS;
  if (selection != RCR_SELECT_GREEDY_INDEX && selection != RCR_SELECT_LIST_RANK) return RCR_BAD_OPTION;
  out = PlanHost();
  out.N = N;
  out.n = n;
  out.m = m;
  out.selection = selection;
  static thread_local Work kept;
  Builder b(parent, N, out);
  std::swap(static_cast<Work &>(b), kept);
  const int rc = b.run(selection);
  if (N <= KEEP_NODES) std::swap(static_cast<Work &>(b), kept);
  return rc;
}

// Lifted tree (Prop. 2): native node i keeps id i as its predecision node i^-;
// every non-leaf i gains a decision node i^+ with id N + (rank of i among the
// non-leaves in increasing id), the child of i^- through the decision edge;
// each native child j of i hangs below i^+ through its uncertainty edge.
int build_lift_plan(const int64_t *parent, int64_t N, int n, int m, int selection, PlanHost &out) {
  if (!parent) return RCR_NULL_ARG;
  if (N < 1 || n < 1 || m < 1 || n + m > RCR_MAX_DIM) return RCR_BAD_DIMS;
  if (N > (int64_t)(INT32_MAX / 4)) return RCR_BAD_DIMS;
  std::vector<char> nonleaf(N, 0);
  for (int64_t j = 0; j < N; ++j) {
    if (parent[j] < -1 || parent[j] >= N) return RCR_INVALID_TREE;
    if (parent[j] >= 0) nonleaf[parent[j]] = 1;
  }
  std::vector<int32_t> plus(N, -1);
  int64_t NL = N;
  for (int64_t i = 0; i < N; ++i)
    if (nonleaf[i]) plus[i] = (int32_t)NL++;
  std::vector<int64_t> lp(NL);
  for (int64_t i = 0; i < N; ++i) lp[i] = parent[i] < 0 ? -1 : plus[parent[i]];
  for (int64_t i = 0; i < N; ++i)
    if (plus[i] >= 0) lp[plus[i]] = i;
  // a cycle of the native tree is a cycle of the lifted one: build_plan rejects it
  int rc = build_plan(lp.data(), NL, n + m, m, selection, out);
  if (rc) return rc;
  out.lift_N = N;
  out.lift_n = n;
  out.lift_plus = std::move(plus);
  return RCR_OK;
}

int build_ragged_plan(const int64_t *parent, int64_t N, const int32_t *n_node, const int32_t *m_edge, int selection,
                      PlanHost &out) {
  if (!parent || !n_node || !m_edge) return RCR_NULL_ARG;
  if (N < 1) return RCR_BAD_DIMS;
  int nmax = 1, mmax = 1;
  for (int64_t v = 0; v < N; ++v) {
    if (parent[v] < -1 || parent[v] >= N) return RCR_INVALID_TREE;
    if (n_node[v] < 1 || n_node[v] > RCR_MAX_DIM) return RCR_BAD_DIMS;
    nmax = std::max(nmax, (int)n_node[v]);
    if (parent[v] >= 0) {
      if (m_edge[v] < 1 || m_edge[v] > RCR_MAX_DIM) return RCR_BAD_DIMS;
      mmax = std::max(mmax, (int)m_edge[v]);
    }
  }
  const int rc = build_plan(parent, N, nmax, mmax, selection, out);
  if (rc) return rc;
  out.rg_n.assign(n_node, n_node + N);
  out.rg_m.resize((size_t)N);
  for (int64_t v = 0; v < N; ++v) out.rg_m[(size_t)v] = parent[v] >= 0 ? m_edge[v] : 0;
  // block sizes per field (node v, edge slot v = (parent, v)): Q q c Delta R S r A B, K P x u lam
  const int64_t N1 = N + 1;
  out.rg_off.assign((size_t)(RG_FIELDS * N1), 0);
  for (int64_t v = 0; v < N; ++v) {
    const int64_t nv = out.rg_n[(size_t)v], mv = out.rg_m[(size_t)v];
    const int64_t np = parent[v] >= 0 ? out.rg_n[(size_t)parent[v]] : 0;
    const int64_t sz[RG_FIELDS] = {nv * nv, nv, nv, nv * nv, mv * mv, np * mv, mv,
                                   nv * np, nv * mv, mv * np, nv * nv, nv, mv, nv};
    for (int f = 0; f < RG_FIELDS; ++f) out.rg_off[(size_t)(f * N1 + v + 1)] = out.rg_off[(size_t)(f * N1 + v)] + sz[f];
  }
  return RCR_OK;
}

int merge_plans(const std::vector<const PlanHost *> &parts, PlanHost &out) {
  if (parts.empty()) return RCR_NULL_ARG;
  for (const PlanHost *p : parts)
    if (p && (p->lift_N || !p->rg_n.empty())) return RCR_BAD_OPTION;  // solved through their own entry points
  const int n = parts[0]->n, m = parts[0]->m;
  out = PlanHost();
  out.n = n;
  out.m = m;
  int64_t N = 0, C = 0, NC = 0;
  int64_t L = 0, LE = 0, LT = 0, LX = 0;
  for (const PlanHost *p : parts) {
    if (!p) return RCR_NULL_ARG;
    if (p->n != n || p->m != m) return RCR_BAD_DIMS;
    N += p->N;
    C += p->n_edge_slots - p->N;
    NC += p->n_contrib;
    L = std::max(L, p->levels());
    LE = std::max(LE, p->expand_levels());
    LT = std::max(LT, p->state_levels());
    LX = std::max(LX, p->sexp_levels());
  }
  if (N + C > (int64_t)(INT32_MAX / 2 - 16) || NC > (int64_t)(INT32_MAX / 2 - 16)) return RCR_BAD_DIMS;
  const size_t k = parts.size();
  std::vector<int64_t> vb(k), ecb(k), cb(k);
  {
    int64_t a = 0, e = N, c = 0;
    for (size_t t = 0; t < k; ++t) {
      vb[t] = a;
      ecb[t] = e;
      cb[t] = c;
      a += parts[t]->N;
      e += parts[t]->n_edge_slots - parts[t]->N;
      c += parts[t]->n_contrib;
    }
  }
  out.N = N;
  out.n_edge_slots = N + C;
  out.n_contrib = NC;
  out.root = parts[0]->root;
  out.selection = parts[0]->selection;
  out.tree_off.resize(k + 1);
  out.parent32.resize(N);
  for (size_t t = 0; t < k; ++t) {
    const PlanHost &p = *parts[t];
    out.tree_off[t] = vb[t];
    for (int64_t v = 0; v < p.N; ++v)
      out.parent32[vb[t] + v] = p.parent32[v] < 0 ? -1 : (int32_t)(vb[t] + p.parent32[v]);
    out.height = std::max(out.height, p.height);
    out.leaves += p.leaves;
    out.max_degree = std::max(out.max_degree, p.max_degree);
    out.rounds = std::max(out.rounds, p.rounds);
    out.n_rake += p.n_rake;
    out.n_compress += p.n_compress;
    out.n_combine += p.n_combine;
    out.n_absorb += p.n_absorb;
  }
  out.tree_off[k] = N;
  auto node = [&](size_t t, int32_t v) { return (int32_t)(vb[t] + v); };
  auto slot = [&](size_t t, int32_t s2) {
    return (int32_t)(s2 < parts[t]->N ? vb[t] + s2 : ecb[t] + (s2 - parts[t]->N));
  };
  auto contrib = [&](size_t t, int32_t c) { return (int32_t)(cb[t] + c); };
  {
    size_t n_ops = 0, n_exp = 0, n_tc = 0, n_sx = 0;
    for (const PlanHost *p : parts) {
      n_ops += p->ops.size();
      n_exp += p->exp_ops.size();
      n_tc += p->tc_ops.size();
      n_sx += p->sx_ops.size();
    }
    out.ops.reserve(n_ops);
    out.exp_ops.reserve(n_exp);
    out.tc_ops.reserve(n_tc);
    out.sx_ops.reserve(n_sx);
  }
  // contraction: level-major, kind-minor, tree order within a (level, kind) group
  auto contraction = [&] {
    out.lvl_off.assign(1, 0);
    out.kind_off.resize((size_t)L * 5);
    for (int64_t lv = 0; lv < L; ++lv) {
      for (int kind = 0; kind < 4; ++kind) {
        out.kind_off[(size_t)lv * 5 + kind] = (int64_t)out.ops.size();
        for (size_t t = 0; t < k; ++t) {
          const PlanHost &p = *parts[t];
          if (lv >= p.levels()) continue;
          for (int64_t i = p.kind_off[(size_t)lv * 5 + kind]; i < p.kind_off[(size_t)lv * 5 + kind + 1]; ++i) {
            OpRec o = p.ops[i];
            switch (o.kind) {
              case OP_RAKE: o.a = node(t, o.a); o.b = slot(t, o.b); o.c = contrib(t, o.c); o.d = node(t, o.d); break;
              case OP_COMBINE: o.a = contrib(t, o.a); o.b = contrib(t, o.b); o.c = contrib(t, o.c); o.d = node(t, o.d); break;
              case OP_ABSORB: o.a = node(t, o.a); o.b = contrib(t, o.b); break;
              default: o.a = node(t, o.a); o.b = slot(t, o.b); o.c = slot(t, o.c); o.d = slot(t, o.d); o.e = node(t, o.e);
            }
            out.ops.push_back(o);
          }
        }
      }
      out.kind_off[(size_t)lv * 5 + 4] = (int64_t)out.ops.size();
      out.lvl_off.push_back((int64_t)out.ops.size());
    }
  };
  auto merge4 = [&](int64_t levels, const std::vector<Op4> PlanHost::*ops, const std::vector<int64_t> PlanHost::*off,
                    std::vector<Op4> &dst, std::vector<int64_t> &doff, int kind) {
    doff.assign(1, 0);
    for (int64_t lv = 0; lv < levels; ++lv) {
      for (size_t t = 0; t < k; ++t) {
        const PlanHost &p = *parts[t];
        const std::vector<int64_t> &po = p.*off;
        if (lv + 1 >= (int64_t)po.size()) continue;
        for (int64_t i = po[lv]; i < po[lv + 1]; ++i) {
          Op4 q = (p.*ops)[i];
          if (kind == 0) {         // expansion {j, r slot, k}
            q.a = node(t, q.a); q.b = slot(t, q.b); q.c = node(t, q.c);
          } else if (kind == 1) {  // composition {l slot, r slot, new slot, j}
            q.a = slot(t, q.a); q.b = slot(t, q.b); q.c = slot(t, q.c); q.d = node(t, q.d);
          } else {                 // state expansion {j, slot, parent}
            q.a = node(t, q.a); q.b = slot(t, q.b); q.c = node(t, q.c);
          }
          dst.push_back(q);
        }
      }
      doff.push_back((int64_t)dst.size());
    }
  };
  auto expansion = [&] { merge4(LE, &PlanHost::exp_ops, &PlanHost::exp_off, out.exp_ops, out.exp_off, 0); };
  auto composition = [&] { merge4(LT, &PlanHost::tc_ops, &PlanHost::tc_off, out.tc_ops, out.tc_off, 1); };
  auto state = [&] { merge4(LX, &PlanHost::sx_ops, &PlanHost::sx_off, out.sx_ops, out.sx_off, 2); };
  // the four parts write disjoint arrays of the merged plan
  run_concurrently(N >= PAR_NODES && !build_on_caller_only, contraction, expansion, composition, state);
  return RCR_OK;
}

int64_t depth_bound(int64_t N) {
  if (N <= 1) return 0;
  // floor(log2((2N - 1) * 36^R)), R = ceil(log_{3/2} N), via exact logs of integers:
  // bits of (2N-1) plus R * log2(36), evaluated with a high-precision float and
  // corrected by an integer comparison on 2^k <= (2N-1) * 36^R using long double.
  int64_t R = 0;
  long double p = 1.0L;
  while (p < (long double)N) {
    p *= 1.5L;
    ++R;
  }
  long double v = log2l((long double)(2 * N - 1)) + (long double)R * log2l(36.0L);
  return (int64_t)floorl(v + 1e-15L);
}

}  // namespace rcr
