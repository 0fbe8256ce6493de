// Device-side planner (Sec. VII): the plan of build_plan with the list-rank
// selection, computed by one workgroup on the GPU.
//
// The same structural rounds as the host planner (rake every non-root leaf,
// reduce each parent's new contributions by the readiness-weighted alphabetic
// code of Lemma 3 and absorb the result, then compress alternate nodes of every
// maximal path of non-root unary nodes), the same earliest-start levels
// (eq. (earliest-level)), static slots and pass schedules, so the plan is the
// host's byte for byte.  The rounds are sequential; inside a round every step
// is data-parallel over the live nodes:
//
//   * the host orders a round's rakes by (parent, sibling key); here every node
//     keeps the position of its edge in a stable children-by-parent array built
//     once (a compression hands the removed node's position to its child, as
//     the host hands over the sibling key), so that order is the order of
//     positions: a radix sort of the round's rakes by position;
//   * the alternation along unary paths is the parity of each node's distance
//     from the top of its path, found by pointer jumping (list ranking);
//   * each sibling group's code tree is built by one thread, emitting its
//     combinations in the host's order (post-order), at offsets known from the
//     group's start (a group of k contributions makes k - 1 combinations and
//     one absorption); a group of more than big_group contributions (a hub)
//     is built by the whole workgroup instead (reduce_big_group);
//   * the four schedules are stable radix sorts of the round records by level.
//
// The program is written once against an executor X: X::each(f) runs f(t) for
// every thread t and then synchronises the workgroup; bodies write memory only
// (never the program's own scalars, which every thread derives identically
// from collective results).  The GPU executor runs it on 1024 threads of one
// workgroup; CpuExec runs the threads one after the other in a chosen order,
// which checks that no phase depends on the order of its threads.
#pragma once

#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/rcr.h"
#include "plan.hpp"

namespace rcr {
namespace dplan {

constexpr int THREADS = 1024;
// Sibling groups of more contributions than this are built by the whole
// workgroup (reduce_big_group), smaller ones by one thread each.
constexpr int32_t BIG_GROUP = 128;

// statistics words written by the program (int64)
enum : int {
  S_STATUS = 0, S_ROOT, S_HEIGHT, S_LEAVES, S_MAXDEG, S_ROUNDS, S_RAKE, S_COMPRESS, S_COMBINE, S_ABSORB,
  S_CONTRIB, S_SLOTS, S_OPS, S_L, S_EXP, S_LE, S_TC, S_LT, S_SX, S_LX, S_COUNT
};

// Device (or, for the emulation, host) arrays of one planning run.
struct Arena {
  const int64_t *parent;
  int64_t N;
  int T;
  // per node
  int32_t *par32, *cnt, *up0, *up1, *dist0, *dist1, *cur_par, *lvlU, *lvlE, *edge_slot, *one_child, *alive, *sel,
      *rem_slot, *rem_par, *comp_r, *comp_k, *rem_kind, *live0, *live1, *leaves, *sorted, *gstart, *elig, *comp, *pos,
      *cout, *eP, *eX, *removal, *gslot, *glev;
  uint64_t *code_hi, *code_lo;  // per sorted rake: prefix weight sum, code word
  int32_t *code_d;              // and the common-prefix length with the previous code
  // a group built by the whole workgroup (reduce_big_group), per split position
  int32_t *bg_A, *bg_R, *bg_par, *bg_lc, *bg_rc, *bg_left, *bg_dep, *bg_idx, *bg_val, *bg_p0, *bg_d0, *bg_p1,
      *bg_d1, *bg_seg, *bigs;
  int32_t big_group;  // groups above this size are built by the whole workgroup
  // per op / slot (2N)
  int32_t *contrib_level, *lT;
  OpRec *raw;
  uint32_t *k0, *v0, *k1, *v1;  // sort buffers
  int64_t *off4;                // bucket offsets of a schedule
  // per thread
  uint32_t *tcount, *hist;      // T and 16 T
  uint64_t *tsum;               // T
  // per round (N + 2)
  int32_t *r_raw, *r_rem, *r_comp_rem, *r_comp_raw;
  // outputs
  OpRec *ops;
  Op4 *exp_ops, *tc_ops, *sx_ops;
  int64_t *lvl_off, *kind_off, *exp_off, *tc_off, *sx_off;
  int64_t *stats;
};

// Lays the arrays out from `base` (every array 256-byte aligned) and returns
// the total size; with base == nullptr only the size is computed.
inline size_t carve(Arena &a, char *base, int64_t N, int T) {
  size_t at = 0;
  const size_t n1 = (size_t)N + 2, n2 = 2 * (size_t)N + 2;
  auto take = [&](auto *&p, size_t count) {
    using E = typename std::remove_reference<decltype(*p)>::type;
    at = (at + 255) & ~size_t(255);
    p = base ? reinterpret_cast<E *>(base + at) : nullptr;
    at += count * sizeof(E);
  };
  int32_t **node[] = {&a.par32,   &a.cnt,    &a.up0,     &a.up1,      &a.dist0,  &a.dist1,    &a.cur_par, &a.lvlU,
                      &a.lvlE,    &a.edge_slot, &a.one_child, &a.alive, &a.sel,    &a.rem_slot, &a.rem_par, &a.comp_r,
                      &a.comp_k,  &a.rem_kind, &a.live0,  &a.live1,    &a.leaves, &a.sorted,   &a.gstart,  &a.elig,
                      &a.comp,    &a.pos,    &a.cout,     &a.eP,     &a.eX,       &a.removal, &a.code_d,
                      &a.gslot,   &a.glev,   &a.bg_A,    &a.bg_R,     &a.bg_par, &a.bg_lc,    &a.bg_rc,   &a.bg_left,
                      &a.bg_dep,  &a.bg_idx, &a.bg_val,  &a.bg_p0,    &a.bg_d0,  &a.bg_p1,    &a.bg_d1,   &a.bigs,
                      &a.r_raw,   &a.r_rem,  &a.r_comp_rem, &a.r_comp_raw};
  for (int32_t **p : node) take(*p, n1);
  take(a.code_hi, n1);
  take(a.code_lo, n1);
  take(a.contrib_level, n2);
  take(a.lT, n2);
  take(a.raw, n2);
  take(a.k0, n2);
  take(a.v0, n2);
  take(a.k1, n2);
  take(a.v1, n2);
  take(a.off4, 4 * n2 + 8);
  take(a.bg_seg, 4 * n1);  // a segment tree over at most 2 N leaves
  take(a.tcount, (size_t)T);
  take(a.hist, 16 * (size_t)T);
  take(a.tsum, (size_t)T);
  take(a.ops, n2);
  take(a.exp_ops, n1);
  take(a.tc_ops, n1);
  take(a.sx_ops, n1);
  take(a.lvl_off, n2);
  take(a.kind_off, 5 * n2);
  take(a.exp_off, n1);
  take(a.tc_off, n1);
  take(a.sx_off, n1);
  take(a.stats, (size_t)S_COUNT);
  a.N = N;
  a.T = T;
  a.big_group = BIG_GROUP;
  return (at + 255) & ~size_t(255);
}

__host__ __device__ inline int bitlen(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// Stable compaction of the indices i < n with pred(i), in increasing i:
// write(i, o) for the o-th of them; returns their number (the executor's own
// implementation; pred must not depend on what write stores).
template <class X, class P, class W>
__host__ __device__ uint32_t compact(X &x, const Arena &a, int64_t n, P pred, W write) {
  return x.compact(a, n, pred, write);
}

// Stable least-significant-digit radix sort of (k[i], v[i]), i < n, on the low
// `bits` bits of the keys, 4 bits per pass (the executor's radix_pass); the
// result is in (k, v) on return (the pointers are swapped with the spare
// buffers as passes go).
template <class X>
__host__ __device__ void radix_sort(X &x, const Arena &a, int64_t n, int bits, uint32_t *&k, uint32_t *&v,
                                    uint32_t *&k2, uint32_t *&v2) {
  for (int sh = 0; sh < bits; sh += 4) {
    x.radix_pass(a, n, sh, k, v, k2, v2);
    uint32_t *tk = k, *tv = v;
    k = k2;
    v = v2;
    k2 = tk;
    v2 = tv;
  }
}

// off[b] = the first q < n with key[q] >= b, for b = 0..B (n where none);
// keys are sorted and below B.
template <class X>
__host__ __device__ void bucket_offsets(X &x, const Arena &a, const uint32_t *key, int64_t n, int64_t B, int64_t *off) {
  x.each([&](int t) {
    for (int64_t q = t; q <= n; q += a.T) {
      const int64_t lo = q == 0 ? 0 : (int64_t)key[q - 1] + 1, hi = q == n ? B : (int64_t)key[q];
      for (int64_t b = lo; b <= hi; ++b) off[b] = q;
    }
  });
}

// The code word of Lemma 3's alphabetic code for weight w = 2^e whose
// predecessors in the group weigh S in all (W the group's total, clW the
// smallest c with 2^c >= W): the leading d = ceil(log2(W / w)) + 1 bits of
// (2 S + w) / (2 W), by restoring division, left-aligned in 64 bits.
__host__ __device__ inline uint64_t code_word(uint64_t S, int e, uint64_t W, int clW) {
  const uint64_t w = (uint64_t)1 << e, D = 2 * W;
  const int d = (clW > e ? clW - e : 0) + 1;
  uint64_t rem = 2 * S + w, q = 0;  // rem < D
  for (int b = 0; b < d; ++b) {
    rem <<= 1;
    q <<= 1;
    if (rem >= D) {
      rem -= D;
      q |= 1;
    }
  }
  return q << (64 - d);
}

// Common-prefix length of two distinct left-aligned code words.
__host__ __device__ inline int32_t lcp_bits(uint64_t a, uint64_t b) { return (int32_t)__builtin_clzll(a ^ b); }

// One sibling group (Lemma 3): the contributions at sorted positions [s0, s1)
// of parent i (their slots and levels staged in gslot, glev); emits its k - 1
// combinations and its absorption at raw[r0 ..] with combination slots c0,
// c0 + 1, ... in the host's order, and updates lvlU[i].
//
// The host builds the code tree by descending one bit at a time: at depth p a
// range splits at its first code with a 1 in bit p, and a range whose codes
// all agree in bit p is a unary vertex (suppressed).  The same tree follows
// from the common-prefix lengths L_j of neighbouring codes j - 1 and j: the
// codes of a range agree in their first min L bits (min over the range's
// inner neighbours), so the host descends to depth min L and splits at the
// first j where L_j = min L (the codes increase, so bit min L flips there
// from 0 to 1, once).  Weights are powers of two and 2 S + w < 2 W, so each
// code word is at most 63 bits, found by a restoring division of d steps.
__host__ __device__ inline void reduce_group(const Arena &a, int32_t s0, int32_t s1, int32_t r0, int32_t c0,
                                             int32_t rnd) {
  const int k = s1 - s0;
  const int32_t i = a.cur_par[a.sorted[s0]];
  const int32_t *gslot = a.gslot + s0, *glev = a.glev + s0;
  int32_t agg, agg_lvl;
  if (k == 1) {
    agg = gslot[0];
    agg_lvl = glev[0];
  } else {
    int32_t lmin = glev[0];
    for (int j = 1; j < k; ++j) lmin = glev[j] < lmin ? glev[j] : lmin;
    int lg = 0;
    while ((1LL << lg) < k) ++lg;
    const int cap = 61 - lg;
    uint64_t W = 0;  // < k 2^cap <= 2^61
    for (int j = 0; j < k; ++j) {
      const int e = glev[j] - lmin;
      W += (uint64_t)1 << (e < cap ? e : cap);
    }
    const int clW = bitlen(W - 1);  // smallest c with 2^c >= W
    uint64_t *code = a.code_lo + s0;  // code words, left-aligned in 64 bits
    int32_t *L = a.code_d + s0;       // L[j]: common-prefix length of codes j - 1 and j
    uint64_t S = 0;
    for (int j = 0; j < k; ++j) {
      const int e0 = glev[j] - lmin, e = e0 < cap ? e0 : cap;
      code[j] = code_word(S, e, W, clW);
      if (j > 0) L[j] = lcp_bits(code[j - 1], code[j]);  // codes are distinct
      S += (uint64_t)1 << e;
    }
    // the host's recursive build, as an explicit stack: frames of (range,
    // stage, split, left result); results return through (ret, ret_lvl)
    struct Frame {
      int lo, hi, s, stage;
      int32_t a, la;
    };
    Frame st[80];  // the code tree is at most 62 deep
    int sp = 0;
    st[sp++] = Frame{0, k - 1, 0, 0, 0, 0};
    int32_t ret = 0, ret_lvl = 0, emitted = 0;
    while (sp > 0) {
      Frame &f = st[sp - 1];
      if (f.stage == 0) {
        if (f.lo == f.hi) {
          ret = gslot[f.lo];
          ret_lvl = glev[f.lo];
          --sp;
          continue;
        }
        int s = f.lo + 1;
        for (int j = f.lo + 2; j <= f.hi; ++j)
          if (L[j] < L[s]) s = j;
        f.s = s;
        f.stage = 1;
        st[sp++] = Frame{f.lo, s - 1, 0, 0, 0, 0};
      } else if (f.stage == 1) {
        f.a = ret;
        f.la = ret_lvl;
        f.stage = 2;
        st[sp++] = Frame{f.s, f.hi, 0, 0, 0, 0};
      } else {
        const int32_t lv = 1 + (f.la > ret_lvl ? f.la : ret_lvl);
        const int32_t out = c0 + emitted;
        a.contrib_level[out] = lv;
        a.raw[r0 + emitted] = OpRec{OP_COMBINE, rnd, lv, f.a, ret, out, i, 0};
        ++emitted;
        ret = out;
        ret_lvl = lv;
        --sp;
      }
    }
    agg = ret;
    agg_lvl = ret_lvl;
  }
  const int32_t lv = 1 + (a.lvlU[i] > agg_lvl ? a.lvlU[i] : agg_lvl);
  a.raw[r0 + k - 1] = OpRec{OP_ABSORB, rnd, lv, i, agg, 0, 0, 0};
  a.lvlU[i] = lv;
}

// Segment trees over positions 0 .. P - 1 (P a power of two, leaves at
// seg[P + q], node v over its children 2 v and 2 v + 1).
// The largest position q < p whose leaf is <= x, 0 when there is none, in a
// tree of minima.
__host__ __device__ inline int32_t seg_last_le(const int32_t *seg, int32_t P, int32_t p, int32_t x) {
  int32_t v = P + p;
  for (; v > 1; v >>= 1) {
    if ((v & 1) && seg[v - 1] <= x) {  // the left sibling's range holds one: its rightmost
      v -= 1;
      while (v < P) v = seg[2 * v + 1] <= x ? 2 * v + 1 : 2 * v;
      return v - P;
    }
  }
  return 0;
}
// The smallest position q > p whose leaf is < x, P when there is none, in a
// tree of minima.
__host__ __device__ inline int32_t seg_first_lt(const int32_t *seg, int32_t P, int32_t p, int32_t x) {
  int32_t v = P + p;
  for (; v > 1; v >>= 1) {
    if (!(v & 1) && seg[v + 1] < x) {  // the right sibling's range holds one: its leftmost
      v += 1;
      while (v < P) v = seg[2 * v] < x ? 2 * v : 2 * v + 1;
      return v - P;
    }
  }
  return P;
}
// The largest leaf of positions lo .. hi in a tree of maxima.
__host__ __device__ inline int32_t seg_max(const int32_t *seg, int32_t P, int32_t lo, int32_t hi) {
  int32_t r = INT32_MIN;
  for (int32_t l = lo + P, h = hi + P + 1; l < h; l >>= 1, h >>= 1) {
    if (l & 1) r = seg[l] > r ? seg[l] : r, ++l;
    if (h & 1) --h, r = seg[h] > r ? seg[h] : r;
  }
  return r;
}

// reduce_group for a large group, by the whole workgroup, with the same
// output.  The code tree splits a range at the first minimum of its
// common-prefix lengths, so it is the Cartesian tree of L_1 .. L_{k-1} with
// ties going to the leftmost; its vertex p (a combination) covers the codes
// A_p .. B_p, where A_p is the nearest q < p with L_q <= L_p (0 when none) and
// B_p + 1 the nearest q > p with L_q < L_p (k when none), both found in a
// segment tree of minima; its parent is whichever of the two has the larger L
// (on a tie the right one, which lies below the left one).  In the host's
// post-order the combination p comes after the k - 1 - (B_p - A_p) vertices
// left of its codes' range minus those of them that are its ancestors, so
// its index is B_p - 1 - (the number of ancestors left of p), which follows
// the chain p -> A_p -> ... by pointer jumping.  Its level is 1 + the larger
// of its operands' levels, that is the largest of (level of a code + its
// depth below p) over the codes A_p .. B_p: depths by pointer jumping along
// the parents, the maxima from a segment tree of maxima.
template <class X>
__host__ __device__ void reduce_big_group(X &x, const Arena &a, int32_t s0, int32_t s1, int32_t r0, int32_t c0,
                                          int32_t rnd) {
  const int T = a.T;
  const int32_t k = s1 - s0, m = k - 1;  // codes 0 .. k - 1, split positions 1 .. m
  const int32_t i = a.cur_par[a.sorted[s0]];
  const int32_t *gslot = a.gslot + s0, *glev = a.glev + s0;
  uint64_t *code = a.code_lo + s0, *S = a.code_hi + s0;
  int32_t *L = a.code_d + s0;
  const int32_t lmin = -x.maxall([&](int t) {
    int32_t mm = INT32_MIN;
    for (int32_t j = t; j < k; j += T) mm = -glev[j] > mm ? -glev[j] : mm;
    return mm;
  });
  int lg = 0;
  while ((1LL << lg) < k) ++lg;
  const int cap = 61 - lg;
  auto expo = [&](int32_t j) {
    const int e = glev[j] - lmin;
    return e < cap ? e : cap;
  };
  // prefix sums of the weights over contiguous chunks
  const int32_t C = (k + T - 1) / T;
  x.each([&](int t) {
    uint64_t sum = 0;
    for (int32_t j = t * C, e = (t + 1) * C < k ? (t + 1) * C : k; j < e; ++j) sum += (uint64_t)1 << expo(j);
    a.tsum[t] = sum;
  });
  const uint64_t W = x.scan64(a.tsum);
  x.each([&](int t) {
    uint64_t sum = a.tsum[t];
    for (int32_t j = t * C, e = (t + 1) * C < k ? (t + 1) * C : k; j < e; ++j) {
      S[j] = sum;
      sum += (uint64_t)1 << expo(j);
    }
  });
  const int clW = bitlen(W - 1);
  x.each([&](int t) {
    for (int32_t j = t; j < k; j += T) code[j] = code_word(S[j], expo(j), W, clW);
  });
  x.each([&](int t) {
    for (int32_t j = 1 + t; j < k; j += T) L[j] = lcp_bits(code[j - 1], code[j]);
  });
  // tree of minima over L (position 0 and those past m never match)
  int32_t P = 1;
  while (P < k) P <<= 1;
  int32_t *seg = a.bg_seg;
  x.each([&](int t) {
    for (int32_t q = t; q < P; q += T) seg[P + q] = (q >= 1 && q <= m) ? L[q] : INT32_MAX;
  });
  for (int32_t h = P >> 1; h >= 1; h >>= 1)
    x.each([&](int t) {
      for (int32_t v = h + t; v < 2 * h; v += T) seg[v] = seg[2 * v] < seg[2 * v + 1] ? seg[2 * v] : seg[2 * v + 1];
    });
  x.each([&](int t) {
    for (int32_t p = 1 + t; p <= m; p += T) {
      const int32_t A = seg_last_le(seg, P, p, L[p]), f = seg_first_lt(seg, P, p, L[p]), R = f >= P ? k : f;
      const bool hl = A >= 1, hr = R <= m;
      a.bg_A[p] = A;
      a.bg_R[p] = R;
      a.bg_par[p] = hl && hr ? (L[A] > L[R] ? A : R) : (hl ? A : (hr ? R : 0));
    }
  });
  x.each([&](int t) {
    for (int32_t p = 1 + t; p <= m; p += T) {
      const int32_t q = a.bg_par[p];
      if (q && p < q) a.bg_lc[q] = p;
      if (q && p > q) a.bg_rc[q] = p;
    }
  });
  // the length of the chain p -> next(p) -> ... -> 0 for every split p, by
  // pointer jumping (position 0 is the chains' common end)
  auto chain = [&](const int32_t *next, int32_t *out) {
    int32_t *p0 = a.bg_p0, *d0 = a.bg_d0, *p1 = a.bg_p1, *d1 = a.bg_d1;
    x.each([&](int t) {
      for (int32_t q = t; q <= m; q += T) {
        const int32_t f = q ? next[q] : 0;
        p0[q] = f;
        d0[q] = f ? 1 : 0;
      }
    });
    for (int it = 0; it < 64; ++it) {
      const bool more = x.any([&](int t) {
        bool c = false;
        for (int32_t q = t; q <= m; q += T) {
          const int32_t w = p0[q];
          d1[q] = d0[q] + d0[w];
          p1[q] = p0[w];
          c |= p0[w] != 0;
        }
        return c;
      });
      int32_t *tp = p0, *td = d0;
      p0 = p1;
      d0 = d1;
      p1 = tp;
      d1 = td;
      if (!more) break;
    }
    x.each([&](int t) {
      for (int32_t q = t; q <= m; q += T) out[q] = d0[q];
    });
  };
  chain(a.bg_A, a.bg_left);  // ancestors left of p
  chain(a.bg_par, a.bg_dep);  // ancestors
  // per code: its level + its depth (that of the deeper adjacent split, + 1)
  x.each([&](int t) {
    for (int32_t l = t; l < k; l += T) {
      const bool hl = l >= 1, hr = l + 1 <= m;
      const int32_t ps = hl && hr ? (L[l] > L[l + 1] ? l : l + 1) : (hl ? l : l + 1);
      a.bg_val[l] = glev[l] + a.bg_dep[ps] + 1;
    }
  });
  x.each([&](int t) {
    for (int32_t q = t; q < P; q += T) seg[P + q] = q < k ? a.bg_val[q] : INT32_MIN;
  });
  for (int32_t h = P >> 1; h >= 1; h >>= 1)
    x.each([&](int t) {
      for (int32_t v = h + t; v < 2 * h; v += T) seg[v] = seg[2 * v] > seg[2 * v + 1] ? seg[2 * v] : seg[2 * v + 1];
    });
  x.each([&](int t) {  // post-order index and level of every combination
    for (int32_t p = 1 + t; p <= m; p += T) {
      const int32_t A = a.bg_A[p], B = a.bg_R[p] - 1;
      a.bg_idx[p] = B - 1 - a.bg_left[p];
      a.bg_val[p] = seg_max(seg, P, A, B) - a.bg_dep[p];
    }
  });
  x.each([&](int t) {
    for (int32_t p = 1 + t; p <= m; p += T) {
      const int32_t A = a.bg_A[p], B = a.bg_R[p] - 1, lv = a.bg_val[p], id = a.bg_idx[p];
      const int32_t lo = A == p - 1 ? gslot[p - 1] : c0 + a.bg_idx[a.bg_lc[p]];
      const int32_t hi = B == p ? gslot[p] : c0 + a.bg_idx[a.bg_rc[p]];
      a.contrib_level[c0 + id] = lv;
      a.raw[r0 + id] = OpRec{OP_COMBINE, rnd, lv, lo, hi, c0 + id, i, 0};
      if (a.bg_par[p] == 0) {  // the root: the group's aggregate, absorbed into i
        const int32_t la = 1 + (a.lvlU[i] > lv ? a.lvlU[i] : lv);
        a.raw[r0 + k - 1] = OpRec{OP_ABSORB, rnd, la, i, c0 + id, 0, 0, 0};
        a.lvlU[i] = la;
      }
    }
  });
}

// The planner.  Returns 0 or a negative RCR_* status; the statistics and
// schedules are in the arena's outputs.
template <class X>
__host__ __device__ int32_t program(X &x, Arena &a) {
  const int64_t N = a.N;
  const int T = a.T;
  // ---- validation, degrees, the root
  const bool bad = x.any([&](int t) {
    bool b = false;
    for (int64_t i = t; i < N; i += T) {
      const int64_t p = a.parent[i];
      if (p < 0) {
        b |= p != -1;
      } else {
        b |= p >= N || p == i;
      }
      a.cnt[i] = 0;
    }
    return b;
  });
  if (bad) return RCR_INVALID_TREE;
  const uint32_t roots = compact(
      x, a, N, [&](int64_t i) { return a.parent[i] == -1; },
      [&](int64_t i, uint32_t o) {
        if (o == 0) a.stats[S_ROOT] = i;
      });
  if (roots != 1) return RCR_INVALID_TREE;
  const int32_t root = (int32_t)a.stats[S_ROOT];
  x.each([&](int t) {
    for (int64_t i = t; i < N; i += T) {
      const int32_t p = (int32_t)a.parent[i];
      a.par32[i] = p;
      if (p >= 0) x.atomic_add(&a.cnt[p], 1);
      a.up0[i] = p < 0 ? (int32_t)i : p;
      a.dist0[i] = p < 0 ? 0 : 1;
    }
  });
  // ---- depths by pointer jumping; a node that never reaches the root lies on a cycle
  {
    int32_t *u = a.up0, *d = a.dist0, *u2 = a.up1, *d2 = a.dist1;
    const int iters = bitlen((uint64_t)N) + 1;
    for (int it = 0; it < iters; ++it) {
      const bool ch = x.any([&](int t) {
        bool c = false;
        for (int64_t i = t; i < N; i += T) {
          const int32_t w = u[i];
          const int64_t s = (int64_t)d[i] + d[w];  // bounded: on a cycle it would grow without end
          d2[i] = s > INT32_MAX ? INT32_MAX : (int32_t)s;
          u2[i] = u[w];
          c |= u2[i] != w;
        }
        return c;
      });
      int32_t *tu = u, *td = d;
      u = u2;
      d = d2;
      u2 = tu;
      d2 = td;
      if (!ch) break;
    }
    const bool cyc = x.any([&](int t) {
      bool c = false;
      for (int64_t i = t; i < N; i += T) c |= u[i] != root;
      return c;
    });
    if (cyc) return RCR_INVALID_TREE;
    const int32_t h = x.maxall([&](int t) {
      int32_t m = 0;
      for (int64_t i = t; i < N; i += T) m = d[i] > m ? d[i] : m;
      return m;
    });
    const int32_t maxdeg = x.maxall([&](int t) {
      int32_t m = 0;
      for (int64_t i = t; i < N; i += T) m = a.cnt[i] > m ? a.cnt[i] : m;
      return m;
    });
    const uint32_t nleaf = compact(
        x, a, N, [&](int64_t i) { return a.cnt[i] == 0; }, [&](int64_t, uint32_t) {});
    x.each([&](int t) {
      if (t == 0) {
        a.stats[S_HEIGHT] = h;
        a.stats[S_MAXDEG] = maxdeg;
        a.stats[S_LEAVES] = nleaf;
      }
    });
  }
  // ---- edge positions: non-root nodes stably sorted by parent
  {
    uint32_t *k = a.k0, *v = a.v0, *k2 = a.k1, *v2 = a.v1;
    const uint32_t n1 = compact(
        x, a, N, [&](int64_t i) { return i != root; },
        [&](int64_t i, uint32_t o) {
          k[o] = (uint32_t)a.par32[i];
          v[o] = (uint32_t)i;
        });
    radix_sort(x, a, n1, bitlen((uint64_t)(N - 1)), k, v, k2, v2);
    x.each([&](int t) {
      for (int64_t q = t; q < (int64_t)n1; q += T) a.pos[v[q]] = (int32_t)q;
    });
  }
  // ---- rounds
  x.each([&](int t) {
    for (int64_t i = t; i < N; i += T) {
      a.cur_par[i] = a.par32[i];
      a.lvlU[i] = a.lvlE[i] = 0;
      a.edge_slot[i] = (int32_t)i;
      a.one_child[i] = -1;
      a.alive[i] = 1;
      a.sel[i] = 0;
      a.rem_slot[i] = a.rem_par[i] = a.comp_r[i] = a.comp_k[i] = -1;
      a.rem_kind[i] = 0;
      a.live0[i] = (int32_t)i;
      a.eP[i] = a.eX[i] = 0;
    }
  });
  int32_t *live = a.live0, *live_next = a.live1;
  int64_t live_n = N;
  int32_t rnd = 0, next_slot = (int32_t)N, next_contrib = 0, raw_n = 0, rem_n = 0;
  int64_t n_rake = 0, n_compress = 0, n_combine = 0, n_absorb = 0;
  while (live_n > 1) {
    ++rnd;
    if (rnd > N) return RCR_INVALID_TREE;  // no progress: cannot happen on a tree (Lemma 2)
    const int32_t round_raw = raw_n, round_rem = rem_n;
    // rakes: every live non-root leaf, in increasing id
    const uint32_t nl = compact(
        x, a, live_n, [&](int64_t q) { return live[q] != root && a.cnt[live[q]] == 0; },
        [&](int64_t q, uint32_t o) { a.leaves[o] = live[q]; });
    x.each([&](int t) {
      if (t == 0) {
        a.r_raw[rnd] = round_raw;
        a.r_rem[rnd] = round_rem;
      }
      for (int64_t q = t; q < (int64_t)nl; q += T) {
        const int32_t j = a.leaves[q];
        const int32_t lv = 1 + (a.lvlU[j] > a.lvlE[j] ? a.lvlU[j] : a.lvlE[j]);
        const int32_t out = next_contrib + (int32_t)q;
        a.contrib_level[out] = lv;
        a.raw[raw_n + q] = OpRec{OP_RAKE, rnd, lv, j, a.edge_slot[j], out, a.cur_par[j], 0};
        a.rem_kind[j] = 1;
        a.rem_slot[j] = a.edge_slot[j];
        a.rem_par[j] = a.cur_par[j];
        a.removal[rem_n + q] = j;
        a.cout[j] = out;
        a.k0[q] = (uint32_t)a.pos[j];
        a.v0[q] = (uint32_t)j;
      }
    });
    n_rake += nl;
    next_contrib += (int32_t)nl;
    raw_n += (int32_t)nl;
    rem_n += (int32_t)nl;
    // the rakes in (parent, sibling) order: the order of their edge positions
    // (distinct), by a radix sort of this round's rakes only
    {
      uint32_t *pk = a.k0, *pv = a.v0, *pk2 = a.k1, *pv2 = a.v1;
      radix_sort(x, a, nl, bitlen((uint64_t)N), pk, pv, pk2, pv2);
      x.each([&](int t) {
        for (int64_t q = t; q < (int64_t)nl; q += T) {
          const int32_t j = (int32_t)pv[q];
          a.sorted[q] = j;
          a.gslot[q] = a.cout[j];
          a.glev[q] = a.contrib_level[a.cout[j]];
        }
      });
    }
    const uint32_t G = compact(
        x, a, nl,
        [&](int64_t q) { return q == 0 || a.cur_par[a.sorted[q]] != a.cur_par[a.sorted[q - 1]]; },
        [&](int64_t q, uint32_t o) { a.gstart[o] = (int32_t)q; });
    {
      const int32_t r0 = raw_n, c0 = next_contrib;
      auto group_end = [&](int64_t g) { return g + 1 < (int64_t)G ? a.gstart[g + 1] : (int32_t)nl; };
      const bool any_big = x.any([&](int t) {
        bool big = false;
        for (int64_t g = t; g < (int64_t)G; g += T) {
          const int32_t s0 = a.gstart[g], s1 = group_end(g);
          if (s1 - s0 <= a.big_group)
            reduce_group(a, s0, s1, r0 + s0, c0 + (s0 - (int32_t)g), rnd);
          else
            big = true;
        }
        return big;
      });
      const uint32_t nbig = !any_big ? 0 : compact(
          x, a, G, [&](int64_t g) { return group_end(g) - a.gstart[g] > a.big_group; },
          [&](int64_t g, uint32_t o) { a.bigs[o] = (int32_t)g; });
      for (uint32_t b = 0; b < nbig; ++b) {
        const int32_t g = a.bigs[b], s0 = a.gstart[g];
        reduce_big_group(x, a, s0, group_end(g), r0 + s0, c0 + (s0 - g), rnd);
      }
    }
    raw_n += (int32_t)nl;
    next_contrib += (int32_t)nl - (int32_t)G;
    n_combine += nl - G;
    n_absorb += G;
    x.each([&](int t) {
      for (int64_t q = t; q < (int64_t)nl; q += T) {
        const int32_t j = a.leaves[q];
        a.alive[j] = 0;
        x.atomic_add(&a.cnt[a.cur_par[j]], -1);
      }
    });
    // unary nodes of the post-rake tree and the single child of each
    x.each([&](int t) {
      for (int64_t q = t; q < live_n; q += T) {
        const int32_t v = live[q];
        if (a.alive[v] && v != root && a.cnt[a.cur_par[v]] == 1) a.one_child[a.cur_par[v]] = v;
      }
    });
    const uint32_t ne = compact(
        x, a, live_n,
        [&](int64_t q) {
          const int32_t v = live[q];
          return a.alive[v] && v != root && a.cnt[v] == 1;
        },
        [&](int64_t q, uint32_t o) { a.elig[o] = live[q]; });
    // list ranking: distance of every unary node from the top of its path
    x.each([&](int t) {
      for (int64_t q = t; q < (int64_t)ne; q += T) a.sel[a.elig[q]] = 2;
    });
    x.each([&](int t) {
      for (int64_t q = t; q < (int64_t)ne; q += T) {
        const int32_t v = a.elig[q], p = a.cur_par[v];
        const bool up = a.sel[p] == 2;
        a.up0[v] = up ? p : v;
        a.dist0[v] = up ? 1 : 0;
      }
    });
    {
      int32_t *u = a.up0, *d = a.dist0, *u2 = a.up1, *d2 = a.dist1;
      for (int it = 0; it < 64; ++it) {
        const bool ch = x.any([&](int t) {
          bool c = false;
          for (int64_t q = t; q < (int64_t)ne; q += T) {
            const int32_t v = a.elig[q], w = u[v];
            d2[v] = d[v] + d[w];
            u2[v] = u[w];
            c |= u2[v] != w;
          }
          return c;
        });
        int32_t *tu = u, *td = d;
        u = u2;
        d = d2;
        u2 = tu;
        d2 = td;
        if (!ch) break;
      }
      x.each([&](int t) {
        for (int64_t q = t; q < (int64_t)ne; q += T) a.sel[a.elig[q]] = (d[a.elig[q]] & 1) == 0 ? 1 : 0;
      });
    }
    // compressions of the selected nodes, in increasing id
    const uint32_t nc = compact(
        x, a, ne, [&](int64_t q) { return a.sel[a.elig[q]] == 1; },
        [&](int64_t q, uint32_t o) { a.comp[o] = a.elig[q]; });
    x.each([&](int t) {
      if (t == 0) {
        a.r_comp_rem[rnd] = rem_n;
        a.r_comp_raw[rnd] = raw_n;
      }
      for (int64_t q = t; q < (int64_t)nc; q += T) {
        const int32_t j = a.comp[q], i = a.cur_par[j], k = a.one_child[j];
        int32_t lv = a.lvlU[j] > a.lvlE[k] ? a.lvlU[j] : a.lvlE[k];
        lv = 1 + (a.lvlE[j] > lv ? a.lvlE[j] : lv);
        const int32_t s = next_slot + (int32_t)q;
        a.raw[raw_n + q] = OpRec{OP_COMPRESS, rnd, lv, j, a.edge_slot[j], a.edge_slot[k], s, k};
        a.rem_kind[j] = 2;
        a.rem_slot[j] = a.edge_slot[j];
        a.rem_par[j] = i;
        a.comp_r[j] = a.edge_slot[k];
        a.comp_k[j] = k;
        a.removal[rem_n + q] = j;
        a.edge_slot[k] = s;
        a.lvlE[k] = lv;
        a.cur_par[k] = i;
        a.pos[k] = a.pos[j];
        a.alive[j] = 0;
      }
    });
    next_slot += (int32_t)nc;
    raw_n += (int32_t)nc;
    rem_n += (int32_t)nc;
    n_compress += nc;
    x.each([&](int t) {
      for (int64_t q = t; q < (int64_t)ne; q += T) a.sel[a.elig[q]] = 0;
    });
    live_n = compact(
        x, a, live_n, [&](int64_t q) { return a.alive[live[q]] != 0; },
        [&](int64_t q, uint32_t o) { live_next[o] = live[q]; });
    int32_t *tl = live;
    live = live_next;
    live_next = tl;
  }
  const int32_t rounds = rnd;
  x.each([&](int t) {
    if (t == 0) {
      a.r_raw[rounds + 1] = raw_n;
      a.r_rem[rounds + 1] = rem_n;
    }
  });

  // ---- contraction levels: ops by (level, kind), stable in creation order
  uint32_t *k = a.k0, *v = a.v0, *k2 = a.k1, *v2 = a.v1;
  const int32_t L = x.maxall([&](int t) {
    int32_t m = 0;
    for (int64_t i = t; i < raw_n; i += T) m = a.raw[i].level > m ? a.raw[i].level : m;
    return m;
  });
  x.each([&](int t) {
    for (int64_t i = t; i < raw_n; i += T) {
      k[i] = (uint32_t)((a.raw[i].level - 1) * 4 + a.raw[i].kind);
      v[i] = (uint32_t)i;
    }
  });
  radix_sort(x, a, raw_n, bitlen((uint64_t)(4 * (int64_t)L)), k, v, k2, v2);
  x.each([&](int t) {
    for (int64_t q = t; q < raw_n; q += T) a.ops[q] = a.raw[v[q]];
  });
  bucket_offsets(x, a, k, raw_n, 4 * (int64_t)L, a.off4);
  x.each([&](int t) {
    for (int64_t l = t; l <= L; l += T) a.lvl_off[l] = a.off4[4 * l];
    for (int64_t l = t; l < L; l += T)
      for (int s = 0; s <= 4; ++s) a.kind_off[5 * l + s] = a.off4[4 * l + s];
  });

  // ---- expansion of compressions: level 1 + that of the child's value, stable in removal order
  for (int32_t r = rounds; r >= 1; --r)
    x.each([&](int t) {
      for (int64_t q = a.r_comp_rem[r] + t; q < a.r_rem[r + 1]; q += T) {
        const int32_t j = a.removal[q];
        a.eP[j] = 1 + a.eP[a.comp_k[j]];
      }
    });
  const int32_t LE = x.maxall([&](int t) {
    int32_t m = 0;
    for (int64_t i = t; i < N; i += T) m = a.eP[i] > m ? a.eP[i] : m;
    return m;
  });
  const uint32_t n_exp = compact(
      x, a, rem_n, [&](int64_t q) { return a.rem_kind[a.removal[q]] == 2; },
      [&](int64_t q, uint32_t o) {
        const int32_t j = a.removal[q];
        k[o] = (uint32_t)(a.eP[j] - 1);
        v[o] = (uint32_t)j;
      });
  radix_sort(x, a, n_exp, bitlen((uint64_t)LE), k, v, k2, v2);
  x.each([&](int t) {
    for (int64_t q = t; q < (int64_t)n_exp; q += T) {
      const int32_t j = (int32_t)v[q];
      a.exp_ops[q] = Op4{j, a.comp_r[j], a.comp_k[j], 0};
    }
  });
  bucket_offsets(x, a, k, n_exp, LE, a.exp_off);

  // ---- composition of edge maps along compressions, stable in creation order
  x.each([&](int t) {
    for (int64_t s = t; s < next_slot; s += T) a.lT[s] = 0;
  });
  for (int32_t r = 1; r <= rounds; ++r)
    x.each([&](int t) {
      for (int64_t q = a.r_comp_raw[r] + t; q < a.r_raw[r + 1]; q += T) {
        const OpRec o = a.raw[q];
        a.lT[o.d] = 1 + (a.lT[o.b] > a.lT[o.c] ? a.lT[o.b] : a.lT[o.c]);
      }
    });
  const int32_t LT = x.maxall([&](int t) {
    int32_t m = 0;
    for (int64_t s = t; s < next_slot; s += T) m = a.lT[s] > m ? a.lT[s] : m;
    return m;
  });
  const uint32_t n_tc = compact(
      x, a, raw_n, [&](int64_t q) { return a.raw[q].kind == OP_COMPRESS; },
      [&](int64_t q, uint32_t o) {
        k[o] = (uint32_t)(a.lT[a.raw[q].d] - 1);
        v[o] = (uint32_t)q;
      });
  radix_sort(x, a, n_tc, bitlen((uint64_t)LT), k, v, k2, v2);
  x.each([&](int t) {
    for (int64_t q = t; q < (int64_t)n_tc; q += T) {
      const OpRec o = a.raw[v[q]];
      a.tc_ops[q] = Op4{o.b, o.c, o.d, o.a};
    }
  });
  bucket_offsets(x, a, k, n_tc, LT, a.tc_off);

  // ---- state expansion: 1 + the level of the parent at removal, stable in removal order
  for (int32_t r = rounds; r >= 1; --r) {
    x.each([&](int t) {  // the round's compressions come after its rakes in removal order
      for (int64_t q = a.r_comp_rem[r] + t; q < a.r_rem[r + 1]; q += T) {
        const int32_t j = a.removal[q];
        a.eX[j] = 1 + a.eX[a.rem_par[j]];
      }
    });
    x.each([&](int t) {
      for (int64_t q = a.r_rem[r] + t; q < a.r_comp_rem[r]; q += T) {
        const int32_t j = a.removal[q];
        a.eX[j] = 1 + a.eX[a.rem_par[j]];
      }
    });
  }
  const int32_t LX = x.maxall([&](int t) {
    int32_t m = 0;
    for (int64_t i = t; i < N; i += T) m = a.eX[i] > m ? a.eX[i] : m;
    return m;
  });
  x.each([&](int t) {
    for (int64_t q = t; q < rem_n; q += T) {
      const int32_t j = a.removal[q];
      k[q] = (uint32_t)(a.eX[j] - 1);
      v[q] = (uint32_t)j;
    }
  });
  radix_sort(x, a, rem_n, bitlen((uint64_t)LX), k, v, k2, v2);
  x.each([&](int t) {
    for (int64_t q = t; q < rem_n; q += T) {
      const int32_t j = (int32_t)v[q];
      a.sx_ops[q] = Op4{j, a.rem_slot[j], a.rem_par[j], 0};
    }
  });
  bucket_offsets(x, a, k, rem_n, LX, a.sx_off);

  x.each([&](int t) {
    if (t == 0) {
      a.stats[S_ROUNDS] = rounds;
      a.stats[S_RAKE] = n_rake;
      a.stats[S_COMPRESS] = n_compress;
      a.stats[S_COMBINE] = n_combine;
      a.stats[S_ABSORB] = n_absorb;
      a.stats[S_CONTRIB] = next_contrib;
      a.stats[S_SLOTS] = next_slot;
      a.stats[S_OPS] = raw_n;
      a.stats[S_L] = L;
      a.stats[S_EXP] = n_exp;
      a.stats[S_LE] = LE;
      a.stats[S_TC] = n_tc;
      a.stats[S_LT] = LT;
      a.stats[S_SX] = rem_n;
      a.stats[S_LX] = LX;
    }
  });
  return 0;
}

// Sequential executor: the threads of each phase one after the other, in the
// order `order` gives (0 increasing, 1 decreasing, 2 odd then even).
struct CpuExec {
  int T = THREADS, order = 0;
  int tid(int k) const {
    if (order == 1) return T - 1 - k;
    if (order == 2) {
      const int odd = T / 2;
      return k < odd ? 2 * k + 1 : 2 * (k - odd);
    }
    return k;
  }
  template <class F>
  void each(F f) {
    for (int k = 0; k < T; ++k) f(tid(k));
  }
  template <class F>
  bool any(F f) {
    bool r = false;
    for (int k = 0; k < T; ++k) r = f(tid(k)) || r;
    return r;
  }
  template <class F>
  int32_t maxall(F f) {
    int32_t m = INT32_MIN;
    for (int k = 0; k < T; ++k) {
      const int32_t v = f(tid(k));
      m = v > m ? v : m;
    }
    return m;
  }
  uint32_t scan(uint32_t *a) {
    uint32_t s = 0;
    for (int t = 0; t < T; ++t) {
      const uint32_t c = a[t];
      a[t] = s;
      s += c;
    }
    return s;
  }
  uint64_t scan64(uint64_t *a) {
    uint64_t s = 0;
    for (int t = 0; t < T; ++t) {
      const uint64_t c = a[t];
      a[t] = s;
      s += c;
    }
    return s;
  }
  void atomic_add(int32_t *p, int32_t v) { *p += v; }

  // Thread t takes the contiguous chunk [t C, (t + 1) C) of the indices.
  template <class P, class W>
  uint32_t compact(const Arena &a, int64_t n, P pred, W write) {
    const int64_t C = (n + T - 1) / T;
    each([&](int t) {
      const int64_t b = t * C, e = b + C < n ? b + C : n;
      uint32_t c = 0;
      for (int64_t i = b; i < e; ++i) c += pred(i) ? 1u : 0u;
      a.tcount[t] = c;
    });
    const uint32_t total = scan(a.tcount);
    each([&](int t) {
      const int64_t b = t * C, e = b + C < n ? b + C : n;
      uint32_t o = a.tcount[t];
      for (int64_t i = b; i < e; ++i)
        if (pred(i)) write(i, o++);
    });
    return total;
  }

  // One stable pass on digit (k >> sh) & 15 from (kk, vv) into (kd, vd):
  // per-thread digit counts over contiguous chunks, scanned digit-major.
  void radix_pass(const Arena &a, int64_t n, int sh, const uint32_t *kk, const uint32_t *vv, uint32_t *kd,
                  uint32_t *vd) {
    const int64_t C = (n + T - 1) / T;
    each([&](int t) {
      uint32_t h[16] = {0};
      const int64_t b = t * C, e = b + C < n ? b + C : n;
      for (int64_t i = b; i < e; ++i) h[(kk[i] >> sh) & 15]++;
      for (int d = 0; d < 16; ++d) a.hist[(size_t)d * T + t] = h[d];
    });
    each([&](int t) {  // thread t owns the digit-major entries [16 t, 16 t + 16)
      uint32_t s = 0;
      for (int j = 0; j < 16; ++j) {
        const uint32_t c = a.hist[(size_t)16 * t + j];
        a.hist[(size_t)16 * t + j] = s;
        s += c;
      }
      a.tcount[t] = s;
    });
    scan(a.tcount);
    each([&](int t) {
      for (int j = 0; j < 16; ++j) a.hist[(size_t)16 * t + j] += a.tcount[t];
    });
    each([&](int t) {
      uint32_t o[16];
      for (int d = 0; d < 16; ++d) o[d] = a.hist[(size_t)d * T + t];
      const int64_t b = t * C, e = b + C < n ? b + C : n;
      for (int64_t i = b; i < e; ++i) {
        const uint32_t p = o[(kk[i] >> sh) & 15]++;
        kd[p] = kk[i];
        vd[p] = vv[i];
      }
    });
  }
};

// Copies a finished run's statistics and schedules (host copies of the arena's
// outputs: `stats`, and the arrays at the sizes the statistics give) into a
// plan.
struct HostOut {
  int64_t stats[S_COUNT];
  std::vector<int32_t> par32;
  std::vector<OpRec> ops;
  std::vector<Op4> exp_ops, tc_ops, sx_ops;
  std::vector<int64_t> lvl_off, kind_off, exp_off, tc_off, sx_off;
};

inline void fill_plan(const HostOut &h, int64_t N, int n, int m, PlanHost &P) {
  P = PlanHost();
  P.N = N;
  P.n = n;
  P.m = m;
  P.selection = RCR_SELECT_LIST_RANK;
  P.root = h.stats[S_ROOT];
  P.height = h.stats[S_HEIGHT];
  P.leaves = h.stats[S_LEAVES];
  P.max_degree = h.stats[S_MAXDEG];
  P.rounds = h.stats[S_ROUNDS];
  P.n_rake = h.stats[S_RAKE];
  P.n_compress = h.stats[S_COMPRESS];
  P.n_combine = h.stats[S_COMBINE];
  P.n_absorb = h.stats[S_ABSORB];
  P.n_contrib = h.stats[S_CONTRIB];
  P.n_edge_slots = h.stats[S_SLOTS];
  P.parent32 = h.par32;
  P.ops = h.ops;
  P.lvl_off = h.lvl_off;
  P.kind_off = h.kind_off;
  P.exp_ops = h.exp_ops;
  P.exp_off = h.exp_off;
  P.tc_ops = h.tc_ops;
  P.tc_off = h.tc_off;
  P.sx_ops = h.sx_ops;
  P.sx_off = h.sx_off;
}

// Element counts of the output arrays of a finished run.
struct OutSizes {
  size_t ops, lvl, kind, exp, exp_off, tc, tc_off, sx, sx_off;
};
inline OutSizes out_sizes(const int64_t *s) {
  return OutSizes{(size_t)s[S_OPS], (size_t)s[S_L] + 1, 5 * (size_t)s[S_L], (size_t)s[S_EXP], (size_t)s[S_LE] + 1,
                  (size_t)s[S_TC],  (size_t)s[S_LT] + 1, (size_t)s[S_SX], (size_t)s[S_LX] + 1};
}

// The planner run on the host by CpuExec over host arrays (the same program
// the GPU runs), for checking the program itself without a GPU; big_group
// sets the size above which sibling groups take the workgroup-wide build.
inline int emulate(const int64_t *parent, int64_t N, int n, int m, int T, int order, PlanHost &P,
                   int32_t big_group = BIG_GROUP) {
  if (!parent) return RCR_NULL_ARG;
  if (N < 1 || n < 1 || m < 1 || n > RCR_MAX_DIM || m > RCR_MAX_DIM) return RCR_BAD_DIMS;
  if (N > (int64_t)(INT32_MAX / 2 - 16)) return RCR_BAD_DIMS;
  Arena a;
  const size_t bytes = carve(a, nullptr, N, T);
  std::vector<uint64_t> mem(bytes / 8 + 1);
  carve(a, reinterpret_cast<char *>(mem.data()), N, T);
  a.parent = parent;
  a.big_group = big_group;
  CpuExec x;
  x.T = T;
  x.order = order;
  const int32_t rc = program(x, a);
  if (rc) return rc;
  HostOut h;
  memcpy(h.stats, a.stats, sizeof(h.stats));
  const OutSizes z = out_sizes(a.stats);
  h.par32.assign(a.par32, a.par32 + N);
  h.ops.assign(a.ops, a.ops + z.ops);
  h.lvl_off.assign(a.lvl_off, a.lvl_off + z.lvl);
  h.kind_off.assign(a.kind_off, a.kind_off + z.kind);
  h.exp_ops.assign(a.exp_ops, a.exp_ops + z.exp);
  h.exp_off.assign(a.exp_off, a.exp_off + z.exp_off);
  h.tc_ops.assign(a.tc_ops, a.tc_ops + z.tc);
  h.tc_off.assign(a.tc_off, a.tc_off + z.tc_off);
  h.sx_ops.assign(a.sx_ops, a.sx_ops + z.sx);
  h.sx_off.assign(a.sx_off, a.sx_off + z.sx_off);
  fill_plan(h, N, n, m, P);
  return 0;
}

}  // namespace dplan
}  // namespace rcr
