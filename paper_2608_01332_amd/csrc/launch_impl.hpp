// Launch sequence of one factor + solve for a padded block size NB.  Each
// instantiation lives in its own translation unit (inst*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "device.hpp"
#include "kernels.hpp"
#include "lfwide.hpp"
#include "tail.hpp"
#include "wideops.hpp"

namespace rcr {

#ifndef HIPCK
#define HIPCK(x)                                                                                      \
  do {                                                                                                \
    hipError_t e_ = (x);                                                                              \
    if (e_ != hipSuccess) {                                                                           \
      fprintf(stderr, "rcr: %s failed: %s (%s:%d)\n", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      return RCR_HIP_ERROR;                                                                           \
    }                                                                                                 \
  } while (0)
#endif

inline unsigned blocks_for(int64_t cnt, int per) { return (unsigned)((cnt + per - 1) / per); }

// Optional HIP event timing on the launch stream, in one of two modes:
//  - per launch (per-level executor): consecutive launches share their
//    boundary events, so a launch's span is its execution plus one marker;
//  - per class run (graph capture): no event is recorded; `split(c)` is
//    called where the kernel class changes to c, so the caller can end the
//    captured graph there and start the next one.
struct Timer {
  PlanObj *P = nullptr;
  hipStream_t st = nullptr;
  bool on = false;
  void (*split)(void *, int) = nullptr;  // per-class-run mode
  void *split_arg = nullptr;
  int run = -2;  // class of the current run (per-class-run mode)
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> spans;
  int launches[RCR_NUM_KERNEL_CLASSES] = {};
  size_t used = 0;
  int cls = 0;
  hipEvent_t last = nullptr;  // boundary after the previous timed launch
  hipEvent_t ev() {
    if (used == P->events.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      P->events.push_back(e);
    }
    return P->events[used++];
  }
  void begin(int c) { cls = c; }
  void end() {}
  void pre() {
    if (!on) return;
    launches[cls] += 1;
    if (split) {
      if (run != cls) {
        split(split_arg, cls);
        run = cls;
      }
      return;
    }
    if (!last) {
      if (!(last = ev())) return;
      (void)hipEventRecord(last, st);
    }
    hipEvent_t b = ev();
    if (!b) return;
    spans.push_back({cls, {last, b}});
  }
  void post() {
    if (!on || split || spans.empty()) return;
    (void)hipEventRecord(spans.back().second.second, st);
    last = spans.back().second.second;
  }
  // an untimed launch follows: the next timed launch starts a new boundary
  // (per-class-run mode: a new run)
  void gap() {
    last = nullptr;
    if (on && split && run != -1) {
      split(split_arg, -1);
      run = -1;
    }
  }
};

#define LAUNCH(tm, ...)          \
  do {                           \
    (tm).pre();                  \
    hipLaunchKernelGGL(__VA_ARGS__); \
    (tm).post();                 \
  } while (0)

// Narrow ranges run by the single-workgroup tail kernels: contraction levels
// [c_begin, nc) whose widths are all <= cap, then expansion levels [0, e_end)
// whose widths are all <= cap.  Empty when fewer than two levels qualify.
struct TailRange {
  int c_begin, c_end, e_begin, e_end;
  int levels() const { return (c_end - c_begin) + (e_end - e_begin); }
};
inline TailRange tail_range(const std::vector<int64_t> &coff, int kstride, int kend,
                            const std::vector<int64_t> *eoff, int64_t cap) {
  const int nc = (int)((coff.size() - (kstride == 1 ? 1 : 0)) / kstride);
  auto ccount = [&](int t) {
    return kstride == 1 ? coff[t + 1] - coff[t] : coff[(size_t)t * kstride + kend] - coff[(size_t)t * kstride];
  };
  int cb = nc;
  while (cb > 0 && ccount(cb - 1) <= cap) --cb;
  int ee = 0;
  if (eoff) {
    const int ne = (int)eoff->size() - 1;
    while (ee < ne && (*eoff)[ee + 1] - (*eoff)[ee] <= cap) ++ee;
  }
  TailRange tr{cb, nc, 0, ee};
  if (tr.levels() < 2) tr = TailRange{nc, nc, 0, 0};
  return tr;
}

// LDS image of a vector tail (vec_tail_bytes) and the shrinking of its range
// to an LDS budget: the wider boundary level leaves the tail first.
inline size_t vec_tail_lds(const TailRange &tr, const std::vector<int64_t> &coff, int cstride, int cend, size_t rc,
                           const std::vector<int64_t> &eoff) {
  const int nc = tr.c_end - tr.c_begin, ne = tr.e_end - tr.e_begin;
  const int64_t ncops = nc ? coff[(size_t)(tr.c_end - 1) * cstride + cend] - coff[(size_t)tr.c_begin * cstride] : 0;
  const int64_t neops = eoff[tr.e_end] - eoff[tr.e_begin];
  return (size_t)16 * (nc + ne) + rc * (size_t)ncops + 16 * (size_t)neops;
}
inline TailRange fit_vec_tail(TailRange tr, const std::vector<int64_t> &coff, int cstride, int cend, size_t rc,
                              const std::vector<int64_t> &eoff, size_t budget) {
  while (tr.levels() >= 2 && vec_tail_lds(tr, coff, cstride, cend, rc, eoff) > budget) {
    const int64_t cw = tr.c_end > tr.c_begin ? coff[(size_t)tr.c_begin * cstride + cend] -
                                                    coff[(size_t)tr.c_begin * cstride]
                                              : -1;
    const int64_t ew = tr.e_end > tr.e_begin ? eoff[tr.e_end] - eoff[tr.e_end - 1] : -1;
    if (cw >= ew)
      ++tr.c_begin;
    else
      --tr.e_end;
  }
  if (tr.levels() < 2) tr = TailRange{tr.c_end, tr.c_end, 0, 0};
  return tr;
}

template <typename K>
inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Launch one phase for working type T and padded sizes (NB, MB) on `st`:
// phase 0 = factor (Algorithm 1, Steps 2-3), phase 1 = solve (Steps 4-6).
// RCR_PHASE_FIRST_RHS on both phases of one solve lets the local factor also
// initialise the solve of the right-hand side in bf (its W, A^cl and K^T are
// still in LDS or registers there), and the solve phase then skips rhs_init.
template <typename T, int NB, int MB>
int launch_phase_nb(PlanObj &P, Bufs<T> bf, Timer &tm, hipStream_t st, int phase_flags) {
  const PlanHost &h = P.host;
  const int phase = phase_flags & 3;
  constexpr int PW = TeamW<NB>::PW;
  constexpr int NM = NB > MB ? NB : MB;
  constexpr int PWm = TeamW<NM>::PW;
  constexpr bool WIDE = MatLay<NB>::WIDE;  // one primitive per wavefront for the level kernels
  const bool fused_rhs = (phase_flags & RCR_PHASE_FIRST_RHS) != 0;
  // local factor flags: 1 initialise the first right-hand side, 2 do not store A^cl
  const int lf_flags = (fused_rhs ? 1 : 0) | (fused_rhs && (phase_flags & RCR_PHASE_ONE_RHS) ? 2 : 0);
  const size_t lds_cond = (size_t)PW * CondLay<NB, MB>::words * sizeof(double);
  const size_t lds_quad = (size_t)PW * lds_quad_words<T, NB>() * sizeof(T);
  const size_t lds_lf = (size_t)PW * LfLay<T, NB, MB>::words * sizeof(double);
  const size_t lds_lfw = (size_t)LfwLay<T, (NB >= 12 ? NB : 12), MB>::words * sizeof(double);
  const size_t lds_rhs = (size_t)PW * team_stride<T>(RhsLay<NB, MB>::words) * sizeof(T);
  const size_t lds_la = (size_t)PWm * team_stride<T>(LaLay<NB, MB>::words) * sizeof(T);
  const size_t lds_rec = (size_t)PW * team_stride<T>(RecLay<NB, MB>::words) * sizeof(T);
  allow_lds(k_condense<T, NB, MB>, lds_cond);
  allow_lds(k_local_factor<T, NB, MB>, lds_lf);
  allow_lds(k_rhs_init<T, NB, MB>, lds_rhs);
  allow_lds(k_local_affine<T, NB, MB>, lds_la);
  allow_lds(k_recover<T, NB, MB>, lds_rec);
  const size_t lds_wide = (size_t)wide_lds_words<T, (NB >= 12 ? NB : 12)>() * sizeof(T);
  const size_t lds_wexp = (size_t)tau_lds_words<T, (NB >= 12 ? NB : 12)>() * sizeof(T);
  const size_t lds_wtc = (size_t)2 * WideCfg<(NB >= 12 ? NB : 12)>::BS * sizeof(T);
  const size_t lds_lvl = WIDE ? lds_wide : lds_quad;  // per wavefront, level kernels
  const unsigned NBk = blocks_for(h.N, PW);
  // tail workgroup sizes
  const size_t kMaxLds = 156 * 1024;
  int mat_waves = (int)std::min<size_t>(MatLay<NB>::MAXW, kMaxLds / lds_lvl);
  if (mat_waves < 1) mat_waves = 1;
  const size_t lds_tail = (size_t)mat_waves * lds_lvl;
  const LaunchCfg &cfg = P.cfg;
  // Defaults (fields left at 0), from timings of chain-probability trees of 1k
  // to 64k nodes: the quadratic tail pays off only in the wide layout, at one
  // round; the vector tails at two rounds in float64 and four in float32.
  const int qr = cfg.quad_tail_rounds == 0 ? (WIDE ? 1 : 0) : (cfg.quad_tail_rounds < 0 ? 0 : cfg.quad_tail_rounds);
  const int64_t mat_cap = (int64_t)qr * mat_waves * MatLay<NB>::PW;
  const int vec_waves = cfg.vec_tail_waves > 0 ? std::min(cfg.vec_tail_waves, 16) : 8;
  const int vr = cfg.vec_tail_rounds == 0 ? (sizeof(T) == 4 ? 4 : 2) : (cfg.vec_tail_rounds < 0 ? 0 : cfg.vec_tail_rounds);
  const int64_t vec_cap = (int64_t)vr * vec_waves * (64 / TeamW<NB>::TW);
  const size_t kVecTailLds = 144 * 1024;
  allow_lds(k_tail_quad<T, NB>, lds_tail);
  allow_lds(k_tail_tc<T, NB>, lds_tail);
  const TailRange tq = tail_range(h.kind_off, 5, 4, &h.exp_off, mat_cap);
  const TailRange ttc = tail_range(h.tc_off, 1, 1, nullptr, mat_cap);
  const TailRange ta = fit_vec_tail(tail_range(h.kind_off, 5, 4, &h.exp_off, vec_cap), h.kind_off, 5, 4,
                                    sizeof(OpRec), h.exp_off, kVecTailLds);
  const TailRange ts = fit_vec_tail(tail_range(h.tc_off, 1, 1, &h.sx_off, vec_cap), h.tc_off, 1, 1, sizeof(Op4),
                                    h.sx_off, kVecTailLds);
  const size_t lds_ta = vec_tail_lds(ta, h.kind_off, 5, 4, sizeof(OpRec), h.exp_off);
  const size_t lds_ts = vec_tail_lds(ts, h.tc_off, 1, 1, sizeof(Op4), h.sx_off);
  allow_lds(k_tail_aff<T, NB, 512>, lds_ta);
  allow_lds(k_tail_aff<T, NB, 1024>, lds_ta);
  allow_lds(k_tail_state<T, NB, 512>, lds_ts);
  allow_lds(k_tail_state<T, NB, 1024>, lds_ts);

  auto seg_of = [&](int64_t t, Seg &sg, int per) {
    unsigned total = 0;
    for (int s = 0; s <= 4; ++s) sg.off[s] = h.kind_off[(size_t)t * 5 + s];
    sg.blk[0] = 0;
    for (int s = 0; s < 4; ++s) {
      total += blocks_for(sg.off[s + 1] - sg.off[s], per);
      sg.blk[s + 1] = (int32_t)total;
    }
    return total;
  };
  if (phase == 0) {
  // ---- condensation.  Wide layout, control size up to 4: condensed in the
  // wide layout, where level 1 (launched on its own) does it for its own
  // edges and the rest in the same launch; U is never copied from Q (readers
  // of a node that no absorb has touched read Q).  Otherwise the team-layout
  // kernel, which also copies U = Q.
  int64_t t_first = 0;
  if constexpr (WIDE && MB == 4) {
    if (P.dev.l1_fusable && tq.c_begin > 0) {
      const int64_t r0 = h.kind_off[0], nr = h.kind_off[1] - r0, c0 = h.kind_off[3], nc = h.kind_off[4] - c0;
      tm.begin(RCR_K_QUAD_CONTRACT);
      allow_lds(k_level1_wide<T, NB>, lds_wide);
      LAUNCH(tm, (k_level1_wide<T, NB>), dim3((unsigned)(nr + nc + P.dev.n_rest)), dim3(64), lds_wide, st, bf,
             P.dev.ops, r0, (int)nr, c0, (int)nc, P.dev.rest);
      t_first = 1;
    } else {
      tm.begin(RCR_K_CONDENSE);
      LAUNCH(tm, (k_condense_wide<T, NB>), dim3((unsigned)h.N), dim3(64), 0, st, bf);
    }
  } else {
    tm.begin(RCR_K_CONDENSE);
    LAUNCH(tm, (k_condense<T, NB, MB>), dim3(NBk), dim3(64), lds_cond, st, bf);
  }

  // ---- quadratic contraction and expansion
  tm.begin(RCR_K_QUAD_CONTRACT);
  for (int64_t t = t_first; t < tq.c_begin; ++t) {
    Seg sg;
    if constexpr (WIDE) {
      const unsigned nb = seg_of(t, sg, 1);
      if (nb) LAUNCH(tm, (k_quad_level_wide<T, NB>), dim3(nb), dim3(64), lds_wide, st, bf, P.dev.ops, sg);
    } else {
      const unsigned nb = seg_of(t, sg, PW);
      if (nb) LAUNCH(tm, (k_quad_level<T, NB>), dim3(nb), dim3(64), lds_quad, st, bf, P.dev.ops, sg);
    }
  }
  if (tq.levels() > 0) {
    tm.begin(RCR_K_QUAD_TAIL);
    LAUNCH(tm, (k_tail_quad<T, NB>), dim3(1), dim3(64 * mat_waves), lds_tail, st, bf, P.dev.ops, P.dev.koff,
           tq.c_begin, tq.c_end, P.dev.exp_ops, P.dev.exp_off, tq.e_begin, tq.e_end);
  }
  tm.begin(RCR_K_QUAD_EXPAND);
  for (int64_t t = tq.e_end; t < h.expand_levels(); ++t) {
    const int64_t cnt = h.exp_off[t + 1] - h.exp_off[t];
    if (cnt <= 0) continue;
    if constexpr (WIDE)
      LAUNCH(tm, (k_quad_expand_wide<T, NB>), dim3((unsigned)cnt), dim3(64), lds_wexp, st, bf, P.dev.exp_ops,
             h.exp_off[t]);
    else
      LAUNCH(tm, (k_quad_expand<T, NB>), dim3(blocks_for(cnt, PW)), dim3(64), lds_quad, st, bf, P.dev.exp_ops,
             h.exp_off[t], cnt);
  }
  tm.begin(RCR_K_LOCAL_FACTOR);
  if constexpr (WIDE) {
    allow_lds(k_local_factor_wide<T, NB, MB>, lds_lfw);
    LAUNCH(tm, (k_local_factor_wide<T, NB, MB>), dim3((unsigned)h.N), dim3(64), lds_lfw, st, bf, lf_flags);
  } else {
    LAUNCH(tm, (k_local_factor<T, NB, MB>), dim3(NBk), dim3(64), lds_lf, st, bf, lf_flags);
  }

  // ---- composite transitions along compressions (with the first right-hand
  // side, levels from 1 on run in the solve phase, merged with affine levels)
  tm.begin(RCR_K_TCOMPOSE);
  const int64_t tc_here = fused_rhs ? std::min<int64_t>(ttc.c_begin, 1) : ttc.c_begin;
  for (int64_t t = 0; t < tc_here; ++t) {
    const int64_t cnt = h.tc_off[t + 1] - h.tc_off[t];
    if (cnt <= 0) continue;
    if constexpr (WIDE)
      LAUNCH(tm, (k_tcompose_wide<T, NB>), dim3((unsigned)cnt), dim3(64), lds_wtc, st, bf, P.dev.tc_ops,
             h.tc_off[t]);
    else
      LAUNCH(tm, (k_tcompose<T, NB>), dim3(blocks_for(cnt, PW)), dim3(64), lds_quad, st, bf, P.dev.tc_ops,
             h.tc_off[t], cnt);
  }
  if (ttc.levels() > 0 && !fused_rhs)
    LAUNCH(tm, (k_tail_tc<T, NB>), dim3(1), dim3(64 * mat_waves), lds_tail, st, bf, P.dev.tc_ops, P.dev.tc_off,
           ttc.c_begin, ttc.c_end);

  } else {
  // ---- solve: affine contraction and expansion
  if (!fused_rhs) {
    tm.begin(RCR_K_RHS_INIT);
    LAUNCH(tm, (k_rhs_init<T, NB, MB>), dim3(NBk), dim3(64), lds_rhs, st, bf);
  }
  tm.begin(RCR_K_AFF_CONTRACT);
  int64_t ta0 = 0;  // first affine level not yet launched
  if (fused_rhs) {
    // composite-transition level i (left over from the factor phase) together
    // with affine level i - 1, which reads only composites of levels below i - 1
    const size_t lds_tcm = WIDE ? lds_wtc : lds_quad;
    for (int64_t i = 1; i < ttc.c_begin; ++i) {
      const int64_t tcnt = h.tc_off[i + 1] - h.tc_off[i];
      const unsigned tcb = tcnt <= 0 ? 0u : (WIDE ? (unsigned)tcnt : blocks_for(tcnt, PW));
      Seg sg{};
      unsigned nb = 0;
      if (ta0 == i - 1 && ta0 < ta.c_begin) nb = seg_of(ta0++, sg, PW);
      if (tcb + nb)
        LAUNCH(tm, (k_tc_aff_level<T, NB>), dim3(tcb + nb), dim3(64), lds_tcm, st, bf, P.dev.tc_ops, h.tc_off[i],
               tcnt, (int)tcb, P.dev.ops, sg);
    }
    if (ttc.levels() > 0) {
      tm.begin(RCR_K_TCOMPOSE);
      LAUNCH(tm, (k_tail_tc<T, NB>), dim3(1), dim3(64 * mat_waves), lds_tail, st, bf, P.dev.tc_ops, P.dev.tc_off,
             ttc.c_begin, ttc.c_end);
      tm.begin(RCR_K_AFF_CONTRACT);
    }
  }
  for (int64_t t = ta0; t < ta.c_begin; ++t) {
    Seg sg;
    const unsigned nb = seg_of(t, sg, PW);
    if (nb) LAUNCH(tm, (k_aff_level<T, NB>), dim3(nb), dim3(64), 0, st, bf, P.dev.ops, sg);
  }
  if (ta.levels() > 0) {
    tm.begin(RCR_K_AFF_TAIL);
    if (vec_waves <= 8)
      LAUNCH(tm, (k_tail_aff<T, NB, 512>), dim3(1), dim3(64 * vec_waves), lds_ta, st, bf, P.dev.ops, P.dev.koff,
             ta.c_begin, ta.c_end, P.dev.exp_ops, P.dev.exp_off, ta.e_begin, ta.e_end);
    else
      LAUNCH(tm, (k_tail_aff<T, NB, 1024>), dim3(1), dim3(64 * vec_waves), lds_ta, st, bf, P.dev.ops, P.dev.koff,
             ta.c_begin, ta.c_end, P.dev.exp_ops, P.dev.exp_off, ta.e_begin, ta.e_end);
  }
  tm.begin(RCR_K_AFF_EXPAND);
  for (int64_t t = ta.e_end; t < h.expand_levels(); ++t) {
    const int64_t cnt = h.exp_off[t + 1] - h.exp_off[t];
    if (cnt > 0)
      LAUNCH(tm, (k_aff_expand<T, NB>), dim3(blocks_for(cnt, PW)), dim3(64), 0, st, bf, P.dev.exp_ops,
             h.exp_off[t], cnt);
  }
  tm.begin(RCR_K_LOCAL_AFFINE);
  LAUNCH(tm, (k_local_affine<T, NB, MB>), dim3(blocks_for(h.N, PWm)), dim3(64), lds_la, st, bf);

  // ---- state offsets and state expansion
  tm.begin(RCR_K_STATE_CONTRACT);
  for (int64_t t = 0; t < ts.c_begin; ++t) {
    const int64_t cnt = h.tc_off[t + 1] - h.tc_off[t];
    if (cnt > 0)
      LAUNCH(tm, (k_state_level<T, NB>), dim3(blocks_for(cnt, PW)), dim3(64), 0, st, bf, P.dev.tc_ops,
             h.tc_off[t], cnt);
  }
  if (ts.levels() > 0) {
    tm.begin(RCR_K_STATE_TAIL);
    if (vec_waves <= 8)
      LAUNCH(tm, (k_tail_state<T, NB, 512>), dim3(1), dim3(64 * vec_waves), lds_ts, st, bf, P.dev.tc_ops,
             P.dev.tc_off, ts.c_begin, ts.c_end, P.dev.sx_ops, P.dev.sx_off, ts.e_begin, ts.e_end);
    else
      LAUNCH(tm, (k_tail_state<T, NB, 1024>), dim3(1), dim3(64 * vec_waves), lds_ts, st, bf, P.dev.tc_ops,
             P.dev.tc_off, ts.c_begin, ts.c_end, P.dev.sx_ops, P.dev.sx_off, ts.e_begin, ts.e_end);
  }
  tm.begin(RCR_K_STATE_EXPAND);
  for (int64_t t = ts.e_end; t < h.sexp_levels(); ++t) {
    const int64_t cnt = h.sx_off[t + 1] - h.sx_off[t];
    if (cnt > 0)
      LAUNCH(tm, (k_state_expand<T, NB>), dim3(blocks_for(cnt, PW)), dim3(64), 0, st, bf, P.dev.sx_ops,
             h.sx_off[t], cnt);
  }
  tm.begin(RCR_K_RECOVER);
  LAUNCH(tm, (k_recover<T, NB, MB>), dim3(NBk), dim3(64), lds_rec, st, bf);
  }
  HIPCK(hipGetLastError());
  return RCR_OK;
}

inline int pad_n(int n) { return n <= 4 ? 4 : n <= 6 ? 6 : n <= 8 ? 8 : n <= 12 ? 12 : 16; }
inline int pad_m(int m) { return m <= 4 ? 4 : m <= 8 ? 8 : 16; }

template <typename T, int NB>
int launch_phase_m(PlanObj &P, Bufs<T> bf, Timer &tm, hipStream_t st, int phase) {
  switch (pad_m(bf.m)) {
    case 4: return launch_phase_nb<T, NB, 4>(P, bf, tm, st, phase);
    case 8: return launch_phase_nb<T, NB, 8>(P, bf, tm, st, phase);
    default: return launch_phase_nb<T, NB, 16>(P, bf, tm, st, phase);
  }
}


}  // namespace rcr
