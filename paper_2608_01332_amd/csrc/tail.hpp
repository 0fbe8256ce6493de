// Single-workgroup "tail" kernels for the narrow dependency levels.
//
// Near the root the contraction levels hold only a few primitives, and so do
// the first levels of the reverse expansion.  Launching one kernel per such
// level costs a launch plus a round trip through memory that another XCD
// wrote.  A tail kernel instead runs a contiguous range of narrow levels -- the
// end of a contraction pass followed by the beginning of its expansion --
// inside one workgroup: every wavefront takes primitives of the current level
// in turn, and consecutive levels are separated by a workgroup barrier
// (workgroup-scope release/acquire), so the dependency order of the plan is
// kept while the data stays in one CU's caches.
#pragma once

#include "kernels.hpp"
#include "wide.hpp"

namespace rcr {

template <int NB>
struct MatLay {
  static constexpr bool WIDE = NB >= 12;
  static constexpr int PW = WIDE ? 1 : TeamW<NB>::PW;  // primitives per wavefront
  static constexpr int TW = WIDE ? 64 : TeamW<NB>::TW;
  static constexpr int MAXW = WIDE ? 16 : 8;           // wavefronts per tail workgroup
  template <typename T>
  static constexpr int lw() {
    if constexpr (WIDE)
      return wide_lds_words<T, NB>();
    else
      return lds_quad_words<T, NB>();
  }
};

#define RCR_TAIL_MAT_KERNEL(NBV) \
  __global__ __attribute__((amdgpu_flat_work_group_size(64, 64 * MatLay<NBV>::MAXW)))

// Quadratic contraction levels [t0, t1) then quadratic expansion levels [e0, e1).
template <typename T, int NB>
RCR_TAIL_MAT_KERNEL(NB) void k_tail_quad(Bufs<T> bf, const OpRec *__restrict__ ops, const int64_t *__restrict__ koff,
                                         int t0, int t1, const Op4 *__restrict__ eops,
                                         const int64_t *__restrict__ eoff, int e0, int e1) {
  using Lay = MatLay<NB>;
  extern __shared__ double smd[];
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int team = Lay::WIDE ? 0 : lane / Lay::TW, r = Lay::WIDE ? 0 : lane % Lay::TW;
  const int nslot = nw * Lay::PW;
  T *L = reinterpret_cast<T *>(smd) + (size_t)(wave * Lay::PW + team) * Lay::template lw<T>();
  for (int t = t0; t < t1; ++t) {
    const int64_t beg = koff[(size_t)t * 5], end = koff[(size_t)t * 5 + 4];
    for (int64_t base = beg + wave * Lay::PW; base < end; base += nslot) {
      const int64_t i = base + team;
      const bool active = i < end;
      const OpRec o = ops[active ? i : end - 1];
      if constexpr (Lay::WIDE)
        quad_op_wide<T, NB>(bf, o, o.kind, L);
      else
        quad_op_team<T, NB>(bf, o, o.kind, L, r, active);
    }
    __syncthreads();
  }
  for (int e = e0; e < e1; ++e) {
    const int64_t beg = eoff[e], end = eoff[e + 1];
    for (int64_t base = beg + wave * Lay::PW; base < end; base += nslot) {
      const int64_t i = base + team;
      const bool active = i < end;
      const Op4 o = eops[active ? i : end - 1];
      if constexpr (Lay::WIDE)
        qexp_op_wide<T, NB>(bf, o, L);
      else
        qexp_op_team<T, NB>(bf, o, L, r, active);
    }
    __syncthreads();
  }
}

// Composite-transition levels [t0, t1).
template <typename T, int NB>
RCR_TAIL_MAT_KERNEL(NB) void k_tail_tc(Bufs<T> bf, const Op4 *__restrict__ ops, const int64_t *__restrict__ off,
                                       int t0, int t1) {
  using Lay = MatLay<NB>;
  extern __shared__ double smd[];
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int team = Lay::WIDE ? 0 : lane / Lay::TW, r = Lay::WIDE ? 0 : lane % Lay::TW;
  const int nslot = nw * Lay::PW;
  T *L = reinterpret_cast<T *>(smd) + (size_t)(wave * Lay::PW + team) * Lay::template lw<T>();
  for (int t = t0; t < t1; ++t) {
    const int64_t beg = off[t], end = off[t + 1];
    for (int64_t base = beg + wave * Lay::PW; base < end; base += nslot) {
      const int64_t i = base + team;
      const bool active = i < end;
      const Op4 o = ops[active ? i : end - 1];
      if constexpr (Lay::WIDE)
        tcomp_op_wide<T, NB>(bf, o, L);
      else
        tcomp_op_team<T, NB>(bf, o, L, r, active);
    }
    __syncthreads();
  }
}

// Affine contraction levels [t0, t1) then affine expansion levels [e0, e1).
template <typename T, int NB>
__global__ __launch_bounds__(1024) void k_tail_aff(Bufs<T> bf, const OpRec *__restrict__ ops,
                                                   const int64_t *__restrict__ koff, int t0, int t1,
                                                   const Op4 *__restrict__ eops, const int64_t *__restrict__ eoff,
                                                   int e0, int e1) {
  constexpr int TW = TeamW<NB>::TW;
  const int slot = threadIdx.x / TW, nslot = blockDim.x / TW, r = threadIdx.x % TW;
  for (int t = t0; t < t1; ++t) {
    const int64_t beg = koff[(size_t)t * 5], end = koff[(size_t)t * 5 + 4];
    for (int64_t i = beg + slot; i < end; i += nslot) {
      const OpRec o = ops[i];
      aff_op<T, NB>(bf, o, o.kind, r);
    }
    __syncthreads();
  }
  for (int e = e0; e < e1; ++e) {
    for (int64_t i = eoff[e] + slot; i < eoff[e + 1]; i += nslot) affexp_op<T, NB>(bf, eops[i], r);
    __syncthreads();
  }
}

// State-offset composition levels [t0, t1) then state expansion levels [e0, e1).
template <typename T, int NB>
__global__ __launch_bounds__(1024) void k_tail_state(Bufs<T> bf, const Op4 *__restrict__ ops,
                                                     const int64_t *__restrict__ off, int t0, int t1,
                                                     const Op4 *__restrict__ xops, const int64_t *__restrict__ xoff,
                                                     int e0, int e1) {
  constexpr int TW = TeamW<NB>::TW;
  const int slot = threadIdx.x / TW, nslot = blockDim.x / TW, r = threadIdx.x % TW;
  for (int t = t0; t < t1; ++t) {
    for (int64_t i = off[t] + slot; i < off[t + 1]; i += nslot) state_op<T, NB>(bf, ops[i], r);
    __syncthreads();
  }
  for (int e = e0; e < e1; ++e) {
    for (int64_t i = xoff[e] + slot; i < xoff[e + 1]; i += nslot) sexp_op<T, NB>(bf, xops[i], r);
    __syncthreads();
  }
}

}  // namespace rcr
