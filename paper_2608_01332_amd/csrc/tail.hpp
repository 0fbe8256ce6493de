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
#include "wideops.hpp"

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
__device__ __forceinline__ void tail_quad(const Bufs<T> &bf, const OpRec *__restrict__ ops,
                                          const int64_t *__restrict__ koff, int t0, int t1,
                                          const Op4 *__restrict__ eops, const int64_t *__restrict__ eoff, int e0,
                                          int e1) {
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

template <typename T, int NB>
RCR_TAIL_MAT_KERNEL(NB) void k_tail_quad(Bufs<T> bf, const OpRec *__restrict__ ops, const int64_t *__restrict__ koff,
                                         int t0, int t1, const Op4 *__restrict__ eops,
                                         const int64_t *__restrict__ eoff, int e0, int e1) {
  if (MatLay<NB>::WIDE && bf.n == NB)  // the primitives specialised for unpadded blocks
    tail_quad<T, NB>(exact_n<NB>(bf), ops, koff, t0, t1, eops, eoff, e0, e1);
  else
    tail_quad<T, NB>(bf, ops, koff, t0, t1, eops, eoff, e0, e1);
}

// Composite-transition levels [t0, t1).
template <typename T, int NB>
__device__ __forceinline__ void tail_tc(const Bufs<T> &bf, const Op4 *__restrict__ ops,
                                        const int64_t *__restrict__ off, int t0, int t1) {
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

template <typename T, int NB>
RCR_TAIL_MAT_KERNEL(NB) void k_tail_tc(Bufs<T> bf, const Op4 *__restrict__ ops, const int64_t *__restrict__ off,
                                       int t0, int t1) {
  if (MatLay<NB>::WIDE && bf.n == NB)
    tail_tc<T, NB>(exact_n<NB>(bf), ops, off, t0, t1);
  else
    tail_tc<T, NB>(bf, ops, off, t0, t1);
}

// ---------------------------------------------------------------- vector tails
// The affine and state passes run matrix-vector primitives whose matrices
// (the transitions T and their composites) are outputs of the factor, known
// before the pass starts.  Their tail kernels therefore (1) copy the level
// bounds and every op record of their levels into LDS once, and (2) prefetch,
// one level ahead, the matrix column (affine: Z = T^T) or row (state) that
// each team needs for its first primitive of the next level.  A level then
// costs one round trip for the vectors the previous level wrote, the
// arithmetic, and the workgroup barrier.
struct VecTailLds {
  int nl, nc;            // levels (contraction first), contraction levels
  int64_t cbase, ebase;  // first contraction / expansion op of the tail
  int64_t ncops, neops;
  size_t bytes;
};

// LDS image: int64 level bounds (2 per level, relative to the op arrays in
// LDS), then the contraction records (RC bytes each), then the expansion
// records (Op4).
template <int RC>
__host__ __device__ inline size_t vec_tail_bytes(int nl, int64_t ncops, int64_t neops) {
  return (size_t)16 * nl + (size_t)RC * ncops + sizeof(Op4) * neops;
}

// Copy the bounds and records into LDS (all threads), then barrier.
template <typename RecC>
__device__ __forceinline__ void vec_tail_stage(char *lds, const RecC *__restrict__ cops, const int64_t *__restrict__ coff,
                                               int cstride, int cend, int t0, int t1, const Op4 *__restrict__ eops,
                                               const int64_t *__restrict__ eoff, int e0, int e1, int64_t &cbase,
                                               int64_t &ebase, RecC *&lc, Op4 *&le, int64_t *&lb) {
  const int nc = t1 - t0, nl = nc + (e1 - e0);
  cbase = nc ? coff[(size_t)t0 * cstride] : 0;
  const int64_t cstop = nc ? coff[(size_t)(t1 - 1) * cstride + cend] : 0;
  ebase = eoff[e0];
  const int64_t estop = eoff[e1];
  lb = reinterpret_cast<int64_t *>(lds);
  lc = reinterpret_cast<RecC *>(lds + 16 * (size_t)nl);
  le = reinterpret_cast<Op4 *>(lds + 16 * (size_t)nl + sizeof(RecC) * (size_t)(cstop - cbase));
  for (int l = threadIdx.x; l < nl; l += blockDim.x) {
    if (l < nc) {
      lb[2 * l] = coff[(size_t)(t0 + l) * cstride] - cbase;
      lb[2 * l + 1] = coff[(size_t)(t0 + l) * cstride + cend] - cbase;
    } else {
      lb[2 * l] = eoff[e0 + l - nc] - ebase;
      lb[2 * l + 1] = eoff[e0 + l - nc + 1] - ebase;
    }
  }
  // records as 16-byte words
  const int4 *gc = reinterpret_cast<const int4 *>(cops + cbase);
  int4 *dc = reinterpret_cast<int4 *>(lc);
  const int64_t wc = (cstop - cbase) * (int64_t)(sizeof(RecC) / 16);
  for (int64_t k = threadIdx.x; k < wc; k += blockDim.x) dc[k] = gc[k];
  const int4 *ge = reinterpret_cast<const int4 *>(eops + ebase);
  int4 *de = reinterpret_cast<int4 *>(le);
  for (int64_t k = threadIdx.x; k < estop - ebase; k += blockDim.x) de[k] = ge[k];
  __syncthreads();
}

// Column r (COL) or row r of the n x n block at g into registers (zero padded).
template <typename T, int NB, bool COL>
__device__ __forceinline__ void vec_mat_line(T (&v)[NB], const T *__restrict__ g, int n, int r) {
  const int rr = r < n ? r : n - 1;
  gather(v, n, [&](int k) { return COL ? g[k * n + rr] : g[rr * n + k]; });
  if (r >= n) zero(v);
}

// Matrix block of an affine-pass primitive (-1: none): rake -> edge slot,
// compress -> left slot; expansion -> right slot.
__device__ __forceinline__ int64_t aff_block(const OpRec &o) {
  return (o.kind == OP_RAKE || o.kind == OP_COMPRESS) ? (int64_t)o.b : -1;
}

// aff_op / affexp_op with the lane's column of Z = T^T already in registers.
template <typename T, int NB>
__device__ __forceinline__ void aff_op_col(const Bufs<T> &bf, const OpRec &o, int r, const T (&col)[NB]) {
  const int n = bf.n;
  if (r >= n) return;
  if (o.kind == OP_RAKE) {  // m = Z h_j + z,  p_j = h_j
    const int64_t j = o.a, e = o.b, out = o.c;
    T hv[NB];
    gather(hv, n, [&](int k) { return bf.h[j * n + k]; });
    bf.cv[out * n + r] = dot_n(col, hv, n, bf.z[e * n + r]);
    bf.p[j * n + r] = bf.h[j * n + r];
  } else if (o.kind == OP_COMBINE) {
    bf.cv[(int64_t)o.c * n + r] = bf.cv[(int64_t)o.a * n + r] + bf.cv[(int64_t)o.b * n + r];
  } else if (o.kind == OP_ABSORB) {
    bf.h[(int64_t)o.a * n + r] += bf.cv[(int64_t)o.b * n + r];
  } else {  // z_new = z_l + Z_l (h_j + z_r)
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T hv[NB], zv[NB];
    gather(hv, n, [&](int k) { return bf.h[j * n + k]; });
    gather(zv, n, [&](int k) { return bf.z[rs * n + k]; });
#pragma unroll
    for (int k = 0; k < NB; ++k) hv[k] += zv[k];
    bf.z[sn * n + r] = dot_n(col, hv, n, bf.z[l * n + r]);
  }
}

template <typename T, int NB>
__device__ __forceinline__ void affexp_op_col(const Bufs<T> &bf, const Op4 &o, int r, const T (&col)[NB]) {
  const int n = bf.n;
  if (r >= n) return;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T pv[NB];
  gather(pv, n, [&](int q) { return bf.p[k * n + q]; });
  bf.p[j * n + r] = dot_n(col, pv, n, bf.h[j * n + r] + bf.z[rs * n + r]);
}

// Affine contraction levels [t0, t1) then affine expansion levels [e0, e1).
// MAXT: the largest workgroup the instance is compiled for (512 leaves each
// lane up to 256 VGPRs; 1024 allows twice the wavefronts with half the
// registers).
template <typename T, int NB, int MAXT>
__device__ __forceinline__ void tail_aff_body(const Bufs<T> &bf, const OpRec *__restrict__ ops, const int64_t *__restrict__ koff, int t0, int t1, const Op4 *__restrict__ eops, const int64_t *__restrict__ eoff, int e0, int e1) {
  constexpr int TW = TeamW<NB>::TW;
  extern __shared__ double smd[];
  int64_t cbase, ebase, *lb;
  OpRec *lc;
  Op4 *le;
  vec_tail_stage<OpRec>(reinterpret_cast<char *>(smd), ops, koff, 5, 4, t0, t1, eops, eoff, e0, e1, cbase, ebase,
                        lc, le, lb);
  const int nc = t1 - t0, nl = nc + (e1 - e0);
  const int slot = threadIdx.x / TW, nslot = blockDim.x / TW, r = threadIdx.x % TW;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  auto block_of = [&](int l, int64_t i) -> int64_t { return l < nc ? aff_block(lc[i]) : (int64_t)le[i].b; };
  T pf[NB];
  {
    const int64_t i = lb[0] + slot;
    const int64_t blk = (nl > 0 && i < lb[1]) ? block_of(0, i) : -1;
    if (blk >= 0) vec_mat_line<T, NB, true>(pf, bf.Tm + blk * nn, n, r);
  }
  for (int l = 0; l < nl; ++l) {
    T nx[NB];
    if (l + 1 < nl) {
      const int64_t i = lb[2 * (l + 1)] + slot;
      const int64_t blk = (i < lb[2 * (l + 1) + 1]) ? block_of(l + 1, i) : -1;
      if (blk >= 0) vec_mat_line<T, NB, true>(nx, bf.Tm + blk * nn, n, r);
    }
    const int64_t b0 = lb[2 * l], b1 = lb[2 * l + 1];
    for (int64_t i = b0 + slot; i < b1; i += nslot) {
      T col[NB];
      if (i == b0 + slot) {
#pragma unroll
        for (int k = 0; k < NB; ++k) col[k] = pf[k];
      } else {
        const int64_t blk = block_of(l, i);
        if (blk >= 0) vec_mat_line<T, NB, true>(col, bf.Tm + blk * nn, n, r);
      }
      if (l < nc)
        aff_op_col<T, NB>(bf, lc[i], r, col);
      else
        affexp_op_col<T, NB>(bf, le[i], r, col);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) pf[k] = nx[k];
  }
}

template <typename T, int NB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_tail_aff(Bufs<T> bf, const OpRec *__restrict__ ops,
                                                   const int64_t *__restrict__ koff, int t0, int t1,
                                                   const Op4 *__restrict__ eops, const int64_t *__restrict__ eoff,
                                                   int e0, int e1) {
  if (bf.n == NB)
    tail_aff_body<T, NB, MAXT>(exact_n<NB>(bf), ops, koff, t0, t1, eops, eoff, e0, e1);
  else
    tail_aff_body<T, NB, MAXT>(bf, ops, koff, t0, t1, eops, eoff, e0, e1);
}

// State-offset composition levels [t0, t1) then state expansion levels [e0, e1):
// b_new = T_r b_l + b_r and x_j = T_s x_i + b_s with the lane's row of T.
template <typename T, int NB, int MAXT>
__device__ __forceinline__ void tail_state_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, const int64_t *__restrict__ off, int t0, int t1, const Op4 *__restrict__ xops, const int64_t *__restrict__ xoff, int e0, int e1) {
  constexpr int TW = TeamW<NB>::TW;
  extern __shared__ double smd[];
  int64_t cbase, ebase, *lb;
  Op4 *lc, *le;
  vec_tail_stage<Op4>(reinterpret_cast<char *>(smd), ops, off, 1, 1, t0, t1, xops, xoff, e0, e1, cbase, ebase, lc,
                      le, lb);
  const int nc = t1 - t0, nl = nc + (e1 - e0);
  const int slot = threadIdx.x / TW, nslot = blockDim.x / TW, r = threadIdx.x % TW;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  // composition {l slot, r slot, new slot, j}: T_r;  expansion {j, slot, parent}: T_slot
  auto block_of = [&](int l, int64_t i) -> int64_t { return (int64_t)(l < nc ? lc[i].b : le[i].b); };
  T pf[NB];
  {
    const int64_t i = lb[0] + slot;
    if (nl > 0 && i < lb[1]) vec_mat_line<T, NB, false>(pf, bf.Tm + block_of(0, i) * nn, n, r);
  }
  for (int l = 0; l < nl; ++l) {
    T nx[NB];
    if (l + 1 < nl) {
      const int64_t i = lb[2 * (l + 1)] + slot;
      if (i < lb[2 * (l + 1) + 1]) vec_mat_line<T, NB, false>(nx, bf.Tm + block_of(l + 1, i) * nn, n, r);
    }
    const int64_t b0 = lb[2 * l], b1 = lb[2 * l + 1];
    for (int64_t i = b0 + slot; i < b1; i += nslot) {
      T row[NB];
      if (i == b0 + slot) {
#pragma unroll
        for (int k = 0; k < NB; ++k) row[k] = pf[k];
      } else {
        vec_mat_line<T, NB, false>(row, bf.Tm + block_of(l, i) * nn, n, r);
      }
      if (r < n) {
        T v[NB];
        if (l < nc) {
          const Op4 o = lc[i];
          gather(v, n, [&](int k) { return bf.b[(int64_t)o.a * n + k]; });
          bf.b[(int64_t)o.c * n + r] = dot_n(row, v, n, bf.b[(int64_t)o.b * n + r]);
        } else {
          const Op4 o = le[i];
          gather(v, n, [&](int k) { return bf.xw[(int64_t)o.c * n + k]; });
          bf.xw[(int64_t)o.a * n + r] = dot_n(row, v, n, bf.b[(int64_t)o.b * n + r]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) pf[k] = nx[k];
  }
}

template <typename T, int NB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_tail_state(Bufs<T> bf, const Op4 *__restrict__ ops,
                                                     const int64_t *__restrict__ off, int t0, int t1,
                                                     const Op4 *__restrict__ xops, const int64_t *__restrict__ xoff,
                                                     int e0, int e1) {
  if (bf.n == NB)
    tail_state_body<T, NB, MAXT>(exact_n<NB>(bf), ops, off, t0, t1, xops, xoff, e0, e1);
  else
    tail_state_body<T, NB, MAXT>(bf, ops, off, t0, t1, xops, xoff, e0, e1);
}

}  // namespace rcr

namespace rcr {

// One launch holding two independent levels of a factor + solve: composite
// transitions of contraction level i (workgroups [0, tc_blocks)) and the
// affine contraction level i - 1 (the rest).  An affine primitive of level
// i - 1 reads only composites of levels below i - 1, so the two never touch
// the same data, and the pair costs one launch instead of two.
template <typename T, int NB>
__device__ __forceinline__ void tc_aff_level(const Bufs<T> &bf, const Op4 *__restrict__ tc_ops, int64_t tc_off,
                                             int64_t tc_cnt, int tc_blocks, const OpRec *__restrict__ ops,
                                             const Seg &sg) {
  const int b = (int)blockIdx.x;
  if (b < tc_blocks) {
    if constexpr (MatLay<NB>::WIDE) {
      extern __shared__ double smd[];
      tcomp_op_wide<T, NB>(bf, tc_ops[tc_off + b], reinterpret_cast<T *>(smd));
    } else {
      tcompose_body<T, NB>(bf, tc_ops, tc_off, tc_cnt, b);
    }
  } else {
    aff_level_body<T, NB>(bf, ops, sg, b - tc_blocks);
  }
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_tc_aff_level(Bufs<T> bf, const Op4 *__restrict__ tc_ops, int64_t tc_off, int64_t tc_cnt,
                                       int tc_blocks, const OpRec *__restrict__ ops, Seg sg) {
  if (bf.n == NB)
    tc_aff_level<T, NB>(exact_n<NB>(bf), tc_ops, tc_off, tc_cnt, tc_blocks, ops, sg);
  else
    tc_aff_level<T, NB>(bf, tc_ops, tc_off, tc_cnt, tc_blocks, ops, sg);
}

}  // namespace rcr
