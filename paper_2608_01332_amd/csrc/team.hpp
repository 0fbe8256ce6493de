// Device building blocks shared by the solver kernels: the working-buffer
// descriptor and the "team" primitives for small dense blocks.
//
// A team is TW consecutive lanes of one 64-lane wavefront (TW = 4, 8 or 16,
// the smallest that covers the padded block size NB); 64 / TW teams share a
// wavefront, and every workgroup is one wavefront, so a team never waits for
// another wavefront and its LDS exchanges need no hardware barrier.  Lane r of a team owns row r of every NB x NB block in
// registers; a block that other lanes must read is staged in the team's LDS
// region, where whole rows are broadcast to the team.  Blocks of dimension
// n < NB are padded with zeros (and the implicit identity of I + ...), which
// leaves the leading n x n results unchanged: the padded coordinates decouple.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "plan.hpp"

namespace rcr {

enum { ST_SINGULAR = 1, ST_NOT_PD = 2, ST_NONFINITE = 4 };

template <typename T>
struct Bufs {
  int n, m, root;
  int64_t N;
  // caller problem (float64, device)
  const double *Q, *q, *c, *De, *R, *S, *r, *A, *B;
  // right-hand side seen by the solve passes
  const T *sq, *sr, *sc;
  // working arrays
  T *U, *EA, *EC, *EP, *CT, *PW, *Finv, *W, *Ginv, *Acl, *Tm, *Kw;
  T *h, *cv, *z, *p, *kff, *b, *xw, *uw, *yw;
  const int32_t *parent;
  // uabs[v] != 0: node v is absorbed into at least once, so its U_v is kept in
  // U; otherwise U_v = Q_v is read from Q (the wide layout writes no copy)
  const int32_t *uabs;
  int *status;
};

// A copy of bf with n (and m) fixed to the padded sizes: kernels run the body
// specialised this way when the problem has no padding, so every bound and
// stride in it is a compile-time constant.
template <int NB, typename T>
__device__ __forceinline__ Bufs<T> exact_n(const Bufs<T> &bf) {
  Bufs<T> b = bf;
  b.n = NB;
  return b;
}
template <int NB, int MB, typename T>
__device__ __forceinline__ Bufs<T> exact_nm(const Bufs<T> &bf) {
  Bufs<T> b = bf;
  b.n = NB;
  b.m = MB;
  return b;
}

template <int NB>
struct TeamW {
  static constexpr int TW = NB <= 4 ? 4 : (NB <= 8 ? 8 : 16);
  static constexpr int PW = 64 / TW;  // teams per wavefront
};

// Ops of one dependency level, grouped by kind: kind s occupies ops
// [off[s], off[s+1]) and workgroups [blk[s], blk[s+1]).  Every workgroup
// therefore executes a single kind, so all its teams follow one code path.
struct Seg {
  int64_t off[5];
  int32_t blk[5];
};

// Stride (in words of T) between the LDS regions of the teams of a
// wavefront: the smallest value >= words that is 1 more than a multiple of
// 128 bytes, so the teams' regions start in different banks and the team-wide
// broadcast reads of one instruction never collide.
template <typename T>
__host__ __device__ constexpr int team_stride(int words) {
  constexpr int K = 128 / (int)sizeof(T);
  return words + ((1 - words) % K + K) % K;
}

// f(std::integral_constant<int, K>) for K = 0 .. N-1 in order: a loop whose
// index is a compile-time constant in the body.
template <typename F, int... K>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
  return fma(a, b, c);
}

// v[k] = at(k) for k < n and 0 for n <= k < NB, with every load issued
// unconditionally (k >= n loads at(n - 1), a valid address, and discards it):
// a load under a per-k condition would be compiled into a branch and a wait
// per k, one memory round trip each, instead of one for all NB.
template <int NB, typename T, typename F>
__device__ __forceinline__ void gather(T (&v)[NB], int n, F at) {
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = at(k < n ? k : n - 1);
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k >= n) v[k] = (T)0;
}

// acc + sum_{k < n} a[k] b[k], in increasing k
template <int NB, typename T>
__device__ __forceinline__ T dot_n(const T (&a)[NB], const T (&b)[NB], int n, T acc) {
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k < n) acc = fmat(a[k], b[k], acc);
  return acc;
}

// Ordering point for a team's LDS traffic.  A workgroup is one wavefront and
// a wavefront executes its LDS instructions in order, so only compiler
// reordering has to be prevented (wavefront-scope fences emit no wait).
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// row[j] = g[r][j] for r, j < n (row stride n), else 0
template <typename T, int NB, typename S>
__device__ __forceinline__ void ld_row(T (&row)[NB], const S *__restrict__ g, int n, int r) {
  // every load issued at once (gather), at a clamped row for the ghost lanes
  const int rr = r < n ? r : n - 1;
  gather(row, n, [&](int j) { return (T)g[(int64_t)rr * n + j]; });
  if (r >= n) {
#pragma unroll
    for (int j = 0; j < NB; ++j) row[j] = (T)0;
  }
}

template <typename T, int NB>
__device__ __forceinline__ void st_row(T *__restrict__ g, const T (&row)[NB], int n, int r, bool active) {
  if (!active || r >= n) return;
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < n) g[(int64_t)r * n + j] = row[j];
}

template <typename T, int NB>
__device__ __forceinline__ void lds_put(T *L, const T (&row)[NB], int r) {
  if (r >= NB) return;
#pragma unroll
  for (int j = 0; j < NB; ++j) L[r * NB + j] = row[j];
}

template <typename T, int NB>
__device__ __forceinline__ void lds_row(T (&row)[NB], const T *L, int k) {
  const int kk = k < NB ? k : NB - 1;
#pragma unroll
  for (int j = 0; j < NB; ++j) row[j] = L[kk * NB + j];
}

template <typename T, int NB>
__device__ __forceinline__ void zero(T (&row)[NB]) {
#pragma unroll
  for (int j = 0; j < NB; ++j) row[j] = (T)0;
}

// The block products below stream LDS rows; every RCR_ROWS_IN_FLIGHT rows the
// accumulators are pinned (an empty asm that reads and writes them) and memory
// accesses are fenced for the compiler, so the loads of later rows are not
// hoisted above the arithmetic of earlier ones (which would exhaust the
// register file).  No instruction is emitted for the fence itself.
#define RCR_ROWS_IN_FLIGHT 2
template <typename T, int W>
__device__ __forceinline__ void pin(T (&acc)[W], int off, int cnt) {
#pragma unroll
  for (int j = 0; j < cnt; ++j) asm volatile("" : "+v"(acc[off + j]));
  asm volatile("" ::: "memory");
}
template <typename T>
__device__ __forceinline__ void pin1(T &x) {
  asm volatile("" : "+v"(x));
}
__device__ __forceinline__ void mem_fence_compiler() { asm volatile("" ::: "memory"); }
#define RCR_ROW_FENCE(k, acc, off, cnt)                                 \
  do {                                                                  \
    if (((k) + 1) % RCR_ROWS_IN_FLIGHT == 0) pin(acc, off, cnt);        \
  } while (0)

// acc[j] += sum_k a[k] * L[k][j]        (a row of A times the block L)
// Products are formed in the accumulator type Acc.
template <typename Acc, int NB, int W, typename TR, typename TL>
__device__ __forceinline__ void mac_rowL(Acc (&acc)[W], int off, const TR (&a)[NB], const TL *L) {
#pragma unroll
  for (int k = 0; k < NB; ++k) {
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[off + j] = fmat((Acc)a[k], (Acc)L[k * NB + j], acc[off + j]);
    RCR_ROW_FENCE(k, acc, off, NB);
  }
}

// acc[j] += sum_k a[k] * L[j][k]        (a row of A times L^T)
template <typename Acc, int NB, int W, typename TR, typename TL>
__device__ __forceinline__ void mac_rowLt(Acc (&acc)[W], int off, const TR (&a)[NB], const TL *L) {
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    Acc s = (Acc)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) s = fmat((Acc)a[k], (Acc)L[j * NB + k], s);
    acc[off + j] += s;
    RCR_ROW_FENCE(j, acc, off, NB);
  }
}

// acc[j] += sum_k L1[k][r] * L2[k][j]   (row r of L1^T L2)
template <typename T, int NB>
__device__ __forceinline__ void mac_colL(T (&acc)[NB], const T *L1, const T *L2, int r) {
  const int rr = r < NB ? r : NB - 1;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T a = L1[k * NB + rr];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = fmat(a, L2[k * NB + j], acc[j]);
    RCR_ROW_FENCE(k, acc, 0, NB);
  }
}

// Gauss-Jordan elimination with partial pivoting of the NB x W system whose
// row r lives in lane r of the team (M[0:NB] the matrix, M[NB:W] the right-hand
// sides).  On return M[NB:W] of lane r is row r of the solution.  The pivot
// row travels through the team's LDS slot Lp (2 W words).  Pivots are chosen
// by a width-TW butterfly argmax of |M[r][k]| over rows r >= k.
// ---------------------------------------------------------------- pivoting
// Pivot key of a candidate row, 32 bits: the float32 magnitude of the entry
// (whose bit pattern orders like an unsigned integer) with its lowest four
// bits replaced by 15 - row, so that one unsigned max over the candidates
// yields a largest magnitude (up to a relative 2^-19, irrelevant to the
// stability of partial pivoting) and its row, an exact tie going to the
// smaller row.  0 marks a lane without a candidate; rows 0..15 only.
__device__ __forceinline__ unsigned piv_key(double v, int row, bool cand) {
  const unsigned b = __float_as_uint((float)fabs(v));
  return cand ? ((b & ~15u) | (unsigned)(15 - row)) : 0u;
}
__device__ __forceinline__ unsigned piv_key(float v, int row, bool cand) {
  const unsigned b = __float_as_uint(fabsf(v));
  return cand ? ((b & ~15u) | (unsigned)(15 - row)) : 0u;
}
__device__ __forceinline__ int piv_row(unsigned key) { return 15 - (int)(key & 15u); }
// no candidate, or a zero (or float32-underflowing) magnitude
__device__ __forceinline__ bool piv_zero(unsigned key) { return (key >> 4) == 0u; }

// Max over the TW lanes of a team, left in every lane: pairs (quad_perm
// [1,0,3,2]), quads (quad_perm [2,3,0,1]), half rows (row_half_mirror), rows
// (row_mirror).  Each step is one v_max_u32 whose first operand is read
// through the DPP permutation; the two wait states before it cover the
// hazard of a DPP read of a VGPR that the previous VALU instruction wrote.
// Every lane of the wavefront must be active.
template <int TW>
__device__ __forceinline__ unsigned team_umax(unsigned v) {
  asm volatile(
      "s_nop 1\n\tv_max_u32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\tv_max_u32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
      : "+v"(v));
  if constexpr (TW >= 8)
    asm volatile("s_nop 1\n\tv_max_u32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf" : "+v"(v));
  if constexpr (TW >= 16)
    asm volatile("s_nop 1\n\tv_max_u32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf" : "+v"(v));
  return v;
}

// Row QK (lanes 16 QK .. 16 QK + 15) of x in every row of the wavefront, lane
// for lane, through the LDS crossbar (ds_bpermute: lane l reads lane
// 16 QK + l % 16).  It issues on the LDS pipe, not the vector ALU, and the
// address is the same for every call with this QK.
template <int QK>
__device__ __forceinline__ int row_bcast_addr() {
  return (int)(((unsigned)(QK << 4) | (threadIdx.x & 15u)) << 2);
}
template <int QK>
__device__ __forceinline__ double row_bcast(double x) {
  const int a = row_bcast_addr<QK>();
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(x));
  return __hiloint2double(hi, lo);
}
template <int QK>
__device__ __forceinline__ float row_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(row_bcast_addr<QK>(), __float_as_int(x)));
}

// 1 / d from the hardware reciprocal refined by Newton steps x <- x (2 - d x)
// (two in float64, one in float32); d is a nonzero pivot.
__device__ __forceinline__ double rcp_nr(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}
__device__ __forceinline__ float rcp_nr(float d) {
  float x = __builtin_amdgcn_rcpf(d);
  const float e = fmaf(-d, x, 1.0f);
  return fmaf(x, e, x);
}

// Gauss-Jordan elimination with partial pivoting of the NB x W system whose
// row r lane r holds in M (rows r >= NB are ghosts).  Rows are never swapped:
// at step k the unused row p of largest |M[k]| becomes the pivot row, is
// scaled by 1 / M_p[k] and eliminated from every other row (Lp: W words).
// Returns the solution row the lane holds on exit: the leading NB x NB block
// is reduced to a permutation, and the lane whose row pivoted at step k holds
// row k of the solution in M[NB..W).  Ghost lanes return their own index.
template <typename T, int NB, int W, int TW>
__device__ __forceinline__ int gj_team(T (&M)[W], T *Lp, int r, int *status) {
  bool used = r >= NB, sing = false;
  int step = r;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const unsigned key = team_umax<TW>(piv_key(M[k], r, !used));
    const int p = piv_row(key);
    sing = sing || piv_zero(key);
    if (r == p) {
#pragma unroll
      for (int j = k; j < W; ++j) Lp[j] = M[j];
    }
    team_sync();
    const T inv = rcp_nr(Lp[k]);
    const T g = (r == p) ? inv - (T)1 : -M[k] * inv;  // the pivot row becomes inv * row
#pragma unroll
    for (int j = k; j < W; ++j) M[j] = fmat(g, Lp[j], M[j]);
    if (r == p) {
      used = true;
      step = k;
    }
    team_sync();
  }
  if ((r & (TW - 1)) == 0 && sing) atomicOr(status, ST_SINGULAR);
  return step;
}

// Row `at` of an NB-wide LDS matrix := row (lanes r >= NB write nothing).
template <typename T, int NB>
__device__ __forceinline__ void lds_put_at(T *L, const T (&row)[NB], int at, int r) {
  if (r >= NB) return;
#pragma unroll
  for (int j = 0; j < NB; ++j) L[at * NB + j] = row[j];
}

// Store 0.5 (X + X^T) where lane r holds row r of X in `row`; Ls is an
// NB x NB LDS scratch that the caller has synchronised for writing.
template <typename T, int NB>
__device__ __forceinline__ void sym_store(T *__restrict__ g, const T (&row)[NB], T *Ls, int n, int r,
                                          bool active) {
  lds_put(Ls, row, r);
  team_sync();
  const int rr = r < NB ? r : NB - 1;
  T out[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) out[j] = (T)0.5 * (row[j] + Ls[j * NB + rr]);
  st_row(g, out, n, r, active);
  team_sync();
}

// ---------------------------------------------------------------- staging
// The PW consecutive nodes [v0, v0 + cnt) of one wavefront own a contiguous
// range of every per-node array.  A tile copies such a range between global
// memory (rn x cn words per node, row-major) and per-team LDS tiles padded to
// RB x CB (team t's tile at lds + t * ts).  Consecutive lanes take consecutive
// padded positions, so the active lanes of one access cover one contiguous
// global range; every load of a tile is issued before any LDS write.
// Padded positions of the LDS tile are written as zero.
template <int PW, int RB, int CB>
struct Tile {
  static constexpr int TOT = PW * RB * CB;
  static constexpr int IT = (TOT + 63) / 64;
};

template <int PW, int RB, int CB, typename S>
__device__ __forceinline__ void stage_load(S (&reg)[(PW * RB * CB + 63) / 64], const S *__restrict__ g, int64_t v0,
                                          int cnt, int rn, int cn, int lane) {
  constexpr int TOT = Tile<PW, RB, CB>::TOT;
  const int64_t w = (int64_t)rn * cn;
#pragma unroll
  for (int k = 0; k < Tile<PW, RB, CB>::IT; ++k) {
    const int p = lane + 64 * k;
    const int t = p / (RB * CB), r = (p / CB) % RB, j = p % CB;
    const bool ok = p < TOT && t < cnt && r < rn && j < cn;
    reg[k] = ok ? g[(v0 + t) * w + r * cn + j] : (S)0;
  }
}

// LDR: LDS row stride of the tile (>= CB; CB + 1 keeps a row-per-lane access
// free of bank conflicts).
template <int PW, int RB, int CB, int LDR = CB, typename S, typename T>
__device__ __forceinline__ void stage_put(T *lds, int ts, const S (&reg)[(PW * RB * CB + 63) / 64], int lane) {
  constexpr int TOT = Tile<PW, RB, CB>::TOT;
#pragma unroll
  for (int k = 0; k < Tile<PW, RB, CB>::IT; ++k) {
    const int p = lane + 64 * k;
    if (p < TOT) {
      const int t = p / (RB * CB), r = (p / CB) % RB, j = p % CB;
      lds[t * ts + r * LDR + j] = (T)reg[k];
    }
  }
}

// LDS tiles -> global rows of nodes t < cnt.  Bit t * tw of `skip` (a ballot
// over lanes, tw = team width) marks a team whose node is not written.  With
// TRANS, the LDS tile holds the transpose of the global block (LDS row j,
// column r -> global row r, column j; the LDS tile is CB x RB).
template <int PW, int RB, int CB, bool TRANS = false, int LDR = CB, typename T, typename D>
__device__ __forceinline__ void stage_store(D *__restrict__ g, const T *lds, int ts, int64_t v0, int cnt, int rn,
                                           int cn, int lane, uint64_t skip = 0, int tw = 64) {
  constexpr int TOT = Tile<PW, RB, CB>::TOT;
  const int64_t w = (int64_t)rn * cn;
#pragma unroll
  for (int k = 0; k < Tile<PW, RB, CB>::IT; ++k) {
    const int p = lane + 64 * k;
    const int t = p / (RB * CB), r = (p / CB) % RB, j = p % CB;
    const bool skipped = (skip >> ((t * tw) & 63)) & 1;
    if (p < TOT && t < cnt && !skipped && r < rn && j < cn)
      g[(v0 + t) * w + r * cn + j] = (D)(TRANS ? lds[t * ts + j * RB + r] : lds[t * ts + r * LDR + j]);
  }
}

// Contiguous copy of `count` words (at most PW * MAXW), converted to D.
template <int MAXC, typename S, typename D>
__device__ __forceinline__ void range_copy(D *__restrict__ dst, const S *__restrict__ src, int count, int lane) {
  S reg[(MAXC + 63) / 64];
#pragma unroll
  for (int k = 0; k < (MAXC + 63) / 64; ++k) {
    const int e = lane + 64 * k;
    reg[k] = e < count ? src[e] : (S)0;
  }
#pragma unroll
  for (int k = 0; k < (MAXC + 63) / 64; ++k) {
    const int e = lane + 64 * k;
    if (e < count) dst[e] = (D)reg[k];
  }
}

// Row r of a team's padded LDS tile (RB rows of CB words) into registers
// (lanes r >= RB read the last row; their values are not used).
template <int RB, int CB, typename T, typename S>
__device__ __forceinline__ void stage_row(T (&row)[CB], const S *tile, int r) {
  const int rr = r < RB ? r : RB - 1;
#pragma unroll
  for (int j = 0; j < CB; ++j) row[j] = (T)tile[rr * CB + j];
}

}  // namespace rcr
