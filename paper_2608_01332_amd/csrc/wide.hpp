// Wide layout of the level kernels for padded block sizes NB in {12, 16}.
//
// One primitive per 64-lane wavefront: lane L = 16 q + r owns row r (rows
// r >= NB are idle ghosts) and column quarter q (columns [q CQ, q CQ + CQ),
// CQ = NB / 4) of every NB x NB block for the Gauss-Jordan elimination; the
// operand blocks live in the wavefront's LDS, and the block products run on
// the float64 matrix cores (mfma.hpp).  A wavefront per primitive quarters the
// per-primitive latency of the one-row-per-lane team layout, which matters on
// the narrow dependency levels near the root where a level holds only a
// handful of primitives.
#pragma once

#include "team.hpp"

namespace rcr {

template <int NB>
struct WideCfg {
  static_assert(NB % 4 == 0 && NB <= 16, "wide layout needs NB in {12, 16}");
  static constexpr int CQ = NB / 4;
  static constexpr int TILE = (NB * NB + 63) / 64;  // block elements per lane when copying
  // LDS row stride of an NB x NB block: one padding word makes the 16 rows a
  // column access touches fall in distinct bank pairs (no 4-way conflicts)
  static constexpr int LD = NB + 1;
  static constexpr int BS = NB * LD;  // LDS words of one block
};

__device__ __forceinline__ int wq_of() { return (int)((threadIdx.x & 63) >> 4); }
__device__ __forceinline__ int wr_of() { return (int)(threadIdx.x & 15); }

// Coalesced fetch of an n x n block (row stride n) into per-lane registers,
// element e = lane + 64 u of the zero-padded NB x NB block.
template <typename T, int NB, typename S>
__device__ __forceinline__ void wfetch(T (&t)[WideCfg<NB>::TILE], const S *__restrict__ g, int n) {
#pragma unroll
  for (int u = 0; u < WideCfg<NB>::TILE; ++u) {
    const int e = (int)(threadIdx.x & 63) + 64 * u;
    const int i = e / NB, j = e - (e / NB) * NB;
    t[u] = (e < NB * NB && i < n && j < n) ? (T)g[i * n + j] : (T)0;
  }
}

template <typename T, int NB>
__device__ __forceinline__ void wput(T *L, int ld, const T (&t)[WideCfg<NB>::TILE]) {
#pragma unroll
  for (int u = 0; u < WideCfg<NB>::TILE; ++u) {
    const int e = (int)(threadIdx.x & 63) + 64 * u;
    const int i = e / NB, j = e - (e / NB) * NB;
    if (e < NB * NB) L[i * ld + j] = t[u];
  }
}

// Coalesced store of the n x n block of a zero-padded tile.
template <typename T, int NB>
__device__ __forceinline__ void wstore_tile(T *__restrict__ g, const T (&t)[WideCfg<NB>::TILE], int n,
                                            bool active) {
  if (!active) return;
#pragma unroll
  for (int u = 0; u < WideCfg<NB>::TILE; ++u) {
    const int e = (int)(threadIdx.x & 63) + 64 * u;
    const int i = e / NB, j = e - (e / NB) * NB;
    if (e < NB * NB && i < n && j < n) g[i * n + j] = t[u];
  }
}

template <typename T, int NB>
__device__ __forceinline__ void wstore_piece(T *__restrict__ g, const T (&p)[WideCfg<NB>::CQ], int n,
                                             bool active) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of();
  if (!active || r >= n) return;
#pragma unroll
  for (int c = 0; c < CQ; ++c) {
    const int j = q * CQ + c;
    if (j < n) g[r * n + j] = p[c];
  }
}

template <typename T, int NB>
__device__ __forceinline__ void wput_piece(T *L, int ld, const T (&p)[WideCfg<NB>::CQ]) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of();
  if (r >= NB) return;
#pragma unroll
  for (int c = 0; c < CQ; ++c) L[r * ld + q * CQ + c] = p[c];
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int lane);
template <>
__device__ __forceinline__ double readlane_t<double>(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float readlane_t<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// m[c] += (m[c] of lane p of this 16-lane row) * g for every c, p in [0, 16)
// wave-uniform: the pivot row's entries reach the other rows through the DPP
// row_newbcast read of the FMA's first operand, with no LDS round trip.  The
// broadcast lane is an immediate of the instruction, so the 16 variants are
// laid out back to back, each of the same byte length (WQ FMAs of 8 bytes and
// a 4-byte branch to the end), and a computed jump (s_getpc / s_setpc) enters
// the variant of p (taken modulo 16).  Seven scalar instructions precede the
// first DPP read and the end carries two wait states, which covers the hazard
// of a DPP read of a VGPR that a VALU instruction has just written on either
// side.  Every lane must be active; s40..s42 are scratch.
#define RCR_JT_HEAD(CASE_BYTES)                   \
  "s_getpc_b64 s[40:41]\n"                        \
  "0:\n\t"                                        \
  "s_and_b32 s42, %[p], 15\n\t"                  \
  "s_mul_i32 s42, s42, " #CASE_BYTES "\n\t"       \
  "s_add_u32 s42, s42, (1f - 0b)\n\t"             \
  "s_add_u32 s40, s40, s42\n\t"                   \
  "s_addc_u32 s41, s41, 0\n\t"                    \
  "s_setpc_b64 s[40:41]\n"                        \
  "1:\n\t"
#define RCR_JT_TAIL "2:\n\ts_nop 1"
#define RCR_FM(OP, I, P) OP " %" #I ", %" #I ", %[g] row_newbcast:" #P " row_mask:0xf bank_mask:0xf\n\t"
#define RCR_C3(OP, P) RCR_FM(OP, 0, P) RCR_FM(OP, 1, P) RCR_FM(OP, 2, P)
#define RCR_C4(OP, P) RCR_C3(OP, P) RCR_FM(OP, 3, P)
#define RCR_C6(OP, P) RCR_C4(OP, P) RCR_FM(OP, 4, P) RCR_FM(OP, 5, P)
#define RCR_C8(OP, P) RCR_C6(OP, P) RCR_FM(OP, 6, P) RCR_FM(OP, 7, P)
#define RCR_C9(OP, P) RCR_C8(OP, P) RCR_FM(OP, 8, P)
#define RCR_C12(OP, P) RCR_C9(OP, P) RCR_FM(OP, 9, P) RCR_FM(OP, 10, P) RCR_FM(OP, 11, P)
#define RCR_CASE(C, OP, P) C(OP, P) "s_branch 2f\n\t"
#define RCR_ALL(C, OP)                                                                                      \
  RCR_CASE(C, OP, 0) RCR_CASE(C, OP, 1) RCR_CASE(C, OP, 2) RCR_CASE(C, OP, 3) RCR_CASE(C, OP, 4)            \
  RCR_CASE(C, OP, 5) RCR_CASE(C, OP, 6) RCR_CASE(C, OP, 7) RCR_CASE(C, OP, 8) RCR_CASE(C, OP, 9)            \
  RCR_CASE(C, OP, 10) RCR_CASE(C, OP, 11) RCR_CASE(C, OP, 12) RCR_CASE(C, OP, 13) RCR_CASE(C, OP, 14)       \
  RCR_CASE(C, OP, 15)
#define RCR_OPS3(m) "+v"(m[0]), "+v"(m[1]), "+v"(m[2])
#define RCR_OPS4(m) RCR_OPS3(m), "+v"(m[3])
#define RCR_OPS6(m) RCR_OPS4(m), "+v"(m[4]), "+v"(m[5])
#define RCR_OPS8(m) RCR_OPS6(m), "+v"(m[6]), "+v"(m[7])
#define RCR_OPS9(m) RCR_OPS8(m), "+v"(m[8])
#define RCR_OPS12(m) RCR_OPS9(m), "+v"(m[9]), "+v"(m[10]), "+v"(m[11])
#define RCR_JT(WQ, CB, OP)                                                                    \
  asm volatile(RCR_JT_HEAD(CB) RCR_ALL(RCR_C##WQ, OP) RCR_JT_TAIL                             \
               : RCR_OPS##WQ(m)                                                               \
               : [g] "v"(g), [p] "s"(p)                                                       \
               : "s40", "s41", "s42", "scc")
template <typename T, int WQ>
__device__ __forceinline__ void row_rank1(T (&m)[WQ], T g, int p) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 4, "float or double");
  static_assert(WQ == 3 || WQ == 4 || WQ == 6 || WQ == 8 || WQ == 9 || WQ == 12,
                "row piece of 3, 4, 6, 8, 9 or 12 words");
  if constexpr (sizeof(T) == 8) {
    if constexpr (WQ == 3) RCR_JT(3, 28, "v_fmac_f64_dpp");
    if constexpr (WQ == 4) RCR_JT(4, 36, "v_fmac_f64_dpp");
    if constexpr (WQ == 6) RCR_JT(6, 52, "v_fmac_f64_dpp");
    if constexpr (WQ == 8) RCR_JT(8, 68, "v_fmac_f64_dpp");
    if constexpr (WQ == 9) RCR_JT(9, 76, "v_fmac_f64_dpp");
    if constexpr (WQ == 12) RCR_JT(12, 100, "v_fmac_f64_dpp");
  } else {
    if constexpr (WQ == 3) RCR_JT(3, 28, "v_fmac_f32_dpp");
    if constexpr (WQ == 4) RCR_JT(4, 36, "v_fmac_f32_dpp");
    if constexpr (WQ == 6) RCR_JT(6, 52, "v_fmac_f32_dpp");
    if constexpr (WQ == 8) RCR_JT(8, 68, "v_fmac_f32_dpp");
    if constexpr (WQ == 9) RCR_JT(9, 76, "v_fmac_f32_dpp");
    if constexpr (WQ == 12) RCR_JT(12, 100, "v_fmac_f32_dpp");
  }
}
#undef RCR_JT
#undef RCR_OPS12
#undef RCR_OPS9
#undef RCR_OPS8
#undef RCR_OPS6
#undef RCR_OPS4
#undef RCR_OPS3
#undef RCR_ALL
#undef RCR_CASE
#undef RCR_C12
#undef RCR_C9
#undef RCR_C8
#undef RCR_C6
#undef RCR_C4
#undef RCR_C3
#undef RCR_FM
#undef RCR_JT_TAIL
#undef RCR_JT_HEAD

// Gauss-Jordan elimination with partial pivoting of the NB x W system staged
// in LDS (LM, row stride W + 1): lane (q, r) works on the piece
// [q WQ, q WQ + WQ) of row r.  Rows are never swapped.  At step k the pivot
// key (piv_key) of column k is reduced over the 16 lanes holding that column
// and made wave-uniform with readlane.  Every lane forms the reciprocal of
// its own column-k entry while the key is reduced, and readlane fetches the
// pivot's from its lane, so the reciprocal is off the step's critical path.
// Each lane's multiplier (its row's entry in column k, held by lane (qk, r))
// is broadcast across the rows of the wavefront through the LDS crossbar
// (row_bcast), and the pivot row's piece reaches every lane of its column
// quarter through the DPP broadcast of row_rank1: no step touches LDS memory.  The pivot row is scaled by
// 1 / pivot and eliminated from every other row.  On return LM holds the
// eliminated system in pivot order: row k is the row that pivoted at step k,
// so columns [NB, W) are the solution.
template <typename T, int NB, int W>
__device__ __forceinline__ void gj_wide(T *LM, int *status, bool report) {
  constexpr int WQ = W / 4, LW = W + 1;
  const int q = wq_of(), r = wr_of();
  T m[WQ];
#pragma unroll
  for (int c = 0; c < WQ; ++c) m[c] = (r < NB) ? LM[r * LW + q * WQ + c] : (T)0;
  bool used = r >= NB, sing = false;
  int step = 0;
  static_for<NB>([&](auto kc) {
    constexpr int k = decltype(kc)::value, qk = k / WQ, ck = k % WQ;
    const T rc = rcp_nr(m[ck]);  // this lane's candidate reciprocal
    const unsigned key = (unsigned)__builtin_amdgcn_readlane(
        (int)team_umax<16>(piv_key(m[ck], r, !used && q == qk)), qk * 16);
    const int p = piv_row(key);
    sing = sing || piv_zero(key);
    const T inv = readlane_t<T>(rc, qk * 16 + p);
    const T f = row_bcast<qk>(m[ck]);  // entry (r, k), held by lane (qk, r)
    const T g = (r == p) ? inv - (T)1 : -f * inv;  // the pivot row becomes inv * row
    row_rank1(m, g, p);
    if (r == p) {
      used = true;
      step = k;
    }
  });
  if (report && (threadIdx.x & 63) == 0 && sing) atomicOr(status, ST_SINGULAR);
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < WQ; ++c) LM[step * LW + q * WQ + c] = m[c];
  }
  team_sync();
}

// In-place inverse of the NB x NB matrix staged in LDS (LM, row stride NB + 1)
// by the elimination of gj_wide without the identity half.  Before the
// rank-1 update of step k, column k, which the update would turn into the
// pivot row's unit column, is set to e_p (p the pivot row): the identity half
// of [F | I] holds e_p in its column p until that step, so the update leaves
// in column k exactly the values (same operations, same bits) the identity
// half's column p would hold, and later steps update it as they would have.
// The result is the inverse in pivot order: row r of the elimination belongs
// at the row of the step where r pivoted, column k at the column of step k's
// pivot row; the final store puts both in place, so LM holds F^-1.
template <typename T, int NB>
__device__ __forceinline__ void gj_inv_wide(T *LM, int *status, bool report) {
  constexpr int WQ = NB / 4, LW = NB + 1;
  const int q = wq_of(), r = wr_of();
  T m[WQ];
  int col[WQ];  // the final column of each of this lane's entries
#pragma unroll
  for (int c = 0; c < WQ; ++c) {
    m[c] = (r < NB) ? LM[r * LW + q * WQ + c] : (T)0;
    col[c] = 0;
  }
  bool used = r >= NB, sing = false;
  int step = 0;
  static_for<NB>([&](auto kc) {
    constexpr int k = decltype(kc)::value, qk = k / WQ, ck = k % WQ;
    const T rc = rcp_nr(m[ck]);
    const unsigned key = (unsigned)__builtin_amdgcn_readlane(
        (int)team_umax<16>(piv_key(m[ck], r, !used && q == qk)), qk * 16);
    const int p = piv_row(key);
    sing = sing || piv_zero(key);
    const T inv = readlane_t<T>(rc, qk * 16 + p);
    const T f = row_bcast<qk>(m[ck]);
    const T g = (r == p) ? inv - (T)1 : -f * inv;
    if (q == qk) {
      m[ck] = (r == p) ? (T)1 : (T)0;
      col[ck] = p;
    }
    row_rank1(m, g, p);
    if (r == p) {
      used = true;
      step = k;
    }
  });
  if (report && (threadIdx.x & 63) == 0 && sing) atomicOr(status, ST_SINGULAR);
  team_sync();  // every lane has read its row before any is overwritten
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < WQ; ++c) LM[step * LW + col[c]] = m[c];
  }
  team_sync();
}

template <typename T, int NB>
__host__ __device__ constexpr int tau_lds_words() {
  // tau_wide: A, C (later Y), Ux (3 NB^2) + the system NB x 2 NB (later scratch)
  return 3 * WideCfg<NB>::BS + NB * (2 * NB + 1);
}

template <typename T, int NB>
__host__ __device__ constexpr int compress_lds_words() {
  // compress: Pt, Ar, Al (3 NB^2 words of T), then the float64 system M
  // (NB x 3 NB, over C_l's block: C_l is dead once the system is formed; later
  // the two symmetrisation scratch blocks); in words of T
  return 3 * WideCfg<NB>::BS + NB * (3 * NB + 1) * (int)(sizeof(double) / sizeof(T));
}

// LDS of a wavefront of the wide contraction-level kernels (rake or compress)
template <typename T, int NB>
__host__ __device__ constexpr int wide_lds_words() {
  return tau_lds_words<T, NB>() > compress_lds_words<T, NB>() ? tau_lds_words<T, NB>() : compress_lds_words<T, NB>();
}

}  // namespace rcr
