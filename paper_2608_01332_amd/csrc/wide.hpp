// Wide layout of the level kernels for padded block sizes NB in {12, 16}.
//
// One primitive per 64-lane wavefront: lane L = 16 q + r owns row r (rows
// r >= NB are idle ghosts) and column quarter q (columns [q CQ, q CQ + CQ),
// CQ = NB / 4) of every NB x NB block; operand blocks live in the wavefront's
// LDS and are read as rows or columns, so a block product costs NB * CQ
// multiply-adds per lane.  This quarters the per-primitive latency of the
// one-row-per-lane team layout, which matters on the narrow dependency levels
// near the root where a level holds only a handful of primitives.
#pragma once

#include "team.hpp"

namespace rcr {

// Operand rows a block product keeps in flight between scheduling pins.
#ifndef RCR_WMM_PIN
#define RCR_WMM_PIN 4
#endif

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

// The lane's quarter of row r of an n x n global block.
template <typename T, int NB, typename S>
__device__ __forceinline__ void wfetch_piece(T (&p)[WideCfg<NB>::CQ], const S *__restrict__ g, int n) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of();
#pragma unroll
  for (int c = 0; c < CQ; ++c) {
    const int j = q * CQ + c;
    p[c] = (r < n && j < n) ? (T)g[r * n + j] : (T)0;
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

// out[c] += sum_k A[r][k] B[k][q CQ + c]
template <typename Acc, int NB, typename TA, typename TB>
__device__ __forceinline__ void wmm_AB(Acc (&out)[WideCfg<NB>::CQ], const TA *A, int lda, const TB *B, int ldb) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of() < NB ? wr_of() : NB - 1;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const Acc a = (Acc)A[r * lda + k];
#pragma unroll
    for (int c = 0; c < CQ; ++c) out[c] = fmat(a, (Acc)B[k * ldb + q * CQ + c], out[c]);
    if (k % RCR_WMM_PIN == RCR_WMM_PIN - 1) pin(out, 0, CQ);
  }
}

// out[c] += sum_k A[k][r] B[k][q CQ + c]      (A^T B)
template <typename Acc, int NB, typename TA, typename TB>
__device__ __forceinline__ void wmm_AtB(Acc (&out)[WideCfg<NB>::CQ], const TA *A, int lda, const TB *B, int ldb) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of() < NB ? wr_of() : NB - 1;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const Acc a = (Acc)A[k * lda + r];
#pragma unroll
    for (int c = 0; c < CQ; ++c) out[c] = fmat(a, (Acc)B[k * ldb + q * CQ + c], out[c]);
    if (k % RCR_WMM_PIN == RCR_WMM_PIN - 1) pin(out, 0, CQ);
  }
}

// out[c] += sum_k A[r][k] B[q CQ + c][k]      (A B^T)
template <typename Acc, int NB, typename TA, typename TB>
__device__ __forceinline__ void wmm_ABt(Acc (&out)[WideCfg<NB>::CQ], const TA *A, int lda, const TB *B, int ldb) {
  constexpr int CQ = WideCfg<NB>::CQ;
  const int q = wq_of(), r = wr_of() < NB ? wr_of() : NB - 1;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const Acc a = (Acc)A[r * lda + k];
#pragma unroll
    for (int c = 0; c < CQ; ++c) out[c] = fmat(a, (Acc)B[(q * CQ + c) * ldb + k], out[c]);
    if (k % RCR_WMM_PIN == RCR_WMM_PIN - 1) pin(out, 0, CQ);
  }
}

// 0.5 (X + X^T) for the lane's piece, X staged in LDS (row stride NB).
template <typename T, int NB>
__device__ __forceinline__ void wsym(T (&p)[WideCfg<NB>::CQ], const T *LX) {
  constexpr int CQ = WideCfg<NB>::CQ, LD = WideCfg<NB>::LD;
  const int q = wq_of(), r = wr_of() < NB ? wr_of() : NB - 1;
#pragma unroll
  for (int c = 0; c < CQ; ++c) p[c] = (T)0.5 * (LX[r * LD + q * CQ + c] + LX[(q * CQ + c) * LD + r]);
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

// Gauss-Jordan elimination with partial pivoting of the NB x W system staged
// in LDS (LM, row stride W + 1): lane (q, r) works on the piece
// [q WQ, q WQ + WQ) of row r.  Rows are never swapped.  At step k the pivot
// key (piv_key) of column k is reduced over the 16 lanes holding that column
// and made wave-uniform with readlane, which also fetches the exact pivot
// value from its lane; each lane's multiplier (its row's entry in column k)
// comes from the lane holding it by a cross-lane permute; only the pivot row
// travels through LDS (Lp: W words).  The pivot row is scaled by 1 / pivot
// and eliminated from every other row.  On return LM holds the eliminated
// system in pivot order: row k is the row that pivoted at step k, so columns
// [NB, W) are the solution.  (LF is unused scratch kept for the layout.)
template <typename T, int NB, int W>
__device__ __forceinline__ void gj_wide(T *LM, T *Lp, T *LF, int *status, bool report) {
  constexpr int WQ = W / 4, LW = W + 1;
  const int q = wq_of(), r = wr_of();
  (void)LF;
  T m[WQ];
#pragma unroll
  for (int c = 0; c < WQ; ++c) m[c] = (r < NB) ? LM[r * LW + q * WQ + c] : (T)0;
  bool used = r >= NB, sing = false;
  int step = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int qk = k / WQ, ck = k % WQ;
    const unsigned key = (unsigned)__builtin_amdgcn_readlane(
        (int)team_umax<16>(piv_key(m[ck], r, !used && q == qk)), qk * 16);
    const int p = piv_row(key);
    sing = sing || piv_zero(key);
    const T piv = readlane_t<T>(m[ck], qk * 16 + p);
    const T f = __shfl(m[ck], qk * 16 + r, 64);  // entry (r, k), held by lane (qk, r)
    if (r == p) {
#pragma unroll
      for (int c = 0; c < WQ; ++c) Lp[q * WQ + c] = m[c];
    }
    const T inv = rcp_nr(piv);
    team_sync();
    const T g = (r == p) ? inv - (T)1 : -f * inv;  // the pivot row becomes inv * row
#pragma unroll
    for (int c = 0; c < WQ; ++c) m[c] = fmat(g, Lp[q * WQ + c], m[c]);
    if (r == p) {
      used = true;
      step = k;
    }
    team_sync();
  }
  if (report && (threadIdx.x & 63) == 0 && sing) atomicOr(status, ST_SINGULAR);
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < WQ; ++c) LM[step * LW + q * WQ + c] = m[c];
  }
  team_sync();
}

template <typename T, int NB>
__host__ __device__ constexpr int wide_lds_words() {
  // compress: Pt, Ar, Al, Cl (4 NB^2 words of T; C_l's block later holds the
  // symmetrisation scratch) + the float64 system M (3 NB^2, later Z), the
  // pivot row (3 NB) and 16 spare words; in words of T
  return 4 * WideCfg<NB>::BS + (NB * (3 * NB + 1) + 3 * NB + 16) * (int)(sizeof(double) / sizeof(T));
}

template <typename T, int NB>
__host__ __device__ constexpr int tau_lds_words() {
  // tau_wide: A, C, Ux, Y (4 NB^2) + the system NB x 2 NB + pivot row (2 NB) + 16 spare
  return 4 * WideCfg<NB>::BS + NB * (2 * NB + 1) + 2 * NB + 16;
}

// tau(alpha, Ux) = Pm + A^T Ux (I + C Ux)^{-1} A  (eq. (terminal-fold)), symmetrised.
// tA, tC, tU: zero-padded tiles of A, C, Ux; pm: the lane's piece of Pm.
template <typename T, int NB>
__device__ __forceinline__ void tau_wide(T *__restrict__ out, const T (&tA)[WideCfg<NB>::TILE],
                                         const T (&tC)[WideCfg<NB>::TILE], const T (&tU)[WideCfg<NB>::TILE],
                                         const T (&pm)[WideCfg<NB>::CQ], T *L, int n, bool active, int *status) {
  constexpr int CQ = WideCfg<NB>::CQ, W = 2 * NB, LW = W + 1, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  T *LA = L, *LC = L + BS, *LU = L + 2 * BS, *LY = L + 3 * BS, *LM = L + 4 * BS;
  T *Lp = LM + NB * LW, *LF = Lp + W;
  const int q = wq_of(), r = wr_of();
  wput<T, NB>(LA, LD, tA);
  wput<T, NB>(LC, LD, tC);
  wput<T, NB>(LU, LD, tU);
  team_sync();
  {
    T s[CQ];
#pragma unroll
    for (int c = 0; c < CQ; ++c) s[c] = (q * CQ + c == r) ? (T)1 : (T)0;
    wmm_AB<T, NB>(s, LC, LD, LU, LD);  // I + C Ux
    if (r < NB) {
#pragma unroll
      for (int c = 0; c < CQ; ++c) {
        LM[r * LW + q * CQ + c] = s[c];
        LM[r * LW + NB + q * CQ + c] = LA[r * LD + q * CQ + c];
      }
    }
  }
  team_sync();
  gj_wide<T, NB, W>(LM, Lp, LF, status, active);
  {
    T y[CQ];
#pragma unroll
    for (int c = 0; c < CQ; ++c) y[c] = (T)0;
    wmm_AB<T, NB>(y, LU, LD, LM + NB, LW);  // Y = Ux X
    wput_piece<T, NB>(LY, LD, y);
  }
  team_sync();
  T o[CQ];
#pragma unroll
  for (int c = 0; c < CQ; ++c) o[c] = (T)0;
  wmm_AtB<T, NB>(o, LA, LD, LY, LD);  // A^T Y
  wput_piece<T, NB>(LC, LD, o);       // C is dead: reuse for the symmetrisation
  team_sync();
  wsym<T, NB>(o, LC);
#pragma unroll
  for (int c = 0; c < CQ; ++c) o[c] += pm[c];
  wstore_piece<T, NB>(out, o, n, active);
}

// One quadratic-contraction primitive of kind s on a whole wavefront (LDS L).
template <typename T, int NB>
__device__ __forceinline__ void quad_op_wide(const Bufs<T> &bf, const OpRec &o, int s, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const bool active = true;
  if (s == OP_RAKE) {
    const int64_t j = o.a, e = o.b, out = o.c;
    T tA[TL], tC[TL], tU[TL], pm[CQ];
    wfetch<T, NB>(tU, bf.U + j * nn, n);
    wfetch<T, NB>(tA, bf.EA + e * nn, n);
    wfetch<T, NB>(tC, bf.EC + e * nn, n);
    wfetch_piece<T, NB>(pm, bf.EP + e * nn, n);
    wstore_tile<T, NB>(bf.PW + j * nn, tU, n, active);  // expansion of a rake: P_j = U_j
    tau_wide<T, NB>(bf.CT + out * nn, tA, tC, tU, pm, L, n, active, bf.status);
  } else if (s == OP_COMBINE || s == OP_ABSORB) {
    T *dst = (s == OP_COMBINE) ? bf.CT + (int64_t)o.c * nn : bf.U + (int64_t)o.a * nn;
    const T *a = (s == OP_COMBINE) ? bf.CT + (int64_t)o.a * nn : bf.U + (int64_t)o.a * nn;
    const T *b = bf.CT + (int64_t)o.b * nn;
    T va[TL], vb[TL];
#pragma unroll
    for (int u = 0; u < TL; ++u) {
      const int e = (int)(threadIdx.x & 63) + 64 * u;
      va[u] = e < n * n ? a[e] : (T)0;
      vb[u] = e < n * n ? b[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < TL; ++u) {
      const int e = (int)(threadIdx.x & 63) + 64 * u;
      if (e < n * n) dst[e] = va[u] + vb[u];
    }
  } else {
    // alpha_{lr} = alpha_r o_{U_j} alpha_l  (eqs. (compress-intermediates), (composition))
    constexpr int W = 3 * NB, LW = W + 1, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
    typedef double ST;  // the (I + C_l Pt) solve is always float64
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T *LPt = L, *LAr = L + BS, *LAl = L + 2 * BS, *LCl = L + 3 * BS;
    ST *LM = reinterpret_cast<ST *>(L + 4 * BS), *Lp = LM + NB * LW, *LF = Lp + W;
    T *LS = LCl;                          // C_l is dead once S and C_l A_r^T are formed
    T *LZ = reinterpret_cast<T *>(LM);    // the system is dead once X and Y are consumed
    const int q = wq_of(), r = wr_of();
    T cr[CQ], pl[CQ];
    {
      T tP[TL], tU[TL], tAr[TL], tAl[TL], tCl[TL];
      wfetch<T, NB>(tP, bf.EP + rs * nn, n);
      wfetch<T, NB>(tU, bf.U + j * nn, n);
      wfetch<T, NB>(tAr, bf.EA + rs * nn, n);
      wfetch<T, NB>(tAl, bf.EA + l * nn, n);
      wfetch<T, NB>(tCl, bf.EC + l * nn, n);
      wfetch_piece<T, NB>(cr, bf.EC + rs * nn, n);
      wfetch_piece<T, NB>(pl, bf.EP + l * nn, n);
#pragma unroll
      for (int u = 0; u < TL; ++u) tP[u] += tU[u];
      wput<T, NB>(LPt, LD, tP);
      wput<T, NB>(LAr, LD, tAr);
      wput<T, NB>(LAl, LD, tAl);
      wput<T, NB>(LCl, LD, tCl);
    }
    team_sync();
    {
      ST sb[CQ], ct[CQ];
#pragma unroll
      for (int c = 0; c < CQ; ++c) {
        sb[c] = (q * CQ + c == r) ? (ST)1 : (ST)0;
        ct[c] = (ST)0;
      }
      wmm_AB<ST, NB>(sb, LCl, LD, LPt, LD);   // S = I + C_l Pt
      wmm_ABt<ST, NB>(ct, LCl, LD, LAr, LD);  // C_l A_r^T
      if (r < NB) {
#pragma unroll
        for (int c = 0; c < CQ; ++c) {
          LM[r * LW + q * CQ + c] = sb[c];
          LM[r * LW + NB + q * CQ + c] = (ST)LAl[r * LD + q * CQ + c];
          LM[r * LW + 2 * NB + q * CQ + c] = ct[c];
        }
      }
    }
    team_sync();
    gj_wide<ST, NB, W>(LM, Lp, LF, bf.status, active);  // [X | Y] = S^{-1} [A_l | C_l A_r^T]
    {
      T an[CQ], z[CQ];
#pragma unroll
      for (int c = 0; c < CQ; ++c) {
        an[c] = (T)0;
        z[c] = (T)0;
      }
      wmm_AB<T, NB>(an, LAr, LD, LM + NB, LW);      // A_r X
      wmm_AB<T, NB>(cr, LAr, LD, LM + 2 * NB, LW);  // C_r + A_r Y
      wmm_AB<T, NB>(z, LPt, LD, LM + NB, LW);       // Pt X
      wstore_piece<T, NB>(bf.EA + sn * nn, an, n, active);
      team_sync();  // every read of the system precedes the writes that reuse it
      wput_piece<T, NB>(LS, LD, cr);
      wput_piece<T, NB>(LZ, LD, z);
    }
    team_sync();
    wsym<T, NB>(cr, LS);
    wstore_piece<T, NB>(bf.EC + sn * nn, cr, n, active);
    T pn[CQ];
#pragma unroll
    for (int c = 0; c < CQ; ++c) pn[c] = (T)0;
    wmm_AtB<T, NB>(pn, LAl, LD, LZ, LD);  // A_l^T Z
    wput_piece<T, NB>(LPt, LD, pn);       // Pt is dead: reuse for the symmetrisation
    team_sync();
    wsym<T, NB>(pn, LPt);
#pragma unroll
    for (int c = 0; c < CQ; ++c) pn[c] += pl[c];
    wstore_piece<T, NB>(bf.EP + sn * nn, pn, n, active);
  }
}

template <typename T, int NB>
__device__ __forceinline__ void qexp_op_wide(const Bufs<T> &bf, const Op4 &o, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T tA[TL], tC[TL], tPk[TL], pm[CQ], uj[CQ];
  wfetch<T, NB>(tA, bf.EA + rs * nn, n);
  wfetch<T, NB>(tC, bf.EC + rs * nn, n);
  wfetch<T, NB>(tPk, bf.PW + k * nn, n);
  wfetch_piece<T, NB>(pm, bf.EP + rs * nn, n);
  wfetch_piece<T, NB>(uj, bf.U + j * nn, n);
#pragma unroll
  for (int c = 0; c < CQ; ++c) pm[c] += uj[c];
  tau_wide<T, NB>(bf.PW + j * nn, tA, tC, tPk, pm, L, n, true, bf.status);
}

template <typename T, int NB>
__device__ __forceinline__ void tcomp_op_wide(const Bufs<T> &bf, const Op4 &o, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  T tl[TL], tr[TL];
  wfetch<T, NB>(tl, bf.Tm + (int64_t)o.a * nn, n);
  wfetch<T, NB>(tr, bf.Tm + (int64_t)o.b * nn, n);
  constexpr int LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  wput<T, NB>(L, LD, tl);
  wput<T, NB>(L + BS, LD, tr);
  team_sync();
  T out[CQ];
#pragma unroll
  for (int c = 0; c < CQ; ++c) out[c] = (T)0;
  wmm_AB<T, NB>(out, L + BS, LD, L, LD);  // T_r T_l
  wstore_piece<T, NB>(bf.Tm + (int64_t)o.c * nn, out, n, true);
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_level_wide(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  extern __shared__ double smd[];
  int s = 0;
  while (s < 3 && (int)blockIdx.x >= sg.blk[s + 1]) ++s;
  const OpRec o = ops[sg.off[s] + (int64_t)(blockIdx.x - sg.blk[s])];
  quad_op_wide<T, NB>(bf, o, s, reinterpret_cast<T *>(smd));
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_expand_wide(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  qexp_op_wide<T, NB>(bf, ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_tcompose_wide(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  tcomp_op_wide<T, NB>(bf, ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
}

}  // namespace rcr
