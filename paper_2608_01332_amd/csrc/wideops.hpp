// Quadratic-pass primitives in the wide layout (one primitive per wavefront,
// NB in {12, 16}): rake, combine, absorb and compress of the contraction,
// the expansion of a compression, and the composite transition of a
// compression.  Block products run on the float64 matrix cores (mfma.hpp);
// the nonsymmetric solves use the wide Gauss-Jordan elimination (wide.hpp).
#pragma once

#include "mfma.hpp"

namespace rcr {

// tau(alpha, Ux) = Pm + A^T Ux (I + C Ux)^{-1} A  (eq. (terminal-fold)),
// symmetrised.  The caller has staged A, C and Ux in L (blocks at 0, BS, 2 BS,
// row stride LD) and synchronised, and passes Pm in the product layout (its
// loads issued with the operand fetches, so they are not a round trip of
// their own at the end); the result is stored to `out` (global).  C's block
// later holds Y = Ux X, and the system's the symmetrisation scratch.
template <typename T, int NB>
__device__ __forceinline__ void tau_wide(T *__restrict__ out, const dv4 &p, T *L, int n, int *status) {
  constexpr int CQ = WideCfg<NB>::CQ, W = 2 * NB, LW = W + 1, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  T *LA = L, *LC = L + BS, *LU = L + 2 * BS, *LM = L + 3 * BS;
  T *LY = LC;
  const int q = wq_of(), r = wr_of();
  {
    const dv4 s = mf_mm<NB, false, false>(mf_ident(NB), LC, LD, LU, LD);  // I + C Ux
    mf_store(LM, LW, s, NB, NB);
    if (r < NB) {
#pragma unroll
      for (int c = 0; c < CQ; ++c) LM[r * LW + NB + q * CQ + c] = LA[r * LD + q * CQ + c];
    }
  }
  team_sync();
  gj_wide<T, NB, W>(LM, status, true);  // X = (I + C Ux)^{-1} A
  {
    const dv4 y = mf_mm<NB, false, false>(mf_zero(), LU, LD, LM + NB, LW);  // Y = Ux X
    mf_store(LY, LD, y, NB, NB);
  }
  team_sync();
  {
    const dv4 o = mf_mm<NB, true, false>(mf_zero(), LA, LD, LY, LD);  // A^T Y
    mf_store(LM, LD, o, NB, NB);  // the system is dead (read by Y before the sync)
  }
  team_sync();
  mf_store(out, n, mf_sym(LM, LD, NB) + p, n, n);
}

// One quadratic-contraction primitive of kind s on a whole wavefront (LDS L).
template <typename T, int NB>
__device__ __forceinline__ void quad_op_wide(const Bufs<T> &bf, const OpRec &o, int s, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  if (s == OP_RAKE) {
    const int64_t j = o.a, e = o.b, out = o.c;
    T tA[TL], tC[TL], tU[TL];
    wfetch<T, NB>(tU, bf.U + j * nn, n);
    wfetch<T, NB>(tA, bf.EA + e * nn, n);
    wfetch<T, NB>(tC, bf.EC + e * nn, n);
    const dv4 pm = mf_load(bf.EP + e * nn, n, n, n);
    wstore_tile<T, NB>(bf.PW + j * nn, tU, n, true);  // expansion of a rake: P_j = U_j
    wput<T, NB>(L, LD, tA);
    wput<T, NB>(L + BS, LD, tC);
    wput<T, NB>(L + 2 * BS, LD, tU);
    team_sync();
    tau_wide<T, NB>(bf.CT + out * nn, pm, L, n, bf.status);
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
    constexpr int W = 3 * NB, LW = W + 1;
    typedef double ST;  // the (I + C_l Pt) solve is always float64
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T *LPt = L, *LAr = L + BS, *LAl = L + 2 * BS, *LCl = L + 3 * BS;
    ST *LM = reinterpret_cast<ST *>(LCl);  // the system overlays C_l
    T *LZ = reinterpret_cast<T *>(LM);  // the system is dead once X and Y are consumed
    T *LS = LZ + BS;
    const int q = wq_of(), r = wr_of();
    {
      T tP[TL], tU[TL], tAr[TL], tAl[TL], tCl[TL];
      wfetch<T, NB>(tP, bf.EP + rs * nn, n);
      wfetch<T, NB>(tU, bf.U + j * nn, n);
      wfetch<T, NB>(tAr, bf.EA + rs * nn, n);
      wfetch<T, NB>(tAl, bf.EA + l * nn, n);
      wfetch<T, NB>(tCl, bf.EC + l * nn, n);
#pragma unroll
      for (int u = 0; u < TL; ++u) tP[u] += tU[u];
      wput<T, NB>(LPt, LD, tP);
      wput<T, NB>(LAr, LD, tAr);
      wput<T, NB>(LAl, LD, tAl);
      wput<T, NB>(LCl, LD, tCl);
    }
    const dv4 cr0 = mf_load(bf.EC + rs * nn, n, n, n);  // C_r
    const dv4 pl = mf_load(bf.EP + l * nn, n, n, n);    // P_l
    team_sync();
    {
      const dv4 sb = mf_mm<NB, false, false>(mf_ident(NB), LCl, LD, LPt, LD);  // S = I + C_l Pt
      const dv4 ct = mf_mm<NB, false, true>(mf_zero(), LCl, LD, LAr, LD);      // C_l A_r^T
      team_sync();  // every read of C_l precedes the system's writes over it
      mf_store(LM, LW, sb, NB, NB);
      mf_store(LM + 2 * NB, LW, ct, NB, NB);
      if (r < NB) {
#pragma unroll
        for (int c = 0; c < CQ; ++c) LM[r * LW + NB + q * CQ + c] = (ST)LAl[r * LD + q * CQ + c];
      }
    }
    team_sync();
    gj_wide<ST, NB, W>(LM, bf.status, true);  // [X | Y] = S^{-1} [A_l | C_l A_r^T]
    const dv4 an = mf_mm<NB, false, false>(mf_zero(), LAr, LD, LM + NB, LW);  // A_r X
    const dv4 cr = mf_mm<NB, false, false>(cr0, LAr, LD, LM + 2 * NB, LW);    // C_r + A_r Y
    const dv4 z = mf_mm<NB, false, false>(mf_zero(), LPt, LD, LM + NB, LW);   // Pt X
    mf_store(bf.EA + sn * nn, n, an, n, n);
    team_sync();  // every read of the system precedes the writes that reuse it
    mf_store(LS, LD, cr, NB, NB);
    mf_store(LZ, LD, z, NB, NB);
    team_sync();
    mf_store(bf.EC + sn * nn, n, mf_sym(LS, LD, NB), n, n);
    const dv4 pn = mf_mm<NB, true, false>(mf_zero(), LAl, LD, LZ, LD);  // A_l^T Z
    mf_store(LPt, LD, pn, NB, NB);                                        // Pt is dead: symmetrisation scratch
    team_sync();
    mf_store(bf.EP + sn * nn, n, mf_sym(LPt, LD, NB) + pl, n, n);
  }
}

// Expansion of one compression: P_j = tau((A_r, C_r, P_r + U_j), P_k)
// (eq. (value-reconstruction)).
template <typename T, int NB>
__device__ __forceinline__ void qexp_op_wide(const Bufs<T> &bf, const Op4 &o, T *L) {
  constexpr int TL = WideCfg<NB>::TILE, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T tA[TL], tC[TL], tPk[TL];
  wfetch<T, NB>(tA, bf.EA + rs * nn, n);
  wfetch<T, NB>(tC, bf.EC + rs * nn, n);
  wfetch<T, NB>(tPk, bf.PW + k * nn, n);
  const dv4 pm = mf_load(bf.EP + rs * nn, n, n, n) + mf_load(bf.U + j * nn, n, n, n);
  wput<T, NB>(L, LD, tA);
  wput<T, NB>(L + BS, LD, tC);
  wput<T, NB>(L + 2 * BS, LD, tPk);
  team_sync();
  tau_wide<T, NB>(bf.PW + j * nn, pm, L, n, bf.status);
}

// Composite transition of one compression: T_new = T_r T_l.
template <typename T, int NB>
__device__ __forceinline__ void tcomp_op_wide(const Bufs<T> &bf, const Op4 &o, T *L) {
  constexpr int TL = WideCfg<NB>::TILE, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  T tl[TL], tr[TL];
  wfetch<T, NB>(tl, bf.Tm + (int64_t)o.a * nn, n);
  wfetch<T, NB>(tr, bf.Tm + (int64_t)o.b * nn, n);
  wput<T, NB>(L, LD, tl);
  wput<T, NB>(L + BS, LD, tr);
  team_sync();
  const dv4 t = mf_mm<NB, false, false>(mf_zero(), L + BS, LD, L, LD);  // T_r T_l
  mf_store(bf.Tm + (int64_t)o.c * nn, n, t, n, n);
}

// The level kernels run the primitive specialised for n = NB when the problem
// has no padding (exact_n).
template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_level_wide(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  extern __shared__ double smd[];
  int s = 0;
  while (s < 3 && (int)blockIdx.x >= sg.blk[s + 1]) ++s;
  const OpRec o = ops[sg.off[s] + (int64_t)(blockIdx.x - sg.blk[s])];
  if (bf.n == NB)
    quad_op_wide<T, NB>(exact_n<NB>(bf), o, s, reinterpret_cast<T *>(smd));
  else
    quad_op_wide<T, NB>(bf, o, s, reinterpret_cast<T *>(smd));
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_expand_wide(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  if (bf.n == NB)
    qexp_op_wide<T, NB>(exact_n<NB>(bf), ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
  else
    qexp_op_wide<T, NB>(bf, ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_tcompose_wide(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  if (bf.n == NB)
    tcomp_op_wide<T, NB>(exact_n<NB>(bf), ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
  else
    tcomp_op_wide<T, NB>(bf, ops[off + blockIdx.x], reinterpret_cast<T *>(smd));
}

}  // namespace rcr
