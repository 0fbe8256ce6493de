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

// The composition of a compression (eqs. (compress-intermediates),
// (composition)) once its operands are staged: Pt = P_r + U_j, A_r, A_l, C_l in
// L (blocks at 0, BS, 2 BS, 3 BS, synchronised), C_r and P_l in the product
// layout.  Writes the new edge record (A, C, P) to slot sn.
template <typename T, int NB>
__device__ __forceinline__ void compress_core(const Bufs<T> &bf, int64_t sn, const dv4 &cr0, const dv4 &pl, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  constexpr int W = 3 * NB, LW = W + 1;
  typedef double ST;  // the (I + C_l Pt) solve is always float64
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  T *LPt = L, *LAr = L + BS, *LAl = L + 2 * BS, *LCl = L + 3 * BS;
  ST *LM = reinterpret_cast<ST *>(LCl);  // the system overlays C_l
  T *LZ = reinterpret_cast<T *>(LM);  // the system is dead once X and Y are consumed
  T *LS = LZ + BS;
  const int q = wq_of(), r = wr_of();
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

// One quadratic-contraction primitive of kind s on a whole wavefront (LDS L).
template <typename T, int NB>
__device__ __forceinline__ void quad_op_wide(const Bufs<T> &bf, const OpRec &o, int s, T *L) {
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  if (s == OP_RAKE) {
    const int64_t j = o.a, e = o.b, out = o.c;
    T tA[TL], tC[TL], tU[TL];
    if (o.round & OPF_U_LIVE)
      wfetch<T, NB>(tU, bf.U + j * nn, n);
    else
      wfetch<T, NB>(tU, bf.Q + j * nn, n);  // never absorbed into: U_j = Q_j
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
    const bool from_q = s == OP_ABSORB && (o.round & OPF_FIRST_ABSORB);  // U_i starts as Q_i
    const double *aq = bf.Q + (int64_t)o.a * nn;
    T va[TL], vb[TL];
#pragma unroll
    for (int u = 0; u < TL; ++u) {
      const int e = (int)(threadIdx.x & 63) + 64 * u;
      va[u] = e < n * n ? (from_q ? (T)aq[e] : a[e]) : (T)0;
      vb[u] = e < n * n ? b[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < TL; ++u) {
      const int e = (int)(threadIdx.x & 63) + 64 * u;
      if (e < n * n) dst[e] = va[u] + vb[u];
    }
  } else {
    // alpha_{lr} = alpha_r o_{U_j} alpha_l  (eqs. (compress-intermediates), (composition))
    const int64_t j = o.a, l = o.b, rs = o.c;
    T *LPt = L, *LAr = L + BS, *LAl = L + 2 * BS, *LCl = L + 3 * BS;
    {
      T tP[TL], tU[TL], tAr[TL], tAl[TL], tCl[TL];
      wfetch<T, NB>(tP, bf.EP + rs * nn, n);
      if (o.round & OPF_U_LIVE)
        wfetch<T, NB>(tU, bf.U + j * nn, n);
      else
        wfetch<T, NB>(tU, bf.Q + j * nn, n);
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
    compress_core<T, NB>(bf, o.d, cr0, pl, L);
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
  const dv4 uj = (o.d & OPF_U_LIVE) ? mf_load(bf.U + j * nn, n, n, n)
                                     : mf_round<T>(mf_load(bf.Q + j * nn, n, n, n));  // U_j = Q_j
  const dv4 pm = mf_load(bf.EP + rs * nn, n, n, n) + uj;
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


// ---------------------------------------------------------------- condensation
// Control condensation of one edge e = (i, j), edge slot j (eq.
// (edge-components)), in the wide layout for padded control size 4, in
// float64: with L the Cholesky factor of R_e,
//   Bt = B_e L^{-T},  St = M_e L^{-T}  (n x m),
//   Abar = A_e - Bt St^T,  Cbar = Delta_j + Bt Bt^T,  Pbar = -St St^T.
// Every lane factors R_e itself (its 16 words are the same for all lanes),
// lane (q, r) forms row r of Bt and St by forward substitution, and each of
// the three products is one v_mfma_f64_16x16x4 whose k index is the control
// index: lane (q, r) supplies Bt[r][q] as the A operand and Bt[r][q] (for
// Bt Bt^T) or St[r][q] (for Bt St^T, St St^T) as the B operand.
template <int NB>
struct EdgeIn {
  dv4 a, d;          // A_e and Delta_j in the product layout
  double b[4], s[4]; // row r of B_e and of M_e
  double R[4][4];    // R_e, padded with the identity
};

template <typename T, int NB>
__device__ __forceinline__ void edge_fetch(const Bufs<T> &bf, int64_t e, EdgeIn<NB> &w) {
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  const int r = wr_of();
  w.a = mf_load(bf.A + e * nn, n, n, n);
  w.d = mf_load(bf.De + e * nn, n, n, n);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    w.b[c] = (r < n && c < m) ? bf.B[e * nm + r * m + c] : 0.0;
    w.s[c] = (r < n && c < m) ? bf.S[e * nm + r * m + c] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) w.R[i][c] = (i < m && c < m) ? bf.R[e * mm + i * m + c] : (i == c ? 1.0 : 0.0);
}

template <int NB>
__device__ __forceinline__ void edge_condense(const EdgeIn<NB> &w, dv4 &ab, dv4 &cb, dv4 &pb, bool &bad) {
  double L[4][4], dinv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) L[i][c] = (c <= i) ? w.R[i][c] : 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = L[c][c];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= L[c][k] * L[c][k];
    bad = bad || !(s > 0.0);
    const double y = rsqrt_nr(s);
    L[c][c] = s * y;
    dinv[c] = y;
#pragma unroll
    for (int i = c + 1; i < 4; ++i) {
      double t = L[i][c];
#pragma unroll
      for (int k = 0; k < c; ++k) t -= L[i][k] * L[c][k];
      L[i][c] = t * dinv[c];
    }
  }
  double bt[4], st[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {  // L bt^T = b^T, L st^T = s^T
    double sb = w.b[c], ss = w.s[c];
#pragma unroll
    for (int k = 0; k < c; ++k) {
      sb -= L[c][k] * bt[k];
      ss -= L[c][k] * st[k];
    }
    bt[c] = sb * dinv[c];
    st[c] = ss * dinv[c];
  }
  const int q = wq_of();
  const double bq = q == 0 ? bt[0] : q == 1 ? bt[1] : q == 2 ? bt[2] : bt[3];
  const double sq = q == 0 ? st[0] : q == 1 ? st[1] : q == 2 ? st[2] : st[3];
  ab = __builtin_amdgcn_mfma_f64_16x16x4f64(-bq, sq, w.a, 0, 0, 0);      // A - Bt St^T
  cb = __builtin_amdgcn_mfma_f64_16x16x4f64(bq, bq, w.d, 0, 0, 0);       // Delta + Bt Bt^T
  pb = __builtin_amdgcn_mfma_f64_16x16x4f64(-sq, sq, mf_zero(), 0, 0, 0);  // -St St^T
}

// Condense one edge slot and store its record (A, C, P) = (Abar, Cbar, Pbar).
template <typename T, int NB>
__device__ __forceinline__ void condense_one_wide(const Bufs<T> &bf, int64_t e) {
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  EdgeIn<NB> w;
  edge_fetch<T, NB>(bf, e, w);
  dv4 ab, cb, pb;
  bool bad = false;
  edge_condense<NB>(w, ab, cb, pb, bad);
  if (bad && (threadIdx.x & 63) == 0) atomicOr(bf.status, ST_NOT_PD);
  mf_store(bf.EA + e * nn, n, ab, n, n);
  mf_store(bf.EC + e * nn, n, cb, n, n);
  mf_store(bf.EP + e * nn, n, pb, n, n);
}

// Level 1 fused with the condensation of its edges.  Every primitive of the
// first dependency level is a rake of an original leaf or a compression of an
// original unary node (no absorb precedes it, so U = Q), and all its edges
// are original slots: it condenses them in registers instead of reading edge
// records, and only the compression's out-edge record (the tape its
// expansion reads) is stored.  Values pass through the working type exactly
// where the unfused path stores and reloads them, so both give the same bits.
template <typename T, int NB>
__device__ __forceinline__ void rake1_wide(const Bufs<T> &bf, const OpRec &o, T *L) {
  constexpr int TL = WideCfg<NB>::TILE, LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, out = o.c;  // edge slot o.b == j
  EdgeIn<NB> w;
  edge_fetch<T, NB>(bf, j, w);
  T tU[TL];
  wfetch<T, NB>(tU, bf.Q + j * nn, n);
  dv4 ab, cb, pb;
  bool bad = false;
  edge_condense<NB>(w, ab, cb, pb, bad);
  if (bad && (threadIdx.x & 63) == 0) atomicOr(bf.status, ST_NOT_PD);
  wstore_tile<T, NB>(bf.PW + j * nn, tU, n, true);  // expansion of a rake: P_j = U_j
  mf_store(L, LD, ab, NB, NB);
  mf_store(L + BS, LD, cb, NB, NB);
  wput<T, NB>(L + 2 * BS, LD, tU);
  team_sync();
  tau_wide<T, NB>(bf.CT + out * nn, mf_round<T>(pb), L, n, bf.status);
}

template <typename T, int NB>
__device__ __forceinline__ void compress1_wide(const Bufs<T> &bf, const OpRec &o, T *L) {
  constexpr int LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.c;  // in-edge slot o.b == j, out-edge slot rs
  EdgeIn<NB> wl, wr;
  edge_fetch<T, NB>(bf, j, wl);
  edge_fetch<T, NB>(bf, rs, wr);
  const dv4 qj = mf_load(bf.Q + j * nn, n, n, n);
  dv4 al, cl, pl, ar, cr, pr;
  bool bad = false;
  edge_condense<NB>(wl, al, cl, pl, bad);
  edge_condense<NB>(wr, ar, cr, pr, bad);
  if (bad && (threadIdx.x & 63) == 0) atomicOr(bf.status, ST_NOT_PD);
  mf_store(bf.EA + rs * nn, n, ar, n, n);  // the out-edge record: the tape of this compression
  mf_store(bf.EC + rs * nn, n, cr, n, n);
  mf_store(bf.EP + rs * nn, n, pr, n, n);
  dv4 pt;  // Pt = P_r + U_j, added in the working type as the stored values would be
#pragma unroll
  for (int v = 0; v < 4; ++v) pt[v] = (double)((T)pr[v] + (T)qj[v]);
  mf_store(L, LD, pt, NB, NB);
  mf_store(L + BS, LD, ar, NB, NB);
  mf_store(L + 2 * BS, LD, al, NB, NB);
  mf_store(L + 3 * BS, LD, cl, NB, NB);
  team_sync();
  compress_core<T, NB>(bf, o.d, mf_round<T>(cr), mf_round<T>(pl), L);
}

// Workgroups [0, nr): the level-1 rakes ops[r0 ..]; [nr, nr + nc): the level-1
// compressions ops[c0 ..]; then the edge slots rest[] that no level-1
// primitive consumes, condensed on their own.
template <typename T, int NB>
__device__ __forceinline__ void level1_body(const Bufs<T> &bf, const OpRec *__restrict__ ops, int64_t r0, int nr,
                                            int64_t c0, int nc, const int32_t *__restrict__ rest, T *L) {
  const int b = (int)blockIdx.x;
  if (b < nr)
    rake1_wide<T, NB>(bf, ops[r0 + b], L);
  else if (b < nr + nc)
    compress1_wide<T, NB>(bf, ops[c0 + (b - nr)], L);
  else
    condense_one_wide<T, NB>(bf, rest[b - nr - nc]);
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_level1_wide(Bufs<T> bf, const OpRec *__restrict__ ops, int64_t r0, int nr, int64_t c0,
                                      int nc, const int32_t *__restrict__ rest) {
  extern __shared__ double smd[];
  if (bf.n == NB)
    level1_body<T, NB>(exact_n<NB>(bf), ops, r0, nr, c0, nc, rest, reinterpret_cast<T *>(smd));
  else
    level1_body<T, NB>(bf, ops, r0, nr, c0, nc, rest, reinterpret_cast<T *>(smd));
}

// The condensation of every edge slot on its own (the first level then reads
// edge records), one edge per wavefront; the root's slot holds no edge.
template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_condense_wide(Bufs<T> bf) {
  const int64_t e = blockIdx.x;
  if (bf.parent[e] < 0) return;
  if (bf.n == NB)
    condense_one_wide<T, NB>(exact_n<NB>(bf), e);
  else
    condense_one_wide<T, NB>(bf, e);
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
