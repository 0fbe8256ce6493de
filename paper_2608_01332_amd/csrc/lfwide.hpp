// Local factor (eqs. (FW), (factor-local)) in the wide layout for NB in
// {12, 16}: one node per 64-lane wavefront, lane (q, r) owning row r and
// column quarter q of every NB x NB block (wide.hpp).  Per node v:
//   F = I + Delta P,  Finv by Gauss-Jordan in place (gj_inv_wide),  W = P Finv;
//   for the edge e = (parent, v):  WB = W B,  H^T = A^T WB + M,
//   G = R + B^T WB (float64 Cholesky),  K = -G^-1 H,  G^-1,
//   A^cl = A + B K,  T = Finv A^cl;
//   at the root P = U is also the output P.
// One wavefront per node shortens the dependent chain of the elimination
// four-fold against a 16-lane team and keeps enough wavefronts resident to
// hide it; the control-sized float64 work (G, its factor and inverse) is
// replicated in registers when m is at most 4.
#pragma once

#include "mfma.hpp"

namespace rcr {

template <typename T, int NB, int MB>
struct LfwLay {
  static constexpr int LD = WideCfg<NB>::LD, BS = WideCfg<NB>::BS, MBP = MB + 1;
  // words of T: P (later W), Delta (later H^T in float64, then A^cl), A, F
  // (inverted in place), B, WB (later K^T) (NB x MB each, row stride MB + 1)
  static constexpr int P = 0, D = BS, A = 2 * BS, M = 3 * BS, B = M + BS, WB = B + NB * MBP, Kt = WB,
                       Cv = WB + NB * MBP, Rv = Cv + NB, tend = Rv + MB;  // c, r: the first right-hand side
  // doubles: H^T (NB x MB; over Delta where it fits), G and G^-1 (MB x MB)
  static constexpr bool HD = D * sizeof(T) % 8 == 0 && NB * MBP * 8 <= BS * (int)sizeof(T);
  static constexpr int dbeg = (tend * (int)sizeof(T) + 7) / 8;
  static constexpr int Ht = HD ? D * (int)sizeof(T) / 8 : dbeg, G = HD ? dbeg : Ht + NB * MBP, Gi = G + MB * MB,
                       words = Gi + MB * MB;
};

// Cholesky factor and inverse of the MB x MB SPD matrix G (row-major in LDS)
// in registers; reports a non-positive pivot through `bad`.
template <int MB>
__device__ __forceinline__ void chol_inv_regs(const double *LG, double (&Gi)[MB][MB], bool &bad) {
  double L[MB][MB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) L[i][j] = (j <= i) ? LG[i * MB + j] : 0.0;
  double dinv[MB];
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    double s = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    bad = bad || !(s > 0.0);
    const double y = rsqrt_nr(s);  // 1 / sqrt(s)
    L[j][j] = s * y;
    dinv[j] = y;
#pragma unroll
    for (int i = j + 1; i < MB; ++i) {
      double t = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t * dinv[j];
    }
  }
  // Li = L^-1 (lower triangular), G^-1 = Li^T Li
  double Li[MB][MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) {
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * Li[k][c];
      Li[i][c] = (i >= c) ? t * dinv[i] : 0.0;
    }
  }
#pragma unroll
  for (int c = 0; c < MB; ++c)
#pragma unroll
    for (int d = 0; d < MB; ++d) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < MB; ++k) s += Li[k][c] * Li[k][d];
      Gi[c][d] = s;
    }
}

template <typename T, int NB, int MB>
__device__ __forceinline__ void local_factor_wide(const Bufs<T> &bf, bool rhs, bool keep_acl) {
  using Ly = LfwLay<T, NB, MB>;
  constexpr int CQ = WideCfg<NB>::CQ, TL = WideCfg<NB>::TILE, LD = Ly::LD, MBP = Ly::MBP;
  constexpr int TB = (NB * MB + 63) / 64;
  extern __shared__ double smd[];
  T *L = reinterpret_cast<T *>(smd);
  T *LP = L + Ly::P, *LDe = L + Ly::D, *LA = L + Ly::A, *LM = L + Ly::M;
  T *LB = L + Ly::B, *LWB = L + Ly::WB, *LKt = L + Ly::Kt, *LCv = L + Ly::Cv, *LRv = L + Ly::Rv;
  double *LH = smd + Ly::Ht, *LG = smd + Ly::G, *LGi = smd + Ly::Gi;
  const int64_t v = blockIdx.x;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  const int q = wq_of(), r = wr_of(), lane = (int)(threadIdx.x & 63);
  const int rr = r < NB ? r : NB - 1;
  const bool isroot = bf.parent[v] < 0;
  const bool edge = !isroot;
  // the lane's entries of M and R, loaded with the blocks (not after the elimination)
  constexpr int CM = (MB + 3) / 4;
  double sv[CM], rv[CM];
#pragma unroll
  for (int k = 0; k < CM; ++k) {
    const int c = q + 4 * k;
    sv[k] = (r < n && c < m) ? bf.S[v * nm + (int64_t)r * m + c] : 0.0;
    rv[k] = (r < MB && c < MB) ? ((r < m && c < m) ? bf.R[v * m * m + r * m + c] : (r == c ? 1.0 : 0.0)) : 0.0;
  }
  // c (lanes 0..NB-1) and r (lanes 16..16+MB-1) of the first right-hand side
  T crhs = (T)0;
  if (rhs) {
    if (lane < n)
      crhs = bf.sc[v * n + lane];
    else if (lane >= 16 && lane - 16 < m)
      crhs = bf.sr[v * m + lane - 16];
  }
  {
    T tP[TL], tD[TL], tA[TL], tB[TB];
    if (isroot && !bf.uabs[v])
      wfetch<T, NB>(tP, bf.Q + v * nn, n);  // a root never absorbed into (a one-node tree): U = Q
    else
      wfetch<T, NB>(tP, (isroot ? bf.U : bf.PW) + v * nn, n);
    wfetch<T, NB>(tD, bf.De + v * nn, n);
    wfetch<T, NB>(tA, bf.A + v * nn, n);
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int e = lane + 64 * u, i = e / MB, c = e % MB;
      tB[u] = (e < NB * MB && i < n && c < m) ? (T)bf.B[v * nm + (int64_t)i * m + c] : (T)0;
    }
    if (isroot) wstore_tile<T, NB>(bf.PW + v * nn, tP, n, true);  // P_root = U_root
    if (lane < NB) LCv[lane] = crhs;
    if (lane >= 16 && lane < 16 + MB) LRv[lane - 16] = crhs;
    wput<T, NB>(LP, LD, tP);
    wput<T, NB>(LDe, LD, tD);
    wput<T, NB>(LA, LD, tA);
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int e = lane + 64 * u, i = e / MB, c = e % MB;
      if (e < NB * MB) LB[i * MBP + c] = tB[u];
    }
  }
  team_sync();
  {  // F = I + Delta P
    const dv4 f = mf_mm<NB, false, false>(mf_ident(NB), LDe, LD, LP, LD);
    mf_store(LM, LD, f, NB, NB);
  }
  team_sync();
  gj_inv_wide<T, NB>(LM, bf.status, true);
  const T *LFi = LM;  // Finv, row stride LD
  {
    mf_store(bf.Finv + v * nn, n, mf_load(LFi, LD, NB, NB), n, n);
    const dv4 w = mf_mm<NB, false, false>(mf_zero(), LP, LD, LFi, LD);  // W = P Finv
    mf_store(bf.W + v * nn, n, w, n, n);
    team_sync();  // the reads of P precede its replacement by W
    mf_store(LP, LD, w, NB, NB);
  }
  team_sync();
  for (int c = q; c < MB; c += 4) {  // WB = W B
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) s = fmat(LP[rr * LD + k], LB[k * MBP + c], s);
    if (r < NB) LWB[r * MBP + c] = s;
  }
  team_sync();
#pragma unroll
  for (int k = 0; k < CM; ++k) {  // H^T = A^T WB + M (float64)
    const int c = q + 4 * k;
    if (c >= MB) break;
    double h = sv[k];
#pragma unroll
    for (int k = 0; k < NB; ++k) h = fma((double)LA[k * LD + rr], (double)LWB[k * MBP + c], h);
    if (r < NB) LH[r * MBP + c] = h;
  }
  if (r < MB) {
#pragma unroll
    for (int k = 0; k < CM; ++k) {  // G = R + B^T WB (float64; padded with the identity)
      const int c = q + 4 * k;
      if (c >= MB) break;
      double g = rv[k];
#pragma unroll
      for (int k = 0; k < NB; ++k) g = fma((double)LB[k * MBP + r], (double)LWB[k * MBP + c], g);
      LG[r * MB + c] = g;
    }
  }
  team_sync();
  if constexpr (MB <= 4) {
    double Gi[MB][MB];
    bool bad = false;
    chol_inv_regs<MB>(LG, Gi, bad);
    if (edge && lane == 0 && bad) atomicOr(bf.status, ST_NOT_PD);
    // G^-1 through LDS: lane 0 writes it, every lane reads row q and entry (r, q)
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int d = 0; d < MB; ++d) LGi[i * MB + d] = Gi[i][d];
    }
    team_sync();
    const int qq = q < MB ? q : 0, rq = r < MB ? r : 0;
    double gq[MB];
#pragma unroll
    for (int d = 0; d < MB; ++d) gq[d] = LGi[qq * MB + d];
    const double grq = LGi[rq * MB + qq];
    if (q < MB) {  // K^T row r, column q = -(G^-1 H^T[r])_q
      double kt = 0.0;
#pragma unroll
      for (int d = 0; d < MB; ++d) kt = fma(-gq[d], LH[rr * MBP + d], kt);
      if (isroot) kt = 0.0;
      if (r < NB) LKt[r * MBP + q] = (T)kt;
      if (r < n && q < m) bf.Kw[v * nm + (int64_t)q * n + r] = (T)kt;
    }
    if (edge && r < m && q < m) bf.Ginv[v * m * m + r * m + q] = (T)grq;
  } else {
    if (lane == 0) {  // Cholesky of G in float64 (lane 0)
      for (int j = 0; j < MB; ++j) {
        double s2 = LG[j * MB + j];
        for (int k = 0; k < j; ++k) s2 -= LG[j * MB + k] * LG[j * MB + k];
        if (edge && !(s2 > 0.0)) atomicOr(bf.status, ST_NOT_PD);
        const double d = sqrt(s2);
        LG[j * MB + j] = d;
        for (int i = j + 1; i < MB; ++i) {
          double t = LG[i * MB + j];
          for (int k = 0; k < j; ++k) t -= LG[i * MB + k] * LG[j * MB + k];
          LG[i * MB + j] = t / d;
        }
      }
    }
    team_sync();
    if (lane < MB) {  // row `lane` of G^-1 by two triangular solves
      const int c = lane;
      double e[MB];
      for (int d = 0; d < MB; ++d) e[d] = (d == c) ? 1.0 : 0.0;
      for (int d = 0; d < MB; ++d) {
        double t = e[d];
        for (int k = 0; k < d; ++k) t -= LG[d * MB + k] * e[k];
        e[d] = t / LG[d * MB + d];
      }
      for (int d = MB - 1; d >= 0; --d) {
        double t = e[d];
        for (int k = d + 1; k < MB; ++k) t -= LG[k * MB + d] * e[k];
        e[d] = t / LG[d * MB + d];
      }
      for (int d = 0; d < MB; ++d) LGi[c * MB + d] = e[d];
    }
    team_sync();
    for (int c = q; c < MB; c += 4) {
      double kt = 0.0;
      for (int d = 0; d < MB; ++d) kt = fma(-LGi[c * MB + d], LH[rr * MBP + d], kt);
      if (isroot) kt = 0.0;
      if (r < NB) LKt[r * MBP + c] = (T)kt;
      if (r < n && c < m) bf.Kw[v * nm + (int64_t)c * n + r] = (T)kt;
    }
    if (edge && r < m) {
      for (int c = q; c < m; c += 4) bf.Ginv[v * m * m + r * m + c] = (T)LGi[r * MB + c];
    }
  }
  team_sync();
  {  // A^cl = A + B K  (K[c][j] = K^T[j][c]); Delta's block (dead since F) keeps it
    T acl[CQ];
#pragma unroll
    for (int cc = 0; cc < CQ; ++cc) {
      const int j = q * CQ + cc;
      T s = LA[rr * LD + j];
#pragma unroll
      for (int c = 0; c < MB; ++c) s = fmat(LB[rr * MBP + c], LKt[j * MBP + c], s);
      acl[cc] = s;
    }
    if (edge && keep_acl) wstore_piece<T, NB>(bf.Acl + v * nn, acl, n, true);
    wput_piece<T, NB>(LDe, LD, acl);
  }
  team_sync();
  {
    const dv4 t = mf_mm<NB, false, false>(mf_zero(), LFi, LD, LDe, LD);  // T = Finv A^cl
    if (edge) mf_store(bf.Tm + v * nn, n, t, n, n);
  }
  if (rhs) {
    // The first right-hand side's h = q and z = K^T r + (A^cl)^T W c (eq.
    // (affine-edge)) from the blocks still in LDS (W over P, A^cl over Delta,
    // K^T), in the arithmetic order of the solve's own initialisation, so the
    // result is the same bit for bit.  B's block (dead) holds W c.
    T *Lwc = LB;
    const bool lead = q == 0;
    T wc = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) wc = fmat(LP[rr * LD + k], LCv[k], wc);
    if (lead && r < NB) Lwc[r] = wc;
    if (lead && r < n) bf.h[v * n + r] = bf.sq[v * n + r];
    team_sync();
    T z = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) z = fmat(LDe[k * LD + rr], Lwc[k], z);
#pragma unroll
    for (int k = 0; k < MB; ++k) z = fmat(LKt[rr * MBP + k], LRv[k], z);
    if (lead && r < n) bf.z[v * n + r] = edge ? z : (T)0;
  }
}

// One node per wavefront; the body is specialised for n = NB (and m = MB)
// when the blocks need no padding (exact_n, exact_nm).
// With bit 1 of flags it also initialises the solve of the right-hand side
// that Bufs carries (sq, sr, sc), which then skips its own initialisation;
// with bit 2 it leaves A^cl unstored (no later right-hand side needs it).
template <typename T, int NB, int MB>
RCR_MAT_KERNEL(NB) void k_local_factor_wide(Bufs<T> bf, int flags) {
  const bool rhs = (flags & 1) != 0, keep_acl = (flags & 2) == 0;
  if (bf.n == NB && bf.m == MB)
    local_factor_wide<T, NB, MB>(exact_nm<NB, MB>(bf), rhs, keep_acl);
  else if (bf.n == NB)
    local_factor_wide<T, NB, MB>(exact_n<NB>(bf), rhs, keep_acl);
  else
    local_factor_wide<T, NB, MB>(bf, rhs, keep_acl);
}

}  // namespace rcr
