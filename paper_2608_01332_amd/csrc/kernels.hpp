// Solver kernels for one padded block size NB (and padded control size MB).
//
// Factor (Algorithm 1, Steps 2-3), matrix primitives on teams of TW lanes:
//   k_condense      eq. (edge-components) and U_i = Q_i
//   k_quad_level    one dependency level: rake (eq. (quadratic-rake), which
//                   also records P_j = U_j, its expansion), combine, absorb,
//                   compress (eqs. (compress-intermediates), (composition))
//   k_quad_expand   one level of P_j = tau((A_r, C_r, P_r + U_j), P_k)
//                   (eq. (value-reconstruction))
//   k_local_factor  eqs. (FW), (factor-local)
//   k_tcompose      composite transition T_r T_l of each compression
//                   (eq. (transition-compose)); with it every solve pass is a
//                   matrix-vector pass
// Solve (Steps 4-6), vector primitives on the same teams:
//   k_rhs_init, k_aff_level, k_aff_expand   eqs. (affine-edge), (affine-rake),
//                                           (affine-compose), their inverses
//   k_local_affine                          eqs. (local-affine-solve), (xroot)
//   k_state_level, k_state_expand           eqs. (state-map), (transition-compose)
//   k_recover                               eq. (recover)
#pragma once

#include "team.hpp"

namespace rcr {

// Register budget of the matrix kernels: at least this many wavefronts per
// SIMD, so the compiler schedules the unrolled block arithmetic within
// 512 / WPE registers instead of spilling or collapsing occupancy.
template <int NB>
constexpr int mat_waves_per_eu() {
  return NB <= 6 ? 4 : (NB <= 8 ? 3 : 2);
}
#define RCR_MAT_KERNEL(NBV) \
  __global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(mat_waves_per_eu<NBV>())))

// ---------------------------------------------------------------- helpers
// tau(alpha, Ux) = Pm + A^T Ux (I + C Ux)^{-1} A, symmetrised, for a team.
//   a, c, pm: rows r of A, C, Pm; ux: row r of Ux.  LDS: LU (Ux), LA (A),
//   LX, LY (NB x NB each), Lp (4 NB).
template <typename T, int NB>
__device__ __forceinline__ void tau_team(T *__restrict__ out, const T (&a)[NB], const T (&c)[NB],
                                         const T (&pm)[NB], const T (&ux)[NB], T *L, int n, int r, bool active,
                                         int *status) {
  constexpr int TW = TeamW<NB>::TW;
  constexpr int W = 2 * NB;
  T *LU = L, *LA = L + NB * NB, *LX = L + 2 * NB * NB, *LY = L + 3 * NB * NB, *Lp = L + 4 * NB * NB;
  lds_put(LU, ux, r);
  lds_put(LA, a, r);
  team_sync();
  T M[W];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    M[q] = (q == r) ? (T)1 : (T)0;
    M[NB + q] = a[q];
  }
  mac_rowL<T, NB, W>(M, 0, c, LU);  // I + C Ux  |  A
  gj_team<T, NB, W, TW>(M, Lp, r, status);
  T x[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) x[q] = M[NB + q];
  lds_put(LX, x, r);
  team_sync();
  T y[NB];
  zero(y);
  mac_rowL<T, NB, NB>(y, 0, ux, LX);  // Y = Ux X
  lds_put(LY, y, r);
  team_sync();
  T o[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) o[q] = (T)0;
  mac_colL<T, NB>(o, LA, LY, r);  // A^T Y
  T full[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) full[q] = o[q];
  // out = Pm + sym(A^T Y)
  lds_put(LX, o, r);
  team_sync();
  const int rr = r < NB ? r : NB - 1;
#pragma unroll
  for (int q = 0; q < NB; ++q) full[q] = pm[q] + (T)0.5 * (o[q] + LX[q * NB + rr]);
  st_row(out, full, n, r, active);
  team_sync();
}

template <typename T, int NB>
__host__ __device__ constexpr int lds_quad_words() {
  // compress: Pt, Ar, Al, X, Y (5 NB^2) + float64 pivot slots (2 * 3 NB doubles);
  // rake: 4 NB^2 + 4 NB.  Counted in words of T.
  return 5 * NB * NB + 6 * NB * (int)(sizeof(double) / sizeof(T));
}

// ---------------------------------------------------------------- factor kernels
template <typename T, int NB, int MB>
RCR_MAT_KERNEL(NB) void k_condense(Bufs<T> bf) {
  // One team per node v: U_v = Q_v; for v != root, in float64 with the
  // Cholesky factor L of R_v:  Bt = B L^{-T},  St = M L^{-T}  (rows, n x m)
  //   Abar = A - Bt St^T,  Cbar = Delta_v + Bt Bt^T,  Pbar = -St St^T.
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  constexpr int LW = MB * MB + 2 * NB * MB;  // doubles per team
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW + team;
  const bool active = v0 < bf.N;
  const int64_t v = active ? v0 : bf.N - 1;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  double *L = smd + team * LW, *LBt = L + MB * MB, *LSt = LBt + NB * MB;
  {
    T q[NB];
    ld_row(q, bf.Q + v * nn, n, r);
    st_row(bf.U + v * nn, q, n, r, active);
  }
  const bool edge = (bf.parent[v] >= 0);
  // Cholesky of R (lane 0, sequential; R padded with the identity)
  if (r == 0) {
    for (int i = 0; i < MB; ++i)
      for (int j = 0; j < MB; ++j)
        L[i * MB + j] = (i < m && j < m) ? bf.R[v * m * m + i * m + j] : (i == j ? 1.0 : 0.0);
    for (int j = 0; j < MB; ++j) {
      double s = L[j * MB + j];
      for (int k = 0; k < j; ++k) s -= L[j * MB + k] * L[j * MB + k];
      if (edge && active && !(s > 0.0)) atomicOr(bf.status, ST_NOT_PD);
      const double d = sqrt(s);
      L[j * MB + j] = d;
      for (int i = j + 1; i < MB; ++i) {
        double t = L[i * MB + j];
        for (int k = 0; k < j; ++k) t -= L[i * MB + k] * L[j * MB + k];
        L[i * MB + j] = t / d;
      }
    }
  }
  team_sync();
  double bt[MB], st[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    bt[c] = (r < n && c < m) ? bf.B[v * nm + (int64_t)r * m + c] : 0.0;
    st[c] = (r < n && c < m) ? bf.S[v * nm + (int64_t)r * m + c] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < MB; ++c) {  // forward substitution L y = row^T
    double sb = bt[c], ss = st[c];
#pragma unroll
    for (int k = 0; k < c; ++k) {
      sb -= L[c * MB + k] * bt[k];
      ss -= L[c * MB + k] * st[k];
    }
    bt[c] = sb / L[c * MB + c];
    st[c] = ss / L[c * MB + c];
  }
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < MB; ++c) {
      LBt[r * MB + c] = bt[c];
      LSt[r * MB + c] = st[c];
    }
  }
  team_sync();
  T oa[NB], oc[NB], op[NB];
  const int rr = r < NB ? r : NB - 1;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double sbb = 0.0, sbs = 0.0, sss = 0.0;
#pragma unroll
    for (int c = 0; c < MB; ++c) {
      const double bj = LBt[j * MB + c], sj = LSt[j * MB + c];
      sbb = fma(bt[c], bj, sbb);
      sbs = fma(bt[c], sj, sbs);
      sss = fma(st[c], sj, sss);
    }
    const bool in = (rr < n && j < n);
    oa[j] = (T)((in ? bf.A[v * nn + (int64_t)rr * n + j] : 0.0) - sbs);
    oc[j] = (T)((in ? bf.De[v * nn + (int64_t)rr * n + j] : 0.0) + sbb);
    op[j] = (T)(-sss);
    pin1(oa[j]);
    pin1(oc[j]);
    pin1(op[j]);
    mem_fence_compiler();
  }
  st_row(bf.EA + v * nn, oa, n, r, active && edge);
  st_row(bf.EC + v * nn, oc, n, r, active && edge);
  st_row(bf.EP + v * nn, op, n, r, active && edge);
}

// One quadratic-contraction primitive of kind s on a team (lane r, LDS L).
template <typename T, int NB>
__device__ __forceinline__ void quad_op_team(const Bufs<T> &bf, const OpRec &o, int s, T *L, int r,
                                             bool active) {
  constexpr int TW = TeamW<NB>::TW;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  if (s == OP_RAKE) {
    const int64_t j = o.a, e = o.b, out = o.c;
    T a[NB], c[NB], pm[NB], u[NB];
    ld_row(u, bf.U + j * nn, n, r);
    ld_row(a, bf.EA + e * nn, n, r);
    ld_row(c, bf.EC + e * nn, n, r);
    ld_row(pm, bf.EP + e * nn, n, r);
    st_row(bf.PW + j * nn, u, n, r, active);  // expansion of a rake: P_j = U_j
    tau_team<T, NB>(bf.CT + out * nn, a, c, pm, u, L, n, r, active, bf.status);
  } else if (s == OP_COMBINE) {
    T a[NB], b[NB];
    ld_row(a, bf.CT + (int64_t)o.a * nn, n, r);
    ld_row(b, bf.CT + (int64_t)o.b * nn, n, r);
#pragma unroll
    for (int q = 0; q < NB; ++q) a[q] += b[q];
    st_row(bf.CT + (int64_t)o.c * nn, a, n, r, active);
  } else if (s == OP_ABSORB) {
    T a[NB], b[NB];
    ld_row(a, bf.U + (int64_t)o.a * nn, n, r);
    ld_row(b, bf.CT + (int64_t)o.b * nn, n, r);
#pragma unroll
    for (int q = 0; q < NB; ++q) a[q] += b[q];
    st_row(bf.U + (int64_t)o.a * nn, a, n, r, active);
  } else {
    // alpha_{lr} = alpha_r o_{U_j} alpha_l
    constexpr int W = 3 * NB;
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T *LPt = L, *LAr = L + NB * NB, *LAl = L + 2 * NB * NB, *LX = L + 3 * NB * NB, *LY = L + 4 * NB * NB;
    T *Lp = L + 5 * NB * NB;
    typedef double ST;  // the compress composition's (I + C_l Pt) solve is always float64
    ST M[W];
    {
      T pt[NB], uj[NB], al[NB], cl[NB];
      ld_row(pt, bf.EP + rs * nn, n, r);
      ld_row(uj, bf.U + j * nn, n, r);
      ld_row(al, bf.EA + l * nn, n, r);
      ld_row(cl, bf.EC + l * nn, n, r);
#pragma unroll
      for (int q = 0; q < NB; ++q) pt[q] += uj[q];
      lds_put(LPt, pt, r);
      lds_put(LAl, al, r);
      {
        T ar[NB];
        ld_row(ar, bf.EA + rs * nn, n, r);
        lds_put(LAr, ar, r);
      }
      team_sync();
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        M[q] = (q == r) ? (ST)1 : (ST)0;
        M[NB + q] = (ST)al[q];
        M[2 * NB + q] = (ST)0;
      }
      mac_rowL<ST, NB, W>(M, 0, cl, LPt);        // S = I + C_l Pt
      mac_rowLt<ST, NB, W>(M, 2 * NB, cl, LAr);  // C_l A_r^T
    }
    gj_team<ST, NB, W, TW>(M, reinterpret_cast<ST *>(Lp), r, bf.status);
    {
      T x[NB], y[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        x[q] = (T)M[NB + q];
        y[q] = (T)M[2 * NB + q];
      }
      lds_put(LX, x, r);
      lds_put(LY, y, r);
    }
    team_sync();
    T cn[NB];
    ld_row(cn, bf.EC + rs * nn, n, r);
    {
      T ar[NB], an[NB];
      lds_row(ar, LAr, r);
      zero(an);
      mac_rowL<T, NB, NB>(an, 0, ar, LX);  // A_r X
      st_row(bf.EA + sn * nn, an, n, r, active);
      mac_rowL<T, NB, NB>(cn, 0, ar, LY);  // C_r + A_r Y
    }
    T z[NB];
    {
      T pt[NB];
      lds_row(pt, LPt, r);
      zero(z);
      mac_rowL<T, NB, NB>(z, 0, pt, LX);  // Pt X
    }
    team_sync();
    lds_put(LPt, z, r);  // Z replaces Pt
    team_sync();
    T pn[NB];
    zero(pn);
    mac_colL<T, NB>(pn, LAl, LPt, r);  // A_l^T Z
    // symmetric stores: C_new via LY, P_new via LX
    {
      const int rr = r < NB ? r : NB - 1;
      lds_put(LY, cn, r);
      lds_put(LX, pn, r);
      team_sync();
      T pl[NB];
      ld_row(pl, bf.EP + l * nn, n, r);
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        cn[q] = (T)0.5 * (cn[q] + LY[q * NB + rr]);
        pn[q] = pl[q] + (T)0.5 * (pn[q] + LX[q * NB + rr]);
      }
      st_row(bf.EC + sn * nn, cn, n, r, active);
      st_row(bf.EP + sn * nn, pn, n, r, active);
    }
  }
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_level(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  constexpr int LW = lds_quad_words<T, NB>();
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  T *L = reinterpret_cast<T *>(smd) + team * LW;
  int s = 0;
  while (s < 3 && (int)blockIdx.x >= sg.blk[s + 1]) ++s;
  const int64_t idx = sg.off[s] + (int64_t)(blockIdx.x - sg.blk[s]) * PW + team;
  const bool active = idx < sg.off[s + 1];
  const OpRec o = ops[active ? idx : sg.off[s + 1] - 1];
  quad_op_team<T, NB>(bf, o, s, L, r, active);
}

// Expansion of one compression on a team: P_j = tau((A_r, C_r, P_r + U_j), P_k).
template <typename T, int NB>
__device__ __forceinline__ void qexp_op_team(const Bufs<T> &bf, const Op4 &o, T *L, int r, bool active) {
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T a[NB], c[NB], pm[NB], uj[NB], pk[NB];
  ld_row(a, bf.EA + rs * nn, n, r);
  ld_row(c, bf.EC + rs * nn, n, r);
  ld_row(pm, bf.EP + rs * nn, n, r);
  ld_row(uj, bf.U + j * nn, n, r);
  ld_row(pk, bf.PW + k * nn, n, r);
#pragma unroll
  for (int q = 0; q < NB; ++q) pm[q] += uj[q];
  tau_team<T, NB>(bf.PW + j * nn, a, c, pm, pk, L, n, r, active, bf.status);
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  constexpr int LW = lds_quad_words<T, NB>();
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  T *L = reinterpret_cast<T *>(smd) + team * LW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  const bool active = q0 < cnt;
  const Op4 o = ops[off + (active ? q0 : cnt - 1)];
  qexp_op_team<T, NB>(bf, o, L, r, active);
}

template <typename T, int NB, int MB>
__host__ __device__ constexpr int lds_lf_words() {
  // P, Finv, A, B, WB (later K^T rows), pivot slots (2 * 2 NB), G (MB^2 float64)
  return 3 * NB * NB + 2 * NB * MB + 4 * NB + 2 * MB * MB;
}

template <typename T, int NB, int MB>
RCR_MAT_KERNEL(NB) void k_local_factor(Bufs<T> bf) {
  // One team per node v:  F = I + Delta P, Finv, W = P F^-1; for v != root and
  // e = (parent, v):  WB = W B,  H^T = A^T WB + M,  G = R + B^T WB (float64
  // Cholesky),  K^T = -H^T G^-1,  G^-1,  A^cl = A + B K,  T = F^-1 A^cl.
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  constexpr int LW = lds_lf_words<T, NB, MB>();
  constexpr int W2 = 2 * NB;
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  T *L = reinterpret_cast<T *>(smd) + team * LW;
  T *LP = L, *LFi = L + NB * NB, *LA = L + 2 * NB * NB, *LB = L + 3 * NB * NB, *LWB = LB + NB * MB;
  T *LKt = LWB, *Lp = LWB + NB * MB;  // K^T rows reuse the WB rows once G and H are formed
  double *LG = reinterpret_cast<double *>(Lp + 4 * NB);  // NB even: 8-byte aligned
  const int64_t v0 = (int64_t)blockIdx.x * PW + team;
  const bool active = v0 < bf.N;
  const int64_t v = active ? v0 : bf.N - 1;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  const bool isroot = (bf.parent[v] < 0);
  const bool edge = active && !isroot;
  const int rr = r < NB ? r : NB - 1;
  T pv[NB], dv[NB];
  ld_row(pv, (isroot ? bf.U : bf.PW) + v * nn, n, r);
  ld_row(dv, bf.De + v * nn, n, r);
  if (isroot) st_row(bf.PW + v * nn, pv, n, r, active);
  lds_put(LP, pv, r);
  T av[NB];
  ld_row(av, bf.A + v * nn, n, r);
  lds_put(LA, av, r);
  T bv[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) bv[c] = (r < n && c < m) ? (T)bf.B[v * nm + (int64_t)r * m + c] : (T)0;
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < MB; ++c) LB[r * MB + c] = bv[c];
  }
  team_sync();
  T M[W2];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    M[q] = (q == r) ? (T)1 : (T)0;
    M[NB + q] = (q == r) ? (T)1 : (T)0;
  }
  mac_rowL<T, NB, W2>(M, 0, dv, LP);  // F = I + Delta P  |  I
  gj_team<T, NB, W2, TW>(M, Lp, r, bf.status);
  T fi[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) fi[q] = M[NB + q];
  st_row(bf.Finv + v * nn, fi, n, r, active);
  lds_put(LFi, fi, r);
  team_sync();
  T wv[NB];
  zero(wv);
  mac_rowL<T, NB, NB>(wv, 0, pv, LFi);  // W = P F^-1
  st_row(bf.W + v * nn, wv, n, r, active);
  // WB row r
  T wb[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) wb[c] = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
#pragma unroll
    for (int c = 0; c < MB; ++c) wb[c] = fmat(wv[k], LB[k * MB + c], wb[c]);
    if (k % 2 == 1) pin(wb, 0, MB);
  }
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < MB; ++c) LWB[r * MB + c] = wb[c];
  }
  team_sync();
  // H^T row r = (A^T WB)[r] + M[r];  G = R + B^T WB by lanes c < m (float64)
  double ht[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) ht[c] = (r < n && c < m) ? bf.S[v * nm + (int64_t)r * m + c] : 0.0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double akr = (double)LA[k * NB + rr];
#pragma unroll
    for (int c = 0; c < MB; ++c) ht[c] = fma(akr, (double)LWB[k * MB + c], ht[c]);
    if (k % 2 == 1) pin(ht, 0, MB);
  }
  for (int c = r; c < MB; c += TW) {
    for (int d = 0; d < MB; ++d) {
      double g = (c < m && d < m) ? bf.R[v * m * m + c * m + d] : (c == d ? 1.0 : 0.0);
      for (int k = 0; k < NB; ++k) g = fma((double)LB[k * MB + c], (double)LWB[k * MB + d], g);
      LG[c * MB + d] = g;
    }
  }
  team_sync();
  if (r == 0) {  // Cholesky of G in float64 (lane 0)
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
  // K^T row r = -G^{-1} H^T[r]  (two triangular solves)
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    double t = ht[c];
#pragma unroll
    for (int k = 0; k < c; ++k) t -= LG[c * MB + k] * ht[k];
    ht[c] = t / LG[c * MB + c];
  }
#pragma unroll
  for (int c = MB - 1; c >= 0; --c) {
    double t = ht[c];
#pragma unroll
    for (int k = c + 1; k < MB; ++k) t -= LG[k * MB + c] * ht[k];
    ht[c] = t / LG[c * MB + c];
  }
  T kt[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) kt[c] = (T)(-ht[c]);
  if (active && r < n) {
#pragma unroll
    for (int c = 0; c < MB; ++c)
      if (c < m) bf.Kw[v * nm + (int64_t)c * n + r] = isroot ? (T)0 : kt[c];
  }
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < MB; ++c) LKt[r * MB + c] = kt[c];
  }
  // G^{-1} rows c (lanes c < m)
  for (int c = r; c < m; c += TW) {
    double e[MB];
#pragma unroll
    for (int d = 0; d < MB; ++d) e[d] = (d == c) ? 1.0 : 0.0;
#pragma unroll
    for (int d = 0; d < MB; ++d) {
      double t = e[d];
#pragma unroll
      for (int k = 0; k < d; ++k) t -= LG[d * MB + k] * e[k];
      e[d] = t / LG[d * MB + d];
    }
#pragma unroll
    for (int d = MB - 1; d >= 0; --d) {
      double t = e[d];
#pragma unroll
      for (int k = d + 1; k < MB; ++k) t -= LG[k * MB + d] * e[k];
      e[d] = t / LG[d * MB + d];
    }
    if (edge) {
#pragma unroll
      for (int d = 0; d < MB; ++d)
        if (d < m) bf.Ginv[v * m * m + c * m + d] = (T)e[d];
    }
  }
  team_sync();
  // A^cl row r = A[r] + B[r] K = A[r][q] + sum_c B[r][c] K^T[q][c]
  T acl[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    T s2 = av[q];
#pragma unroll
    for (int c = 0; c < MB; ++c) s2 = fmat(bv[c], LKt[q * MB + c], s2);
    acl[q] = s2;
    pin1(acl[q]);
    mem_fence_compiler();
  }
  st_row(bf.Acl + v * nn, acl, n, r, edge);
  lds_put(LP, acl, r);  // A^cl replaces P in LDS
  team_sync();
  T tv[NB];
  zero(tv);
  mac_rowL<T, NB, NB>(tv, 0, fi, LP);  // T = F^-1 A^cl
  st_row(bf.Tm + v * nn, tv, n, r, edge);
}

// Composite transition of one compression on a team: T_new = T_r T_l.
template <typename T, int NB>
__device__ __forceinline__ void tcomp_op_team(const Bufs<T> &bf, const Op4 &o, T *L, int r, bool active) {
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  T tl[NB], tr[NB], out[NB];
  ld_row(tl, bf.Tm + (int64_t)o.a * nn, n, r);
  ld_row(tr, bf.Tm + (int64_t)o.b * nn, n, r);
  lds_put(L, tl, r);
  team_sync();
  zero(out);
  mac_rowL<T, NB, NB>(out, 0, tr, L);  // T_r T_l
  st_row(bf.Tm + (int64_t)o.c * nn, out, n, r, active);
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_tcompose(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  T *L = reinterpret_cast<T *>(smd) + team * lds_quad_words<T, NB>();
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  const bool active = q0 < cnt;
  const Op4 o = ops[off + (active ? q0 : cnt - 1)];
  tcomp_op_team<T, NB>(bf, o, L, r, active);
}

// ---------------------------------------------------------------- solve kernels
// Vector primitives: one team per op, lane r computes entry r.  Inputs that
// every lane needs are read from global memory (broadcast within a team).

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_rhs_init(Bufs<T> bf) {
  // h_i = q_i;  z_e = K_e^T r_e + (A^cl_e)^T W_j c_j  (eq. (affine-edge))
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t v = (int64_t)blockIdx.x * PW + team;
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n;
  if (r < n) bf.h[v * n + r] = bf.sq[v * n + r];
  if (bf.parent[v] < 0) {
    if (r < n) bf.z[v * n + r] = (T)0;
    return;
  }
  T wc = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (r < n && k < n) wc = fmat(bf.W[v * nn + r * n + k], bf.sc[v * n + k], wc);
  T s = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T wk = __shfl(wc, k, TW);
    if (r < n && k < n) s = fmat(bf.Acl[v * nn + k * n + r], wk, s);
  }
#pragma unroll
  for (int k = 0; k < MB; ++k)
    if (r < n && k < m) s = fmat(bf.Kw[v * n * m + k * n + r], bf.sr[v * m + k], s);
  if (r < n) bf.z[v * n + r] = s;
}

// One affine-contraction primitive of kind s (lane r of its team).
template <typename T, int NB>
__device__ __forceinline__ void aff_op(const Bufs<T> &bf, const OpRec &o, int s, int r) {
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  if (r >= n) return;
  if (s == OP_RAKE) {  // m = Z h_j + z,  Z = T^T;  p_j = h_j
    const int64_t j = o.a, e = o.b, out = o.c;
    T acc = bf.z[e * n + r];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) acc = fmat(bf.Tm[e * nn + k * n + r], bf.h[j * n + k], acc);
    bf.cv[out * n + r] = acc;
    bf.p[j * n + r] = bf.h[j * n + r];
  } else if (s == OP_COMBINE) {
    bf.cv[(int64_t)o.c * n + r] = bf.cv[(int64_t)o.a * n + r] + bf.cv[(int64_t)o.b * n + r];
  } else if (s == OP_ABSORB) {
    bf.h[(int64_t)o.a * n + r] += bf.cv[(int64_t)o.b * n + r];
  } else {  // z_new = z_l + Z_l (h_j + z_r)
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T acc = bf.z[l * n + r];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) acc = fmat(bf.Tm[l * nn + k * n + r], bf.h[j * n + k] + bf.z[rs * n + k], acc);
    bf.z[sn * n + r] = acc;
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_aff_level(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  int s = 0;
  while (s < 3 && (int)blockIdx.x >= sg.blk[s + 1]) ++s;
  const int64_t idx = sg.off[s] + (int64_t)(blockIdx.x - sg.blk[s]) * PW + team;
  if (idx >= sg.off[s + 1]) return;
  aff_op<T, NB>(bf, ops[idx], s, r);
}

// Affine expansion of one compression: p_j = Z_r p_k + h_j + z_r.
template <typename T, int NB>
__device__ __forceinline__ void affexp_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T acc = bf.h[j * n + r] + bf.z[rs * n + r];
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (q < n) acc = fmat(bf.Tm[rs * nn + q * n + r], bf.p[k * n + q], acc);
  bf.p[j * n + r] = acc;
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_aff_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                   int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  affexp_op<T, NB>(bf, ops[off + q0], r);
}

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_local_affine(Bufs<T> bf) {
  // f = Delta p - c, g = p - W f; e = (parent, v): k = -G^-1 (r + B^T g),
  // b = F^-1 (B k - f); root: x = -F^-1 f.  Teams cover max(NB, MB) lanes.
  constexpr int NM = NB > MB ? NB : MB;
  constexpr int TW = TeamW<NM>::TW, PW = TeamW<NM>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t v = (int64_t)blockIdx.x * PW + team;
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  const bool isroot = (bf.parent[v] < 0);
  const T *pv = isroot ? bf.h + v * n : bf.p + v * n;
  T f = (T)0;
  if (r < n) {
    f = -bf.sc[v * n + r];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) f = fmat((T)bf.De[v * nn + r * n + k], pv[k], f);
  }
  if (isroot) {
    if (r < n) bf.p[v * n + r] = pv[r];
    T x = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const T fk = __shfl(f, k, TW);
      if (r < n && k < n) x = fmat(-bf.Finv[v * nn + r * n + k], fk, x);
    }
    if (r < n) bf.xw[v * n + r] = x;
    return;
  }
  T g = (r < n) ? pv[r] : (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T fk = __shfl(f, k, TW);
    if (r < n && k < n) g = fmat(-bf.W[v * nn + r * n + k], fk, g);
  }
  T t = (r < m) ? bf.sr[v * m + r] : (T)0;  // lane c < m: r_c + (B^T g)_c
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T gk = __shfl(g, k, TW);
    if (r < m && k < n) t = fmat((T)bf.B[v * nm + k * m + r], gk, t);
  }
  T kk = (T)0;
#pragma unroll
  for (int d = 0; d < MB; ++d) {
    const T td = __shfl(t, d < TW ? d : 0, TW);
    if (r < m && d < m) kk = fmat(-bf.Ginv[v * m * m + r * m + d], td, kk);
  }
  if (r < m) bf.kff[v * m + r] = kk;
  T wv = -f;  // lane r < n: (B k - f)_r
#pragma unroll
  for (int d = 0; d < MB; ++d) {
    const T kd = __shfl(kk, d < TW ? d : 0, TW);
    if (r < n && d < m) wv = fmat((T)bf.B[v * nm + r * m + d], kd, wv);
  }
  T bb = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const T wk = __shfl(wv, k, TW);
    if (r < n && k < n) bb = fmat(bf.Finv[v * nn + r * n + k], wk, bb);
  }
  if (r < n) bf.b[v * n + r] = bb;
}

// State-offset composition of one compression: b_new = T_r b_l + b_r.
template <typename T, int NB>
__device__ __forceinline__ void state_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t l = o.a, rs = o.b, sn = o.c;
  T acc = bf.b[rs * n + r];
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k < n) acc = fmat(bf.Tm[rs * nn + r * n + k], bf.b[l * n + k], acc);
  bf.b[sn * n + r] = acc;
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_state_level(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                    int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  state_op<T, NB>(bf, ops[off + q0], r);
}

// State expansion of one removed node: x_j = T_s x_i + b_s.
template <typename T, int NB>
__device__ __forceinline__ void sexp_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, sl = o.b, i = o.c;
  T acc = bf.b[sl * n + r];
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k < n) acc = fmat(bf.Tm[sl * nn + r * n + k], bf.xw[i * n + k], acc);
  bf.xw[j * n + r] = acc;
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_state_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                     int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  sexp_op<T, NB>(bf, ops[off + q0], r);
}

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_recover(Bufs<T> bf) {
  // y_v = P_v x_v + p_v;  u_e = K_e x_parent + k_e;  non-finite check
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t v = (int64_t)blockIdx.x * PW + team;
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  bool bad = false;
  if (r < n) {
    T y = bf.p[v * n + r];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) y = fmat(bf.PW[v * nn + r * n + k], bf.xw[v * n + k], y);
    bf.yw[v * n + r] = y;
    bad = !isfinite((double)y) || !isfinite((double)bf.xw[v * n + r]);
  }
  for (int c = r; c < m; c += TW) {
    T u = (T)0;
    const int64_t i = bf.parent[v];
    if (i >= 0) {
      u = bf.kff[v * m + c];
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < n) u = fmat(bf.Kw[v * nm + c * n + k], bf.xw[i * n + k], u);
    }
    bf.uw[v * m + c] = u;
    bad = bad || !isfinite((double)u);
  }
  if (bad) atomicOr(bf.status, ST_NONFINITE);
}

}  // namespace rcr
