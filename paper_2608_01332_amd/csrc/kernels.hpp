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
// The team-layout local factor holds more per lane than the level kernels;
// its LDS already limits it to 3 wavefronts per SIMD from NB = 6 on.
template <int NB>
constexpr int lf_waves_per_eu() {
  return NB <= 4 ? 4 : (NB <= 8 ? 3 : 2);
}

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
  const int row = gj_team<T, NB, W, TW>(M, Lp, r, status);
  T x[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) x[q] = M[NB + q];
  lds_put_at(LX, x, row, r);
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
  return team_stride<T>(5 * NB * NB + 6 * NB * (int)(sizeof(double) / sizeof(T)));
}

// ---------------------------------------------------------------- factor kernels
// The single-pass kernels (condense, local factor, right-hand-side init, local
// affine solve, recovery) give each wavefront PW consecutive nodes, one per
// team.  Their per-node blocks are contiguous ranges, moved between HBM and
// per-team LDS tiles with coalesced accesses (team.hpp, stage_*), so the row
// layout of the team arithmetic never reaches global memory.

// Per-team LDS of k_condense (doubles): A, Delta and the output Pbar (NB x NB;
// A and Delta are overwritten by Abar and Cbar), B, S, Bt, St (NB x MB), R (MB x MB).
template <int NB, int MB>
struct CondLay {
  static constexpr int LA = NB + 1, LB = MB + 1;  // padded strides of the tiles read a row per lane
  static constexpr int A = 0, D = NB * LA, P = 2 * NB * LA, B = 3 * NB * LA, S = B + NB * LB, Bt = S + NB * LB,
                       St = Bt + NB * MB, R = St + NB * MB, words = team_stride<double>(R + MB * MB);
};

template <typename T, int NB, int MB>
__device__ __forceinline__ void condense_body(const Bufs<T> &bf) {
  // One team per node v: U_v = Q_v; for v != root, in float64 with the
  // Cholesky factor L of R_v:  Bt = B L^{-T},  St = M L^{-T}  (rows, n x m)
  //   Abar = A - Bt St^T,  Cbar = Delta_v + Bt Bt^T,  Pbar = -St St^T.
  using Ly = CondLay<NB, MB>;
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW, TS = Ly::words;
  extern __shared__ double smd[];
  const int lane = threadIdx.x & 63, team = lane / TW, r = lane % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW;
  const int cnt = (int)((bf.N - v0) < PW ? (bf.N - v0) : PW);
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n;
  range_copy<PW * NB * NB>(bf.U + v0 * nn, bf.Q + v0 * nn, cnt * (int)nn, lane);  // U = Q
  {
    double ra[Tile<PW, NB, NB>::IT], rd[Tile<PW, NB, NB>::IT];
    stage_load<PW, NB, NB>(ra, bf.A, v0, cnt, n, n, lane);
    stage_load<PW, NB, NB>(rd, bf.De, v0, cnt, n, n, lane);
    double rb[Tile<PW, NB, MB>::IT], rs[Tile<PW, NB, MB>::IT], rq[Tile<PW, MB, MB>::IT];
    stage_load<PW, NB, MB>(rb, bf.B, v0, cnt, n, m, lane);
    stage_load<PW, NB, MB>(rs, bf.S, v0, cnt, n, m, lane);
    stage_load<PW, MB, MB>(rq, bf.R, v0, cnt, m, m, lane);
    stage_put<PW, NB, NB, Ly::LA>(smd + Ly::A, TS, ra, lane);
    stage_put<PW, NB, NB, Ly::LA>(smd + Ly::D, TS, rd, lane);
    stage_put<PW, NB, MB, Ly::LB>(smd + Ly::B, TS, rb, lane);
    stage_put<PW, NB, MB, Ly::LB>(smd + Ly::S, TS, rs, lane);
    stage_put<PW, MB, MB>(smd + Ly::R, TS, rq, lane);
  }
  team_sync();
  const bool active = team < cnt;
  const int64_t v = v0 + (active ? team : 0);
  const bool edge = active && bf.parent[v] >= 0;
  const uint64_t noedge = __ballot(r == 0 && !edge);
  double *L = smd + team * TS, *LR = L + Ly::R, *LBt = L + Ly::Bt, *LSt = L + Ly::St;
  // Cholesky of R (lane 0, sequential; padded with the identity)
  if (r == 0) {
    for (int i = 0; i < MB; ++i)
      for (int j = 0; j < MB; ++j)
        if (i >= m || j >= m) LR[i * MB + j] = (i == j) ? 1.0 : 0.0;
    for (int j = 0; j < MB; ++j) {
      double s = LR[j * MB + j];
      for (int k = 0; k < j; ++k) s -= LR[j * MB + k] * LR[j * MB + k];
      if (edge && !(s > 0.0)) atomicOr(bf.status, ST_NOT_PD);
      const double d = sqrt(s);
      LR[j * MB + j] = d;
      for (int i = j + 1; i < MB; ++i) {
        double t = LR[i * MB + j];
        for (int k = 0; k < j; ++k) t -= LR[i * MB + k] * LR[j * MB + k];
        LR[i * MB + j] = t / d;
      }
    }
  }
  team_sync();
  const int rr = r < NB ? r : NB - 1;
  double bt[MB], st[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    bt[c] = L[Ly::B + rr * Ly::LB + c];
    st[c] = L[Ly::S + rr * Ly::LB + c];
  }
#pragma unroll
  for (int c = 0; c < MB; ++c) {  // forward substitution L y = row^T
    double sb = bt[c], ss = st[c];
#pragma unroll
    for (int k = 0; k < c; ++k) {
      sb -= LR[c * MB + k] * bt[k];
      ss -= LR[c * MB + k] * st[k];
    }
    bt[c] = sb / LR[c * MB + c];
    st[c] = ss / LR[c * MB + c];
  }
  if (r < NB) {
#pragma unroll
    for (int c = 0; c < MB; ++c) {
      LBt[r * MB + c] = bt[c];
      LSt[r * MB + c] = st[c];
    }
  }
  team_sync();
  double oa[NB], oc[NB], op[NB];
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
    oa[j] = L[Ly::A + rr * Ly::LA + j] - sbs;
    oc[j] = L[Ly::D + rr * Ly::LA + j] + sbb;
    op[j] = -sss;
    pin1(oa[j]);
    pin1(oc[j]);
    pin1(op[j]);
    mem_fence_compiler();
  }
  if (r < NB) {  // each lane overwrites only its own rows of A and Delta
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      L[Ly::A + r * Ly::LA + j] = oa[j];
      L[Ly::D + r * Ly::LA + j] = oc[j];
      L[Ly::P + r * Ly::LA + j] = op[j];
    }
  }
  team_sync();
  // the edge records of every team but the edge-less ones (the root, idle teams)
  stage_store<PW, NB, NB, false, Ly::LA>(bf.EA, smd + Ly::A, TS, v0, cnt, n, n, lane, noedge, TW);
  stage_store<PW, NB, NB, false, Ly::LA>(bf.EC, smd + Ly::D, TS, v0, cnt, n, n, lane, noedge, TW);
  stage_store<PW, NB, NB, false, Ly::LA>(bf.EP, smd + Ly::P, TS, v0, cnt, n, n, lane, noedge, TW);
}

template <typename T, int NB, int MB>
RCR_MAT_KERNEL(NB) void k_condense(Bufs<T> bf) {
  if (bf.n == NB && bf.m == MB)
    condense_body<T, NB, MB>(exact_nm<NB, MB>(bf));
  else if (bf.n == NB)
    condense_body<T, NB, MB>(exact_n<NB>(bf));
  else
    condense_body<T, NB, MB>(bf);
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
    T cn[NB], pl[NB];  // C_r and P_l, fetched with the other operands (not a round trip of their own later)
    ld_row(cn, bf.EC + rs * nn, n, r);
    ld_row(pl, bf.EP + l * nn, n, r);
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
    const int row = gj_team<ST, NB, W, TW>(M, reinterpret_cast<ST *>(Lp), r, bf.status);
    {
      T x[NB], y[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        x[q] = (T)M[NB + q];
        y[q] = (T)M[2 * NB + q];
      }
      lds_put_at(LX, x, row, r);
      lds_put_at(LY, y, row, r);
    }
    team_sync();
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
__device__ __forceinline__ void quad_level_body(const Bufs<T> &bf, const OpRec *__restrict__ ops, const Seg &sg) {
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

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_level(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  if (bf.n == NB)
    quad_level_body<T, NB>(exact_n<NB>(bf), ops, sg);
  else
    quad_level_body<T, NB>(bf, ops, sg);
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
__device__ __forceinline__ void quad_expand_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
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

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_quad_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  if (bf.n == NB)
    quad_expand_body<T, NB>(exact_n<NB>(bf), ops, off, cnt);
  else
    quad_expand_body<T, NB>(bf, ops, off, cnt);
}

// Per-team LDS of k_local_factor.  Words of T: P (then W, then A^cl), Finv,
// A (later T = F^-1 A^cl), B, WB (later K^T), pivot slots; then doubles: G
// (MB x MB).  Delta, S and R are read by their rows' own lanes straight from
// global memory, which keeps the footprint (and so the occupancy) of this
// latency-bound kernel at eight wavefronts per compute unit for NB = 12.
template <typename T, int NB, int MB>
struct LfLay {
  static constexpr int P = 0, Fi = NB * NB, A = 2 * NB * NB, B = 3 * NB * NB, WB = B + NB * MB, Lp = WB + NB * MB,
                       tend = Lp + 4 * NB;
  static constexpr int dbeg = (tend * (int)sizeof(T) + 7) / 8;  // in doubles
  static constexpr int G = dbeg, words = team_stride<double>(G + MB * MB);  // doubles per team
};

template <typename T, int NB, int MB>
__device__ __forceinline__ void local_factor_body(const Bufs<T> &bf, bool rhs, bool keep_acl) {
  // One team per node v:  F = I + Delta P, Finv, W = P F^-1; for v != root and
  // e = (parent, v):  WB = W B,  H^T = A^T WB + M,  G = R + B^T WB (float64
  // Cholesky),  K^T = -H^T G^-1,  G^-1,  A^cl = A + B K,  T = F^-1 A^cl.
  // With rhs: also h = q and z = K^T r + (A^cl)^T W c of the right-hand side
  // in bf (eq. (affine-edge)), in rhs_init's arithmetic order.
  using Ly = LfLay<T, NB, MB>;
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW, TS = Ly::words;
  constexpr int TST = TS * (int)(sizeof(double) / sizeof(T));  // team stride in words of T
  constexpr int W2 = 2 * NB;
  extern __shared__ double smd[];
  T *smt = reinterpret_cast<T *>(smd);
  const int lane = threadIdx.x & 63, team = lane / TW, r = lane % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW;
  const int cnt = (int)((bf.N - v0) < PW ? (bf.N - v0) : PW);
  const int n = bf.n, m = bf.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m;
  {
    T rp[Tile<PW, NB, NB>::IT];
    double ra[Tile<PW, NB, NB>::IT], rb[Tile<PW, NB, MB>::IT];
    stage_load<PW, NB, NB>(rp, bf.PW, v0, cnt, n, n, lane);
    stage_load<PW, NB, NB>(ra, bf.A, v0, cnt, n, n, lane);
    stage_load<PW, NB, MB>(rb, bf.B, v0, cnt, n, m, lane);
    stage_put<PW, NB, NB>(smt + Ly::P, TST, rp, lane);
    stage_put<PW, NB, NB>(smt + Ly::A, TST, ra, lane);
    stage_put<PW, NB, MB>(smt + Ly::B, TST, rb, lane);
  }
  team_sync();
  const bool active = team < cnt;
  const int64_t v = v0 + (active ? team : 0);
  const bool isroot = active && bf.parent[v] < 0;
  const bool edge = active && !isroot;
  const uint64_t noedge = __ballot(r == 0 && !edge);
  T *L = smt + team * TST;
  T *LP = L + Ly::P, *LFi = L + Ly::Fi, *LA = L + Ly::A, *LB = L + Ly::B, *LWB = L + Ly::WB;
  T *LKt = LWB, *Lp = L + Ly::Lp;
  double *LG = smd + team * TS + Ly::G;
  T *Lrhs = reinterpret_cast<T *>(LG);  // c, then r, of the right-hand side (G's block while it is free)
  constexpr int RPL = (MB + TW - 1) / TW;  // entries of r per lane: r, r + TW, ...
  T c_own = (T)0, r_own[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) r_own[i] = (T)0;
  if (rhs && active) {
    if (r < n) c_own = bf.sc[v * n + r];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (r + i * TW < m) r_own[i] = bf.sr[v * m + r + i * TW];
    if (r < n) bf.h[v * n + r] = bf.sq[v * n + r];
  }
  if (r < NB) Lrhs[r] = c_own;
  if (isroot) {  // P_root = U_root (eq. (value-reconstruction) at the root), also its output
    T u[NB];
    ld_row(u, bf.U + v * nn, n, r);
    st_row(bf.PW + v * nn, u, n, r, true);
    lds_put(LP, u, r);
  }
  team_sync();
  const int rr = r < NB ? r : NB - 1;
  T pv[NB], dv[NB], av[NB], bv[MB];
  stage_row<NB, NB>(pv, LP, r);
  ld_row(dv, bf.De + v * nn, n, r);
  stage_row<NB, NB>(av, LA, r);
  stage_row<NB, MB>(bv, LB, r);
  T M[W2];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    M[q] = (q == r) ? (T)1 : (T)0;
    M[NB + q] = (q == r) ? (T)1 : (T)0;
  }
  mac_rowL<T, NB, W2>(M, 0, dv, LP);  // F = I + Delta P  |  I
  const int row = gj_team<T, NB, W2, TW>(M, Lp, r, bf.status);
  T fi[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) fi[q] = M[NB + q];
  lds_put_at(LFi, fi, row, r);
  team_sync();
  lds_row(fi, LFi, r);  // row r of F^-1
  T wv[NB];
  zero(wv);
  mac_rowL<T, NB, NB>(wv, 0, pv, LFi);  // W = P F^-1
  lds_put(LP, wv, r);                   // P was last read for F: its tile passes W out
  T wc = (T)0;                          // (W c)_r of the right-hand side
  if (rhs) {
#pragma unroll
    for (int k = 0; k < NB; ++k) wc = fmat(wv[k], Lrhs[k], wc);
  }
  team_sync();
  stage_store<PW, NB, NB>(bf.W, smt + Ly::P, TST, v0, cnt, n, n, lane);
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
  // K^T row r = -G^{-1} H^T[r]  (two triangular solves); zero at the root
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
  for (int c = 0; c < MB; ++c) kt[c] = isroot ? (T)0 : (T)(-ht[c]);
  if (r < NB) {  // WB was last read before the Cholesky
#pragma unroll
    for (int c = 0; c < MB; ++c) LKt[r * MB + c] = kt[c];
  }
  // G^{-1} rows c (lanes c < m), m x m per edge
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
  lds_put(LP, acl, r);  // A^cl replaces W (already stored)
  team_sync();
  T tv[NB];
  zero(tv);
  mac_rowL<T, NB, NB>(tv, 0, fi, LP);  // T = F^-1 A^cl
  lds_put(LA, tv, r);                  // A was last read for H^T
  team_sync();
  stage_store<PW, NB, NB>(bf.Finv, smt + Ly::Fi, TST, v0, cnt, n, n, lane);
  if (keep_acl) stage_store<PW, NB, NB>(bf.Acl, smt + Ly::P, TST, v0, cnt, n, n, lane, noedge, TW);
  stage_store<PW, NB, NB>(bf.Tm, smt + Ly::A, TST, v0, cnt, n, n, lane, noedge, TW);
  stage_store<PW, MB, NB, true>(bf.Kw, smt + Ly::WB, TST, v0, cnt, m, n, lane);  // K = (K^T)^T, m x n
  if (rhs) {  // G's block is dead since the G^-1 rows, the pivot-row scratch since the elimination
    if (r < NB) Lp[r] = wc;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (r + i * TW < MB) Lrhs[r + i * TW] = r_own[i];
    team_sync();
    T z = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) z = fmat(LP[k * NB + rr], Lp[k], z);  // (A^cl)^T W c
#pragma unroll
    for (int k = 0; k < MB; ++k) z = fmat(kt[k], Lrhs[k], z);  // + K^T r
    if (active && r < n) bf.z[v * n + r] = edge ? z : (T)0;
  }
}

template <typename T, int NB, int MB>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(lf_waves_per_eu<NB>())))
void k_local_factor(Bufs<T> bf, int flags) {  // flags as for k_local_factor_wide
  const bool rhs = (flags & 1) != 0, keep_acl = (flags & 2) == 0;
  if (bf.n == NB && bf.m == MB)
    local_factor_body<T, NB, MB>(exact_nm<NB, MB>(bf), rhs, keep_acl);
  else if (bf.n == NB)
    local_factor_body<T, NB, MB>(exact_n<NB>(bf), rhs, keep_acl);
  else
    local_factor_body<T, NB, MB>(bf, rhs, keep_acl);
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
__device__ __forceinline__ void tcompose_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt,
                                              int64_t blk) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  extern __shared__ double smd[];
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  T *L = reinterpret_cast<T *>(smd) + team * lds_quad_words<T, NB>();
  const int64_t q0 = blk * PW + team;
  const bool active = q0 < cnt;
  const Op4 o = ops[off + (active ? q0 : cnt - 1)];
  tcomp_op_team<T, NB>(bf, o, L, r, active);
}

template <typename T, int NB>
RCR_MAT_KERNEL(NB) void k_tcompose(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  if (bf.n == NB)
    tcompose_body<T, NB>(exact_n<NB>(bf), ops, off, cnt, blockIdx.x);
  else
    tcompose_body<T, NB>(bf, ops, off, cnt, blockIdx.x);
}

// ---------------------------------------------------------------- solve kernels
// Vector primitives: one team per op, lane r computes entry r.  Inputs that
// every lane needs are read from global memory (broadcast within a team).

// Per-team LDS of k_rhs_init (words of T): W (NB rows of stride NB + 1,
// read a row per lane), A^cl (NB x NB), K (MB x NB), c, W c, z (NB), r (MB).
template <int NB, int MB>
struct RhsLay {
  static constexpr int LW = NB + 1;
  static constexpr int W = 0, Acl = NB * LW, K = Acl + NB * NB, c = K + MB * NB, wc = c + NB, z = wc + NB,
                       r = z + NB, words = r + MB;
};

template <typename T, int NB, int MB>
__device__ __forceinline__ void rhs_init_body(const Bufs<T> &bf) {
  // h_i = q_i;  z_e = K_e^T r_e + (A^cl_e)^T W_j c_j  (eq. (affine-edge))
  using Ly = RhsLay<NB, MB>;
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW, TS = team_stride<T>(Ly::words);
  extern __shared__ double smd[];
  T *smt = reinterpret_cast<T *>(smd);
  const int lane = threadIdx.x & 63, team = lane / TW, r = lane % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW;
  const int cnt = (int)((bf.N - v0) < PW ? (bf.N - v0) : PW);
  const int n = bf.n, m = bf.m;
  range_copy<PW * NB>(bf.h + v0 * n, bf.sq + v0 * n, cnt * n, lane);  // h = q
  {
    T rw[Tile<PW, NB, NB>::IT], ra[Tile<PW, NB, NB>::IT], rk[Tile<PW, MB, NB>::IT];
    T rc[Tile<PW, 1, NB>::IT], rr_[Tile<PW, 1, MB>::IT];
    stage_load<PW, NB, NB>(rw, bf.W, v0, cnt, n, n, lane);
    stage_load<PW, NB, NB>(ra, bf.Acl, v0, cnt, n, n, lane);
    stage_load<PW, MB, NB>(rk, bf.Kw, v0, cnt, m, n, lane);
    stage_load<PW, 1, NB>(rc, bf.sc, v0, cnt, 1, n, lane);
    stage_load<PW, 1, MB>(rr_, bf.sr, v0, cnt, 1, m, lane);
    stage_put<PW, NB, NB, Ly::LW>(smt + Ly::W, TS, rw, lane);
    stage_put<PW, NB, NB>(smt + Ly::Acl, TS, ra, lane);
    stage_put<PW, MB, NB>(smt + Ly::K, TS, rk, lane);
    stage_put<PW, 1, NB>(smt + Ly::c, TS, rc, lane);
    stage_put<PW, 1, MB>(smt + Ly::r, TS, rr_, lane);
  }
  team_sync();
  const bool active = team < cnt;
  const int64_t v = v0 + (active ? team : 0);
  const bool edge = active && bf.parent[v] >= 0;
  T *L = smt + team * TS;
  const int rr = r < NB ? r : NB - 1;
  T wc = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) wc = fmat(L[Ly::W + rr * Ly::LW + k], L[Ly::c + k], wc);
  if (r < NB) L[Ly::wc + r] = wc;
  team_sync();
  T s = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) s = fmat(L[Ly::Acl + k * NB + rr], L[Ly::wc + k], s);
#pragma unroll
  for (int k = 0; k < MB; ++k) s = fmat(L[Ly::K + k * NB + rr], L[Ly::r + k], s);
  if (r < NB) L[Ly::z + r] = edge ? s : (T)0;  // no edge at the root: z = 0
  team_sync();
  stage_store<PW, 1, NB>(bf.z, smt + Ly::z, TS, v0, cnt, 1, n, lane);
}

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_rhs_init(Bufs<T> bf) {
  if (bf.n == NB && bf.m == MB)
    rhs_init_body<T, NB, MB>(exact_nm<NB, MB>(bf));
  else if (bf.n == NB)
    rhs_init_body<T, NB, MB>(exact_n<NB>(bf));
  else
    rhs_init_body<T, NB, MB>(bf);
}

// One affine-contraction primitive of kind s (lane r of its team).
template <typename T, int NB>
__device__ __forceinline__ void aff_op(const Bufs<T> &bf, const OpRec &o, int s, int r) {
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  if (r >= n) return;
  if (s == OP_RAKE) {  // m = Z h_j + z,  Z = T^T;  p_j = h_j
    const int64_t j = o.a, e = o.b, out = o.c;
    T tv[NB], hv[NB];
    gather(tv, n, [&](int k) { return bf.Tm[e * nn + k * n + r]; });
    gather(hv, n, [&](int k) { return bf.h[j * n + k]; });
    bf.cv[out * n + r] = dot_n(tv, hv, n, bf.z[e * n + r]);
    bf.p[j * n + r] = bf.h[j * n + r];
  } else if (s == OP_COMBINE) {
    bf.cv[(int64_t)o.c * n + r] = bf.cv[(int64_t)o.a * n + r] + bf.cv[(int64_t)o.b * n + r];
  } else if (s == OP_ABSORB) {
    bf.h[(int64_t)o.a * n + r] += bf.cv[(int64_t)o.b * n + r];
  } else {  // z_new = z_l + Z_l (h_j + z_r)
    const int64_t j = o.a, l = o.b, rs = o.c, sn = o.d;
    T tv[NB], hv[NB], zv[NB];
    gather(tv, n, [&](int k) { return bf.Tm[l * nn + k * n + r]; });
    gather(hv, n, [&](int k) { return bf.h[j * n + k]; });
    gather(zv, n, [&](int k) { return bf.z[rs * n + k]; });
#pragma unroll
    for (int k = 0; k < NB; ++k) hv[k] += zv[k];
    bf.z[sn * n + r] = dot_n(tv, hv, n, bf.z[l * n + r]);
  }
}

template <typename T, int NB>
__device__ __forceinline__ void aff_level_body(const Bufs<T> &bf, const OpRec *__restrict__ ops, const Seg &sg,
                                               int blk) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  int s = 0;
  while (s < 3 && blk >= sg.blk[s + 1]) ++s;
  const int64_t idx = sg.off[s] + (int64_t)(blk - sg.blk[s]) * PW + team;
  if (idx >= sg.off[s + 1]) return;
  aff_op<T, NB>(bf, ops[idx], s, r);
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_aff_level(Bufs<T> bf, const OpRec *__restrict__ ops, Seg sg) {
  if (bf.n == NB)
    aff_level_body<T, NB>(exact_n<NB>(bf), ops, sg, blockIdx.x);
  else
    aff_level_body<T, NB>(bf, ops, sg, blockIdx.x);
}

// Affine expansion of one compression: p_j = Z_r p_k + h_j + z_r.
template <typename T, int NB>
__device__ __forceinline__ void affexp_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T tv[NB], pv[NB];
  gather(tv, n, [&](int q) { return bf.Tm[rs * nn + q * n + r]; });
  gather(pv, n, [&](int q) { return bf.p[k * n + q]; });
  bf.p[j * n + r] = dot_n(tv, pv, n, bf.h[j * n + r] + bf.z[rs * n + r]);
}

template <typename T, int NB>
__device__ __forceinline__ void aff_expand_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  affexp_op<T, NB>(bf, ops[off + q0], r);
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_aff_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                   int64_t cnt) {
  if (bf.n == NB)
    aff_expand_body<T, NB>(exact_n<NB>(bf), ops, off, cnt);
  else
    aff_expand_body<T, NB>(bf, ops, off, cnt);
}

// Per-team LDS of k_local_affine (words of T): Delta, W, Finv (NB rows of
// stride NB + 1), B (NB rows of stride MB + 1), G^-1 (MB x MB), p, c, f, g,
// B k - f, b (NB), r, t, k (MB).  The padded strides keep the row-per-lane
// reads free of bank conflicts.
template <int NB, int MB>
struct LaLay {
  static constexpr int LR = NB + 1, LB = MB + 1;
  static constexpr int D = 0, W = NB * LR, Fi = 2 * NB * LR, B = 3 * NB * LR, Gi = B + NB * LB, p = Gi + MB * MB,
                       c = p + NB, f = c + NB, g = f + NB, wv = g + NB, b = wv + NB, r = b + NB, t = r + MB,
                       k = t + MB, words = k + MB;
};

template <typename T, int NB, int MB>
__device__ __forceinline__ void local_affine_body(const Bufs<T> &bf) {
  // f = Delta p - c, g = p - W f; e = (parent, v): k = -G^-1 (r + B^T g),
  // b = F^-1 (B k - f); root: x = -F^-1 f.  Teams cover max(NB, MB) lanes.
  using Ly = LaLay<NB, MB>;
  constexpr int NM = NB > MB ? NB : MB;
  constexpr int TW = TeamW<NM>::TW, PW = TeamW<NM>::PW, TS = team_stride<T>(Ly::words);
  extern __shared__ double smd[];
  T *smt = reinterpret_cast<T *>(smd);
  const int lane = threadIdx.x & 63, team = lane / TW, r = lane % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW;
  const int cnt = (int)((bf.N - v0) < PW ? (bf.N - v0) : PW);
  const int n = bf.n, m = bf.m;
  {
    double rd[Tile<PW, NB, NB>::IT], rb[Tile<PW, NB, MB>::IT];
    T rw[Tile<PW, NB, NB>::IT], rf[Tile<PW, NB, NB>::IT], rg[Tile<PW, MB, MB>::IT];
    T rp[Tile<PW, 1, NB>::IT], rc[Tile<PW, 1, NB>::IT], rr_[Tile<PW, 1, MB>::IT];
    stage_load<PW, NB, NB>(rd, bf.De, v0, cnt, n, n, lane);
    stage_load<PW, NB, NB>(rw, bf.W, v0, cnt, n, n, lane);
    stage_load<PW, NB, NB>(rf, bf.Finv, v0, cnt, n, n, lane);
    stage_load<PW, NB, MB>(rb, bf.B, v0, cnt, n, m, lane);
    stage_load<PW, MB, MB>(rg, bf.Ginv, v0, cnt, m, m, lane);
    stage_load<PW, 1, NB>(rp, bf.p, v0, cnt, 1, n, lane);
    stage_load<PW, 1, NB>(rc, bf.sc, v0, cnt, 1, n, lane);
    stage_load<PW, 1, MB>(rr_, bf.sr, v0, cnt, 1, m, lane);
    stage_put<PW, NB, NB, Ly::LR>(smt + Ly::D, TS, rd, lane);
    stage_put<PW, NB, NB, Ly::LR>(smt + Ly::W, TS, rw, lane);
    stage_put<PW, NB, NB, Ly::LR>(smt + Ly::Fi, TS, rf, lane);
    stage_put<PW, NB, MB, Ly::LB>(smt + Ly::B, TS, rb, lane);
    stage_put<PW, MB, MB>(smt + Ly::Gi, TS, rg, lane);
    stage_put<PW, 1, NB>(smt + Ly::p, TS, rp, lane);
    stage_put<PW, 1, NB>(smt + Ly::c, TS, rc, lane);
    stage_put<PW, 1, MB>(smt + Ly::r, TS, rr_, lane);
  }
  team_sync();
  const bool active = team < cnt;
  const int64_t v = v0 + (active ? team : 0);
  const bool isroot = active && bf.parent[v] < 0;
  const bool edge = active && !isroot;
  const uint64_t noedge = __ballot(r == 0 && !edge);
  T *L = smt + team * TS;
  if (isroot && r < n) {  // the root's value vector is h_root; it is also p_root
    const T hv = bf.h[v * n + r];
    L[Ly::p + r] = hv;
    bf.p[v * n + r] = hv;
  }
  team_sync();
  const int rr = r < NB ? r : NB - 1;
  const int rm = r < MB ? r : MB - 1;
  T f = -L[Ly::c + rr];
#pragma unroll
  for (int k = 0; k < NB; ++k) f = fmat(L[Ly::D + rr * Ly::LR + k], L[Ly::p + k], f);
  if (r < NB) L[Ly::f + r] = f;
  team_sync();
  if (isroot) {  // x_root = -F^-1 f  (eq. (xroot))
    T x = (T)0;
#pragma unroll
    for (int k = 0; k < NB; ++k) x = fmat(-L[Ly::Fi + rr * Ly::LR + k], L[Ly::f + k], x);
    if (r < n) bf.xw[v * n + r] = x;
  }
  T g = L[Ly::p + rr];
#pragma unroll
  for (int k = 0; k < NB; ++k) g = fmat(-L[Ly::W + rr * Ly::LR + k], L[Ly::f + k], g);
  if (r < NB) L[Ly::g + r] = g;
  team_sync();
  T t = L[Ly::r + rm];  // lane c < m: r_c + (B^T g)_c
#pragma unroll
  for (int k = 0; k < NB; ++k) t = fmat(L[Ly::B + k * Ly::LB + rm], L[Ly::g + k], t);
  if (r < MB) L[Ly::t + r] = t;
  team_sync();
  T kk = (T)0;
#pragma unroll
  for (int d = 0; d < MB; ++d) kk = fmat(-L[Ly::Gi + rm * MB + d], L[Ly::t + d], kk);
  if (r < MB) L[Ly::k + r] = kk;
  team_sync();
  T wv = -f;  // lane r < n: (B k - f)_r
#pragma unroll
  for (int d = 0; d < MB; ++d) wv = fmat(L[Ly::B + rr * Ly::LB + d], L[Ly::k + d], wv);
  if (r < NB) L[Ly::wv + r] = wv;
  team_sync();
  T bb = (T)0;
#pragma unroll
  for (int k = 0; k < NB; ++k) bb = fmat(L[Ly::Fi + rr * Ly::LR + k], L[Ly::wv + k], bb);
  if (r < NB) L[Ly::b + r] = bb;
  team_sync();
  stage_store<PW, 1, MB>(bf.kff, smt + Ly::k, TS, v0, cnt, 1, m, lane, noedge, TW);
  stage_store<PW, 1, NB>(bf.b, smt + Ly::b, TS, v0, cnt, 1, n, lane, noedge, TW);
}

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_local_affine(Bufs<T> bf) {
  if (bf.n == NB && bf.m == MB)
    local_affine_body<T, NB, MB>(exact_nm<NB, MB>(bf));
  else if (bf.n == NB)
    local_affine_body<T, NB, MB>(exact_n<NB>(bf));
  else
    local_affine_body<T, NB, MB>(bf);
}

// State-offset composition of one compression: b_new = T_r b_l + b_r.
template <typename T, int NB>
__device__ __forceinline__ void state_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t l = o.a, rs = o.b, sn = o.c;
  T tv[NB], bv[NB];
  gather(tv, n, [&](int k) { return bf.Tm[rs * nn + r * n + k]; });
  gather(bv, n, [&](int k) { return bf.b[l * n + k]; });
  bf.b[sn * n + r] = dot_n(tv, bv, n, bf.b[rs * n + r]);
}

template <typename T, int NB>
__device__ __forceinline__ void state_level_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  state_op<T, NB>(bf, ops[off + q0], r);
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_state_level(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                    int64_t cnt) {
  if (bf.n == NB)
    state_level_body<T, NB>(exact_n<NB>(bf), ops, off, cnt);
  else
    state_level_body<T, NB>(bf, ops, off, cnt);
}

// State expansion of one removed node: x_j = T_s x_i + b_s.
template <typename T, int NB>
__device__ __forceinline__ void sexp_op(const Bufs<T> &bf, const Op4 &o, int r) {
  if (r >= bf.n) return;
  const int n = bf.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t j = o.a, sl = o.b, i = o.c;
  T tv[NB], xv[NB];
  gather(tv, n, [&](int k) { return bf.Tm[sl * nn + r * n + k]; });
  gather(xv, n, [&](int k) { return bf.xw[i * n + k]; });
  bf.xw[j * n + r] = dot_n(tv, xv, n, bf.b[sl * n + r]);
}

template <typename T, int NB>
__device__ __forceinline__ void state_expand_body(const Bufs<T> &bf, const Op4 *__restrict__ ops, int64_t off, int64_t cnt) {
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW;
  const int team = threadIdx.x / TW, r = threadIdx.x % TW;
  const int64_t q0 = (int64_t)blockIdx.x * PW + team;
  if (q0 >= cnt) return;
  sexp_op<T, NB>(bf, ops[off + q0], r);
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_state_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                     int64_t cnt) {
  if (bf.n == NB)
    state_expand_body<T, NB>(exact_n<NB>(bf), ops, off, cnt);
  else
    state_expand_body<T, NB>(bf, ops, off, cnt);
}

// Per-team LDS of k_recover (words of T): P (NB rows), K (MB rows), both of
// stride NB + 1 (read a row per lane), x, p, x of the parent, y (NB), k, u (MB).
template <int NB, int MB>
struct RecLay {
  static constexpr int LR = NB + 1;
  static constexpr int P = 0, K = NB * LR, x = K + MB * LR, p = x + NB, xp = p + NB, y = xp + NB, k = y + NB,
                       u = k + MB, words = u + MB;
};

template <typename T, int NB, int MB>
__device__ __forceinline__ void recover_body(const Bufs<T> &bf) {
  // y_v = P_v x_v + p_v;  u_e = K_e x_parent + k_e;  non-finite check
  using Ly = RecLay<NB, MB>;
  constexpr int TW = TeamW<NB>::TW, PW = TeamW<NB>::PW, TS = team_stride<T>(Ly::words);
  extern __shared__ double smd[];
  T *smt = reinterpret_cast<T *>(smd);
  const int lane = threadIdx.x & 63, team = lane / TW, r = lane % TW;
  const int64_t v0 = (int64_t)blockIdx.x * PW;
  const int cnt = (int)((bf.N - v0) < PW ? (bf.N - v0) : PW);
  const int n = bf.n, m = bf.m;
  {
    T rp[Tile<PW, NB, NB>::IT], rk[Tile<PW, MB, NB>::IT], rx[Tile<PW, 1, NB>::IT], rv[Tile<PW, 1, NB>::IT];
    T rf[Tile<PW, 1, MB>::IT];
    stage_load<PW, NB, NB>(rp, bf.PW, v0, cnt, n, n, lane);
    stage_load<PW, MB, NB>(rk, bf.Kw, v0, cnt, m, n, lane);
    stage_load<PW, 1, NB>(rx, bf.xw, v0, cnt, 1, n, lane);
    stage_load<PW, 1, NB>(rv, bf.p, v0, cnt, 1, n, lane);
    stage_load<PW, 1, MB>(rf, bf.kff, v0, cnt, 1, m, lane);
    stage_put<PW, NB, NB, Ly::LR>(smt + Ly::P, TS, rp, lane);
    stage_put<PW, MB, NB, Ly::LR>(smt + Ly::K, TS, rk, lane);
    stage_put<PW, 1, NB>(smt + Ly::x, TS, rx, lane);
    stage_put<PW, 1, NB>(smt + Ly::p, TS, rv, lane);
    stage_put<PW, 1, MB>(smt + Ly::k, TS, rf, lane);
  }
  const bool active = team < cnt;
  const int64_t v = v0 + (active ? team : 0);
  const int64_t i = active ? (int64_t)bf.parent[v] : -1;
  T *L = smt + team * TS;
  if (r < NB) L[Ly::xp + r] = (i >= 0 && r < n) ? bf.xw[i * n + r] : (T)0;  // x of the parent (a gather)
  team_sync();
  const int rr = r < NB ? r : NB - 1;
  T y = L[Ly::p + rr];
#pragma unroll
  for (int k = 0; k < NB; ++k) y = fmat(L[Ly::P + rr * Ly::LR + k], L[Ly::x + k], y);
  if (r < NB) L[Ly::y + r] = y;
  bool bad = active && r < n && (!isfinite((double)y) || !isfinite((double)L[Ly::x + r]));
  for (int c = r; c < MB; c += TW) {
    T u = (T)0;
    if (i >= 0) {
      u = L[Ly::k + c];
#pragma unroll
      for (int k = 0; k < NB; ++k) u = fmat(L[Ly::K + c * Ly::LR + k], L[Ly::xp + k], u);
    }
    L[Ly::u + c] = u;
    bad = bad || (active && c < m && !isfinite((double)u));
  }
  if (bad) atomicOr(bf.status, ST_NONFINITE);
  team_sync();
  stage_store<PW, 1, NB>(bf.yw, smt + Ly::y, TS, v0, cnt, 1, n, lane);
  stage_store<PW, 1, MB>(bf.uw, smt + Ly::u, TS, v0, cnt, 1, m, lane);
}

template <typename T, int NB, int MB>
__global__ __launch_bounds__(64) void k_recover(Bufs<T> bf) {
  if (bf.n == NB && bf.m == MB)
    recover_body<T, NB, MB>(exact_nm<NB, MB>(bf));
  else if (bf.n == NB)
    recover_body<T, NB, MB>(exact_n<NB>(bf));
  else
    recover_body<T, NB, MB>(bf);
}

}  // namespace rcr
