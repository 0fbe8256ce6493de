// HIP kernels (gfx950) and the launch sequence of one factor + solve.
//
// Mapping.  Every matrix primitive (condensation, rake, compress, their
// expansion, local factor, composite transition) is executed by one 64-lane
// wavefront = one workgroup; its n x n blocks (n <= 16) are staged in LDS,
// products are computed lane-per-output-element, nonsymmetric solves
// (I + C U, S = I + C_l Pt, F = I + Delta P) use Gauss-Jordan elimination with
// partial pivoting, and the SPD solves (R_e, G_e) use Cholesky.  Vector
// primitives (affine and state passes, recovery) run on 16-lane teams, four
// per wavefront, exchanging values with width-16 shuffles.  Node and edge data
// are structure-of-arrays with one contiguous block per node or edge slot, so
// each primitive reads its operands as contiguous runs.
//
// Data flow (Algorithm 1):
//   condense (eq. (edge-components)); U_i = Q_i             (one launch)
//   quadratic contraction: rake (eq. (quadratic-rake)), combine, absorb,
//     compress (eq. (quadratic-compress)), one launch per dependency level;
//     a rake also records P_j = U_j, its expansion
//   quadratic expansion of compressions (eq. (quadratic-expand-compress))
//   local factors (eqs. (FW), (factor-local)) and the composite transition
//     matrices of every compression (T_r T_l of eq. (transition-compose));
//     these are RHS-independent, so the solve passes below are vector-only
//   affine contraction/expansion (eqs. (affine-edge), (affine-rake),
//     (affine-compose)), local affine solve and root state (eqs.
//     (local-affine-solve), (xroot)), state-offset contraction and state
//     expansion (eqs. (state-map), (transition-compose)), recovery (eq. (recover)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "device.hpp"

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
  int *status;
};

// ------------------------------------------------------------ 64-lane helpers
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  return fma(a, b, c);
}

// C (r x c) = | += | -= op(A) op(B) with op(A) r x k, op(B) k x c; leading dimensions
// are row strides.  C must not alias A or B.
template <typename T, bool TA, bool TB, int MODE>
__device__ __forceinline__ void mm64(T *C, int ldc, const T *A, int lda, const T *B, int ldb, int r,
                                     int k, int c) {
  const int total = r * c;
  for (int e = threadIdx.x; e < total; e += 64) {
    const int i = e / c, j = e - i * c;
    T s = 0;
    for (int l = 0; l < k; ++l) {
      const T a = TA ? A[l * lda + i] : A[i * lda + l];
      const T bb = TB ? B[j * ldb + l] : B[l * ldb + j];
      s = fma_t(a, bb, s);
    }
    if (MODE == 0)
      C[i * ldc + j] = s;
    else if (MODE == 1)
      C[i * ldc + j] += s;
    else
      C[i * ldc + j] -= s;
  }
}

template <typename D, typename S>
__device__ __forceinline__ void load64(D *dst, const S *__restrict__ src, int count) {
  for (int e = threadIdx.x; e < count; e += 64) dst[e] = (D)src[e];
}

// Gauss-Jordan elimination with partial pivoting on the n x w row-major matrix
// M (row stride ld): solves M[:, :n] X = M[:, n:w]; X is left in M[:, n:w].
// Columns left of the pivot are never read again and are not cleared.
template <typename T>
__device__ void gj64(T *M, int ld, int n, int w, int *status) {
  const int lane = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    T v = (lane >= k && lane < n) ? (T)fabs(M[lane * ld + k]) : (T)-1;
    int idx = lane;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      const T ov = __shfl_xor(v, off, 16);
      const int oi = __shfl_xor(idx, off, 16);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = __shfl(idx, 0);
    const T pv = __shfl(v, 0);
    if (lane == 0 && !(pv > (T)0)) atomicOr(status, ST_SINGULAR);
    if (p != k) {
      for (int cc = k + lane; cc < w; cc += 64) {
        const T t = M[k * ld + cc];
        M[k * ld + cc] = M[p * ld + cc];
        M[p * ld + cc] = t;
      }
      __syncthreads();
    }
    const T inv = (T)1 / M[k * ld + k];
    for (int cc = k + 1 + lane; cc < w; cc += 64) M[k * ld + cc] *= inv;
    __syncthreads();
    const int wc = w - k - 1;
    for (int e = lane; e < n * wc; e += 64) {
      const int rr = e / wc, cc = k + 1 + (e - rr * wc);
      if (rr != k) M[rr * ld + cc] = fma_t(-M[rr * ld + k], M[k * ld + cc], M[rr * ld + cc]);
    }
    __syncthreads();
  }
}

// Cholesky G = L L^T of the SPD m x m matrix G (row stride ldg, lower part used)
// followed by the solve G X = RHS for the nr columns of RHS (row stride ldr).
template <typename T>
__device__ void chol64(T *G, int ldg, int m, T *RHS, int ldr, int nr, int *status) {
  const int lane = threadIdx.x;
  for (int j = 0; j < m; ++j) {
    if (lane == 0) {
      T s = G[j * ldg + j];
      for (int k = 0; k < j; ++k) s -= G[j * ldg + k] * G[j * ldg + k];
      if (!(s > (T)0)) atomicOr(status, ST_NOT_PD);
      G[j * ldg + j] = sqrt(s);
    }
    __syncthreads();
    for (int i = j + 1 + lane; i < m; i += 64) {
      T t = G[i * ldg + j];
      for (int k = 0; k < j; ++k) t -= G[i * ldg + k] * G[j * ldg + k];
      G[i * ldg + j] = t / G[j * ldg + j];
    }
    __syncthreads();
  }
  for (int cc = lane; cc < nr; cc += 64) {
    for (int i = 0; i < m; ++i) {
      T t = RHS[i * ldr + cc];
      for (int k = 0; k < i; ++k) t -= G[i * ldg + k] * RHS[k * ldr + cc];
      RHS[i * ldr + cc] = t / G[i * ldg + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      T t = RHS[i * ldr + cc];
      for (int k = i + 1; k < m; ++k) t -= G[k * ldg + i] * RHS[k * ldr + cc];
      RHS[i * ldr + cc] = t / G[i * ldg + i];
    }
  }
  __syncthreads();
}

// out = Pm + sym(O)  (n x n), stored to global
template <typename T>
__device__ __forceinline__ void store_sym_plus(T *__restrict__ out, const T *Pm, const T *O, int n) {
  for (int e = threadIdx.x; e < n * n; e += 64) {
    const int i = e / n, j = e - i * n;
    out[e] = Pm[e] + (T)0.5 * (O[i * n + j] + O[j * n + i]);
  }
}

// tau(alpha, Uj) = Pm + A^T Uj (I + C Uj)^{-1} A  (eq. (terminal-fold)), symmetrised.
// A, C, Pm, Uj already in LDS; scratch M (n x 2n), Y, O in LDS.
template <typename T>
__device__ void tau64(T *__restrict__ out, const T *A, const T *C, const T *Pm, const T *Uj, T *M, T *Y,
                      T *O, int n, int *status) {
  const int n2 = 2 * n;
  mm64<T, false, false, 0>(M, n2, C, n, Uj, n, n, n, n);
  for (int e = threadIdx.x; e < n * n; e += 64) {
    const int i = e / n, j = e - i * n;
    M[i * n2 + n + j] = A[e];
  }
  __syncthreads();
  if (threadIdx.x < n) M[threadIdx.x * n2 + threadIdx.x] += (T)1;
  __syncthreads();
  gj64<T>(M, n2, n, n2, status);
  mm64<T, false, false, 0>(Y, n, Uj, n, M + n, n2, n, n, n);
  __syncthreads();
  mm64<T, true, false, 0>(O, n, A, n, Y, n, n, n, n);
  __syncthreads();
  store_sym_plus(out, Pm, O, n);
}

// ------------------------------------------------------------ factor kernels
// Local control condensation (eq. (edge-components)), one workgroup per node v:
// U_v = Q_v; for v != root the edge slot v gets
//   Abar = A - B R^-1 M^T,  Cbar = Delta_v + B R^-1 B^T,  Pbar = -M R^-1 M^T.
// Always evaluated in float64 (R Cholesky), stored in the working type.
template <typename T>
__global__ __launch_bounds__(64) void k_condense(Bufs<T> bf) {
  extern __shared__ double smd[];
  const int64_t v = blockIdx.x;
  const int n = bf.n, m = bf.m, nn = n * n, nm = n * m, n2 = 2 * n;
  for (int e = threadIdx.x; e < nn; e += 64) bf.U[v * nn + e] = (T)bf.Q[v * nn + e];
  if (v == bf.root) return;
  double *Rs = smd;            // m x m
  double *Rhs = Rs + m * m;    // m x 2n : [B^T | M^T]
  double *Bs = Rhs + m * n2;   // n x m
  double *Ss = Bs + nm;        // n x m
  double *O = Ss + nm;         // n x n
  load64(Rs, bf.R + v * m * m, m * m);
  load64(Bs, bf.B + v * nm, nm);
  load64(Ss, bf.S + v * nm, nm);
  __syncthreads();
  for (int e = threadIdx.x; e < m * n2; e += 64) {
    const int i = e / n2, cc = e - i * n2;
    Rhs[e] = cc < n ? Bs[cc * m + i] : Ss[(cc - n) * m + i];
  }
  __syncthreads();
  chol64<double>(Rs, m, m, Rhs, n2, n2, bf.status);
  mm64<double, false, false, 0>(O, n, Bs, m, Rhs + n, n2, n, m, n);  // B R^-1 M^T
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += 64) bf.EA[v * nn + e] = (T)(bf.A[v * nn + e] - O[e]);
  __syncthreads();
  mm64<double, false, false, 0>(O, n, Bs, m, Rhs, n2, n, m, n);  // B R^-1 B^T
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += 64) {
    const int i = e / n, j = e - i * n;
    bf.EC[v * nn + e] = (T)(bf.De[v * nn + e] + 0.5 * (O[i * n + j] + O[j * n + i]));
  }
  __syncthreads();
  mm64<double, false, false, 0>(O, n, Ss, m, Rhs + n, n2, n, m, n);  // M R^-1 M^T
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += 64) {
    const int i = e / n, j = e - i * n;
    bf.EP[v * nn + e] = (T)(-0.5 * (O[i * n + j] + O[j * n + i]));
  }
}

// One dependency level of the quadratic contraction (Sec. IV-C dataflow).
template <typename T>
__global__ __launch_bounds__(64) void k_quad_level(Bufs<T> bf, const OpRec *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  T *sm = reinterpret_cast<T *>(smd);
  const OpRec o = ops[off + blockIdx.x];
  const int n = bf.n, nn = n * n;
  if (o.kind == OP_RAKE) {
    // m_{i<-j} = tau(alpha_e, U_j); P_j = U_j (expansion of a rake)
    const int64_t j = o.a, e = o.b, out = o.c;
    T *A = sm, *C = A + nn, *Pm = C + nn, *Uj = Pm + nn, *M = Uj + nn, *Y = M + 2 * nn, *O = Y + nn;
    load64(A, bf.EA + e * nn, nn);
    load64(C, bf.EC + e * nn, nn);
    load64(Pm, bf.EP + e * nn, nn);
    load64(Uj, bf.U + j * nn, nn);
    __syncthreads();
    for (int q = threadIdx.x; q < nn; q += 64) bf.PW[j * nn + q] = Uj[q];
    tau64<T>(bf.CT + out * nn, A, C, Pm, Uj, M, Y, O, n, bf.status);
  } else if (o.kind == OP_COMBINE) {
    const int64_t a = o.a, b = o.b, out = o.c;
    for (int q = threadIdx.x; q < nn; q += 64) bf.CT[out * nn + q] = bf.CT[a * nn + q] + bf.CT[b * nn + q];
  } else if (o.kind == OP_ABSORB) {
    const int64_t i = o.a, agg = o.b;
    for (int q = threadIdx.x; q < nn; q += 64) bf.U[i * nn + q] += bf.CT[agg * nn + q];
  } else {
    // alpha_{lr} = alpha_r o_{U_j} alpha_l   (eqs. (compress-intermediates), (composition))
    const int64_t j = o.a, l = o.b, r = o.c, s = o.d;
    const int n3 = 3 * n;
    T *Al = sm, *Cl = Al + nn, *Pl = Cl + nn, *Ar = Pl + nn, *Cr = Ar + nn, *Pt = Cr + nn;
    T *M = Pt + nn, *Z = M + 3 * nn, *O = Z + nn;
    load64(Al, bf.EA + l * nn, nn);
    load64(Cl, bf.EC + l * nn, nn);
    load64(Pl, bf.EP + l * nn, nn);
    load64(Ar, bf.EA + r * nn, nn);
    load64(Cr, bf.EC + r * nn, nn);
    for (int q = threadIdx.x; q < nn; q += 64) Pt[q] = bf.EP[r * nn + q] + bf.U[j * nn + q];
    __syncthreads();
    mm64<T, false, false, 0>(M, n3, Cl, n, Pt, n, n, n, n);          // C_l Pt
    mm64<T, false, true, 0>(M + 2 * n, n3, Cl, n, Ar, n, n, n, n);   // C_l A_r^T
    for (int q = threadIdx.x; q < nn; q += 64) {
      const int i = q / n, jj = q - i * n;
      M[i * n3 + n + jj] = Al[q];
    }
    __syncthreads();
    if (threadIdx.x < n) M[threadIdx.x * n3 + threadIdx.x] += (T)1;
    __syncthreads();
    gj64<T>(M, n3, n, n3, bf.status);                                // [X | Y] = S^-1 [A_l | C_l A_r^T]
    mm64<T, false, false, 0>(bf.EA + s * nn, n, Ar, n, M + n, n3, n, n, n);  // A_r X
    mm64<T, false, false, 0>(O, n, Ar, n, M + 2 * n, n3, n, n, n);   // A_r Y
    mm64<T, false, false, 0>(Z, n, Pt, n, M + n, n3, n, n, n);       // Pt X
    __syncthreads();
    store_sym_plus(bf.EC + s * nn, Cr, O, n);
    __syncthreads();
    mm64<T, true, false, 0>(O, n, Al, n, Z, n, n, n, n);             // A_l^T Pt X
    __syncthreads();
    store_sym_plus(bf.EP + s * nn, Pl, O, n);
  }
}

// One level of the expansion of compressions: P_j = tau((A_r, C_r, P_r + U_j), P_k)
// (eq. (value-reconstruction)).
template <typename T>
__global__ __launch_bounds__(64) void k_quad_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  T *sm = reinterpret_cast<T *>(smd);
  const Op4 o = ops[off + blockIdx.x];
  const int n = bf.n, nn = n * n;
  const int64_t j = o.a, r = o.b, k = o.c;
  T *A = sm, *C = A + nn, *Pm = C + nn, *Pk = Pm + nn, *M = Pk + nn, *Y = M + 2 * nn, *O = Y + nn;
  load64(A, bf.EA + r * nn, nn);
  load64(C, bf.EC + r * nn, nn);
  for (int q = threadIdx.x; q < nn; q += 64) Pm[q] = bf.EP[r * nn + q] + bf.U[j * nn + q];
  load64(Pk, bf.PW + k * nn, nn);
  __syncthreads();
  tau64<T>(bf.PW + j * nn, A, C, Pm, Pk, M, Y, O, n, bf.status);
}

// Local factors (eqs. (FW), (factor-local)), one workgroup per node v:
//   F_v = I + Delta_v P_v, Finv_v, W_v = P_v F_v^-1;
//   for v != root and its edge e = (parent, v):
//   G = R + B^T W_v B (Cholesky), H = B^T W_v A + M^T, K = -G^-1 H,
//   A^cl = A + B K, T_e = F_v^-1 A^cl.
template <typename T>
__global__ __launch_bounds__(64) void k_local_factor(Bufs<T> bf) {
  extern __shared__ double smd[];
  T *sm = reinterpret_cast<T *>(smd);
  const int64_t v = blockIdx.x;
  const int n = bf.n, m = bf.m, nn = n * n, nm = n * m, n2 = 2 * n;
  T *Pv = sm, *Dv = Pv + nn, *M = Dv + nn, *Wl = M + 2 * nn, *Bs = Wl + nn, *As = Bs + nm, *BtW = As + nn;
  T *Gm = BtW + nm, *RH = Gm + m * m, *Kl = RH + m * (n + m), *Al = Kl + nm;
  const bool isroot = (v == bf.root);
  const T *Psrc = isroot ? bf.U + v * nn : bf.PW + v * nn;
  load64(Pv, Psrc, nn);
  load64(Dv, bf.De + v * nn, nn);
  __syncthreads();
  if (isroot)
    for (int q = threadIdx.x; q < nn; q += 64) bf.PW[v * nn + q] = Pv[q];
  mm64<T, false, false, 0>(M, n2, Dv, n, Pv, n, n, n, n);
  for (int q = threadIdx.x; q < nn; q += 64) {
    const int i = q / n, jj = q - i * n;
    M[i * n2 + n + jj] = (i == jj) ? (T)1 : (T)0;
  }
  __syncthreads();
  if (threadIdx.x < n) M[threadIdx.x * n2 + threadIdx.x] += (T)1;
  __syncthreads();
  gj64<T>(M, n2, n, n2, bf.status);  // M[:, n:2n] = F^-1
  mm64<T, false, false, 0>(Wl, n, Pv, n, M + n, n2, n, n, n);
  for (int q = threadIdx.x; q < nn; q += 64) {
    const int i = q / n, jj = q - i * n;
    bf.Finv[v * nn + q] = M[i * n2 + n + jj];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += 64) bf.W[v * nn + q] = Wl[q];
  if (isroot) {
    for (int q = threadIdx.x; q < nm; q += 64) bf.Kw[v * nm + q] = 0;
    return;
  }
  load64(Bs, bf.B + v * nm, nm);
  load64(As, bf.A + v * nn, nn);
  load64(Gm, bf.R + v * m * m, m * m);
  const int ldr = n + m;
  for (int q = threadIdx.x; q < m * ldr; q += 64) {
    const int i = q / ldr, cc = q - i * ldr;
    RH[q] = cc < n ? (T)bf.S[(int64_t)v * nm + cc * m + i] : (T)((cc - n) == i ? 1 : 0);
  }
  __syncthreads();
  mm64<T, true, false, 0>(BtW, n, Bs, m, Wl, n, m, n, n);  // B^T W
  __syncthreads();
  mm64<T, false, false, 1>(Gm, m, BtW, n, Bs, m, m, n, m);   // G = R + B^T W B
  mm64<T, false, false, 1>(RH, ldr, BtW, n, As, n, m, n, n); // H = M^T + B^T W A
  __syncthreads();
  chol64<T>(Gm, m, m, RH, ldr, ldr, bf.status);             // [G^-1 H | G^-1]
  for (int q = threadIdx.x; q < nm; q += 64) {
    const int i = q / n, jj = q - i * n;
    const T kq = -RH[i * ldr + jj];
    Kl[q] = kq;
    bf.Kw[v * nm + q] = kq;
  }
  for (int q = threadIdx.x; q < m * m; q += 64) {
    const int i = q / m, jj = q - i * m;
    bf.Ginv[v * m * m + q] = RH[i * ldr + n + jj];
  }
  __syncthreads();
  mm64<T, false, false, 0>(Al, n, Bs, m, Kl, n, n, m, n);  // B K
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += 64) {
    Al[q] += As[q];
    bf.Acl[v * nn + q] = Al[q];
  }
  __syncthreads();
  mm64<T, false, false, 0>(bf.Tm + v * nn, n, M + n, n2, Al, n, n, n, n);  // T = F^-1 A^cl
}

// Composite transition matrix of a compression: T_new = T_r T_l (eq. (transition-compose)).
template <typename T>
__global__ __launch_bounds__(64) void k_tcompose(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off) {
  extern __shared__ double smd[];
  T *sm = reinterpret_cast<T *>(smd);
  const Op4 o = ops[off + blockIdx.x];
  const int n = bf.n, nn = n * n;
  T *Tl = sm, *Tr = sm + nn;
  load64(Tl, bf.Tm + (int64_t)o.a * nn, nn);
  load64(Tr, bf.Tm + (int64_t)o.b * nn, nn);
  __syncthreads();
  mm64<T, false, false, 0>(bf.Tm + (int64_t)o.c * nn, n, Tr, n, Tl, n, n, n, n);
}

// ------------------------------------------------------------ solve kernels (16-lane teams)
#define TEAM 16
#define TEAMS_PER_BLOCK 16

// h_i = q_i; z_e = K_e^T r_e + (A^cl_e)^T W_j c_j  (eq. (affine-edge)), e = (parent, j), slot j.
template <typename T>
__global__ __launch_bounds__(256) void k_rhs_init(Bufs<T> bf) {
  const int64_t v = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m, nn = n * n;
  if (r < n) bf.h[v * n + r] = bf.sq[v * n + r];
  if (v == bf.root) {
    if (r < n) bf.z[v * n + r] = 0;
    return;
  }
  T wc = 0;
  if (r < n)
    for (int k = 0; k < n; ++k) wc = fma_t(bf.W[v * nn + r * n + k], bf.sc[v * n + k], wc);
  T s = 0;
  for (int k = 0; k < n; ++k) {
    const T wk = __shfl(wc, k, TEAM);
    if (r < n) s = fma_t(bf.Acl[v * nn + k * n + r], wk, s);
  }
  if (r < n) {
    for (int k = 0; k < bf.m; ++k) s = fma_t(bf.Kw[v * n * m + k * n + r], bf.sr[v * m + k], s);
    bf.z[v * n + r] = s;
  }
}

// One level of the affine contraction: rake m = Z h_j + z with Z = T^T (eq. (affine-rake)),
// p_j = h_j; combine; absorb; compress z_new = z_l + Z_l (h_j + z_r) (eq. (affine-compose)).
template <typename T>
__global__ __launch_bounds__(256) void k_aff_level(Bufs<T> bf, const OpRec *__restrict__ ops, int64_t off,
                                                   int64_t cnt) {
  const int64_t qq = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (qq >= cnt) return;
  const OpRec o = ops[off + qq];
  const int n = bf.n, nn = n * n;
  if (r >= n) return;
  if (o.kind == OP_RAKE) {
    const int64_t j = o.a, e = o.b, out = o.c;
    T s = bf.z[e * n + r];
    for (int k = 0; k < n; ++k) s = fma_t(bf.Tm[e * nn + k * n + r], bf.h[j * n + k], s);
    bf.cv[out * n + r] = s;
    bf.p[j * n + r] = bf.h[j * n + r];
  } else if (o.kind == OP_COMBINE) {
    bf.cv[(int64_t)o.c * n + r] = bf.cv[(int64_t)o.a * n + r] + bf.cv[(int64_t)o.b * n + r];
  } else if (o.kind == OP_ABSORB) {
    bf.h[(int64_t)o.a * n + r] += bf.cv[(int64_t)o.b * n + r];
  } else {
    const int64_t j = o.a, l = o.b, rr = o.c, s = o.d;
    T acc = bf.z[l * n + r];
    for (int k = 0; k < n; ++k)
      acc = fma_t(bf.Tm[l * nn + k * n + r], bf.h[j * n + k] + bf.z[rr * n + k], acc);
    bf.z[s * n + r] = acc;
  }
}

// Affine expansion of compressions: p_j = Z_r p_k + h_j + z_r.
template <typename T>
__global__ __launch_bounds__(256) void k_aff_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                    int64_t cnt) {
  const int64_t qq = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (qq >= cnt) return;
  const Op4 o = ops[off + qq];
  const int n = bf.n, nn = n * n;
  if (r >= n) return;
  const int64_t j = o.a, rs = o.b, k = o.c;
  T s = bf.h[j * n + r] + bf.z[rs * n + r];
  for (int q = 0; q < n; ++q) s = fma_t(bf.Tm[rs * nn + q * n + r], bf.p[k * n + q], s);
  bf.p[j * n + r] = s;
}

// Local affine solve (eq. (local-affine-solve)) and root state (eq. (xroot)):
//   f = Delta p - c, g = p - W f; for e = (parent, v): k = -G^-1 (r + B^T g),
//   b = F_v^-1 (B k - f); at the root x = -F^-1 f.
template <typename T>
__global__ __launch_bounds__(256) void k_local_affine(Bufs<T> bf) {
  const int64_t v = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m, nn = n * n, nm = n * m;
  const bool isroot = (v == bf.root);
  const T *pv = isroot ? bf.h + v * n : bf.p + v * n;
  T f = 0;
  if (r < n) {
    f = -bf.sc[v * n + r];
    for (int k = 0; k < n; ++k) f = fma_t((T)bf.De[v * nn + r * n + k], pv[k], f);
  }
  if (isroot && r < n) bf.p[v * n + r] = pv[r];
  if (isroot) {
    T x = 0;
    for (int k = 0; k < n; ++k) {
      const T fk = __shfl(f, k, TEAM);
      if (r < n) x = fma_t(-bf.Finv[v * nn + r * n + k], fk, x);
    }
    if (r < n) bf.xw[v * n + r] = x;
    return;
  }
  T g = 0;
  if (r < n) g = pv[r];
  for (int k = 0; k < n; ++k) {
    const T fk = __shfl(f, k, TEAM);
    if (r < n) g = fma_t(-bf.W[v * nn + r * n + k], fk, g);
  }
  T t = 0;  // lane c < m: r_c + (B^T g)_c
  if (r < m) t = bf.sr[v * m + r];
  for (int k = 0; k < n; ++k) {
    const T gk = __shfl(g, k, TEAM);
    if (r < m) t = fma_t((T)bf.B[v * nm + k * m + r], gk, t);
  }
  T kk = 0;
  for (int d = 0; d < m; ++d) {
    const T td = __shfl(t, d, TEAM);
    if (r < m) kk = fma_t(-bf.Ginv[v * m * m + r * m + d], td, kk);
  }
  if (r < m) bf.kff[v * m + r] = kk;
  T wv = -f;  // lane r < n: (B k - f)_r
  for (int d = 0; d < m; ++d) {
    const T kd = __shfl(kk, d, TEAM);
    if (r < n) wv = fma_t((T)bf.B[v * nm + r * m + d], kd, wv);
  }
  T bb = 0;
  for (int k = 0; k < n; ++k) {
    const T wk = __shfl(wv, k, TEAM);
    if (r < n) bb = fma_t(bf.Finv[v * nn + r * n + k], wk, bb);
  }
  if (r < n) bf.b[v * n + r] = bb;
}

// State-offset composition along compressions: b_new = T_r b_l + b_r.
template <typename T>
__global__ __launch_bounds__(256) void k_state_level(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                     int64_t cnt) {
  const int64_t qq = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (qq >= cnt) return;
  const Op4 o = ops[off + qq];
  const int n = bf.n, nn = n * n;
  if (r >= n) return;
  const int64_t l = o.a, rs = o.b, s = o.c;
  T acc = bf.b[rs * n + r];
  for (int k = 0; k < n; ++k) acc = fma_t(bf.Tm[rs * nn + r * n + k], bf.b[l * n + k], acc);
  bf.b[s * n + r] = acc;
}

// State expansion: x_j = T_s x_i + b_s (edge slot s into j and parent i at removal).
template <typename T>
__global__ __launch_bounds__(256) void k_state_expand(Bufs<T> bf, const Op4 *__restrict__ ops, int64_t off,
                                                      int64_t cnt) {
  const int64_t qq = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (qq >= cnt) return;
  const Op4 o = ops[off + qq];
  const int n = bf.n, nn = n * n;
  if (r >= n) return;
  const int64_t j = o.a, s = o.b, i = o.c;
  T acc = bf.b[s * n + r];
  for (int k = 0; k < n; ++k) acc = fma_t(bf.Tm[s * nn + r * n + k], bf.xw[i * n + k], acc);
  bf.xw[j * n + r] = acc;
}

// Recovery (eq. (recover)): y_v = P_v x_v + p_v; u_e = K_e x_parent + k_e; flags non-finite values.
template <typename T>
__global__ __launch_bounds__(256) void k_recover(Bufs<T> bf) {
  const int64_t v = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (v >= bf.N) return;
  const int n = bf.n, m = bf.m, nn = n * n, nm = n * m;
  bool bad = false;
  if (r < n) {
    T y = bf.p[v * n + r];
    for (int k = 0; k < n; ++k) y = fma_t(bf.PW[v * nn + r * n + k], bf.xw[v * n + k], y);
    bf.yw[v * n + r] = y;
    bad = !isfinite((double)y) || !isfinite((double)bf.xw[v * n + r]);
  }
  if (r < m) {
    T u = 0;
    if (v != bf.root) {
      const int64_t i = bf.parent[v];
      u = bf.kff[v * m + r];
      for (int k = 0; k < n; ++k) u = fma_t(bf.Kw[v * nm + r * n + k], bf.xw[i * n + k], u);
    }
    bf.uw[v * m + r] = u;
    bad = bad || !isfinite((double)u);
  }
  if (bad) atomicOr(bf.status, ST_NONFINITE);
}

__global__ void k_zero_status(int *st, double *resid) {
  if (threadIdx.x < 4) st[threadIdx.x] = 0;
  if (threadIdx.x == 0) resid[0] = 0.0;
}

// Max-abs residual of the four KKT blocks of eq. (kkt), in float64, one 16-lane team per node v:
//   node   Q x + q - y + sum_children (M u + A^T y_child)
//   edge   M^T x_i + R u + r + B^T y_v;  A x_i + B u + c - x_v - Delta_v y_v   (v != root)
//   root   c - x - Delta y
__global__ __launch_bounds__(256) void k_kkt_residual(int64_t N, int n, int m, int root, const double *Q,
                                                      const double *q, const double *c, const double *De,
                                                      const double *R, const double *S, const double *rr,
                                                      const double *A, const double *B, const double *x,
                                                      const double *u, const double *y,
                                                      const int32_t *parent, const int32_t *coff,
                                                      const int32_t *cidx, double *out) {
  const int64_t v = (int64_t)blockIdx.x * TEAMS_PER_BLOCK + threadIdx.x / TEAM;
  const int r = threadIdx.x & (TEAM - 1);
  if (v >= N) return;
  const int nn = n * n, nm = n * m;
  double worst = 0.0;
  if (r < n) {
    double s = q[v * n + r] - y[v * n + r];
    for (int k = 0; k < n; ++k) s += Q[v * nn + r * n + k] * x[v * n + k];
    for (int32_t t = coff[v]; t < coff[v + 1]; ++t) {
      const int64_t j = cidx[t];
      for (int k = 0; k < m; ++k) s += S[j * nm + r * m + k] * u[j * m + k];
      for (int k = 0; k < n; ++k) s += A[j * nn + k * n + r] * y[j * n + k];
    }
    worst = fabs(s);
    if (v == root) {
      double t = c[v * n + r] - x[v * n + r];
      for (int k = 0; k < n; ++k) t -= De[v * nn + r * n + k] * y[v * n + k];
      worst = fmax(worst, fabs(t));
    } else {
      const int64_t i = parent[v];
      double t = c[v * n + r] - x[v * n + r];
      for (int k = 0; k < n; ++k) t += A[v * nn + r * n + k] * x[i * n + k] - De[v * nn + r * n + k] * y[v * n + k];
      for (int k = 0; k < m; ++k) t += B[v * nm + r * m + k] * u[v * m + k];
      worst = fmax(worst, fabs(t));
    }
  }
  if (r < m && v != root) {
    const int64_t i = parent[v];
    double t = rr[v * m + r];
    for (int k = 0; k < n; ++k) t += S[v * nm + k * m + r] * x[i * n + k] + B[v * nm + k * m + r] * y[v * n + k];
    for (int k = 0; k < m; ++k) t += R[v * m * m + r * m + k] * u[v * m + k];
    worst = fmax(worst, fabs(t));
  }
  if (!(worst == worst)) worst = INFINITY;
  for (int off = 8; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off, TEAM));
  if (r == 0 && worst > 0.0)
    atomicMax(reinterpret_cast<unsigned long long *>(out), (unsigned long long)__double_as_longlong(worst));
}

// ------------------------------------------------------------ host side
static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

WsLayout workspace_layout(const PlanHost &ph, int precision) {
  const size_t N = (size_t)ph.N, n = (size_t)ph.n, m = (size_t)ph.m, nn = n * n;
  const size_t S = (size_t)ph.n_edge_slots, NC = (size_t)std::max<int64_t>(ph.n_contrib, 1);
  const size_t es = precision == RCR_FP64 ? 8 : 4;
  WsLayout L;
  size_t cur = 0;
  auto take = [&](size_t elems) {
    size_t at = cur;
    cur = align_up(cur + elems * es, 256);
    return at / es;
  };
  L.U = take(N * nn);
  L.EA = take(S * nn);
  L.EC = take(S * nn);
  L.EP = take(S * nn);
  L.CT = take(NC * nn);
  L.Finv = take(N * nn);
  L.W = take(N * nn);
  L.Ginv = take(N * m * m);
  L.Acl = take(N * nn);
  L.Tm = take(S * nn);
  L.h = take(N * n);
  L.cv = take(NC * n);
  L.z = take(S * n);
  L.p = take(N * n);
  L.kff = take(N * m);
  L.b = take(S * n);
  if (precision == RCR_FP64) {
    L.PW = L.Kw = L.xw = L.uw = L.yw = (size_t)-1;  // the caller's outputs are used in place
    L.rq = L.rr = L.rc = L.d_x = L.d_u = L.d_y = (size_t)-1;
  } else {
    L.PW = take(N * nn);
    L.Kw = take(N * m * n);
    L.xw = take(N * n);
    L.uw = take(N * m);
    L.yw = take(N * n);
    L.rq = take(N * n);
    L.rr = take(N * m);
    L.rc = take(N * n);
    size_t at = align_up(cur, 256);
    L.d_x = at / 8;
    cur = align_up(at + N * n * 8, 256);
    L.d_u = cur / 8;
    cur = align_up(cur + N * m * 8, 256);
    L.d_y = cur / 8;
    cur = align_up(cur + N * n * 8, 256);
  }
  L.total_bytes = cur;
  return L;
}

#define HIPCK(x)                        \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) {             \
      fprintf(stderr, "rcr: %s failed: %s (%s:%d)\n", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      return RCR_HIP_ERROR;             \
    }                                   \
  } while (0)

int plan_upload(PlanObj &P) {
  if (P.dev.ops) return RCR_OK;
  const PlanHost &h = P.host;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  P.dev.device = dev;
  auto up = [&](void **dst, const void *src, size_t bytes) -> int {
    size_t b = std::max<size_t>(bytes, 16);
    if (hipMalloc(dst, b) != hipSuccess) return RCR_OOM;
    P.dev.bytes += b;
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return RCR_HIP_ERROR;
    return RCR_OK;
  };
  int rc;
  if ((rc = up((void **)&P.dev.ops, h.ops.data(), h.ops.size() * sizeof(OpRec)))) return rc;
  if ((rc = up((void **)&P.dev.exp_ops, h.exp_ops.data(), h.exp_ops.size() * sizeof(Op4)))) return rc;
  if ((rc = up((void **)&P.dev.tc_ops, h.tc_ops.data(), h.tc_ops.size() * sizeof(Op4)))) return rc;
  if ((rc = up((void **)&P.dev.sx_ops, h.sx_ops.data(), h.sx_ops.size() * sizeof(Op4)))) return rc;
  if ((rc = up((void **)&P.dev.parent, h.parent32.data(), h.parent32.size() * sizeof(int32_t)))) return rc;
  std::vector<int32_t> coff(h.N + 1, 0), cidx(std::max<int64_t>(h.N, 1), 0);
  for (int64_t j = 0; j < h.N; ++j)
    if (h.parent32[j] >= 0) coff[h.parent32[j] + 1]++;
  for (int64_t i = 0; i < h.N; ++i) coff[i + 1] += coff[i];
  {
    std::vector<int32_t> fill(coff.begin(), coff.end() - 1);
    for (int64_t j = 0; j < h.N; ++j)
      if (h.parent32[j] >= 0) cidx[fill[h.parent32[j]]++] = (int32_t)j;
  }
  if ((rc = up((void **)&P.dev.child_off, coff.data(), coff.size() * sizeof(int32_t)))) return rc;
  if ((rc = up((void **)&P.dev.child_idx, cidx.data(), cidx.size() * sizeof(int32_t)))) return rc;
  if (hipMalloc((void **)&P.status, 256) != hipSuccess) return RCR_OOM;
  if (hipMalloc((void **)&P.resid, 256) != hipSuccess) return RCR_OOM;
  HIPCK(hipMemset(P.status, 0, 256));
  HIPCK(hipMemset(P.resid, 0, 256));
  return RCR_OK;
}

void plan_release_device(PlanObj &P) {
  for (auto &kv : P.graphs) (void)hipGraphExecDestroy(kv.second);
  P.graphs.clear();
  for (hipEvent_t e : P.events) (void)hipEventDestroy(e);
  P.events.clear();
  void *ptrs[] = {P.dev.ops, P.dev.exp_ops, P.dev.tc_ops, P.dev.sx_ops, P.dev.parent, P.dev.child_off,
                  P.dev.child_idx, P.status, P.resid, P.ws[0], P.ws[1]};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  P.dev = PlanDev();
  P.status = nullptr;
  P.resid = nullptr;
  P.ws[0] = P.ws[1] = nullptr;
  P.ws_bytes[0] = P.ws_bytes[1] = 0;
}

static inline unsigned blocks_for(int64_t cnt, int per) { return (unsigned)((cnt + per - 1) / per); }

// Per-kernel-class HIP event bracketing (optional).
struct Timer {
  PlanObj *P = nullptr;
  hipStream_t st = nullptr;
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> spans;
  size_t used = 0;
  hipEvent_t ev() {
    if (used == P->events.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      P->events.push_back(e);
    }
    return P->events[used++];
  }
  void begin(int cls) {
    if (!on) return;
    hipEvent_t a = ev(), b = ev();
    if (!a || !b) return;
    (void)hipEventRecord(a, st);
    spans.push_back({cls, {a, b}});
  }
  void end() {
    if (!on || spans.empty()) return;
    (void)hipEventRecord(spans.back().second.second, st);
  }
};

template <typename T>
static size_t lds_matrix_bytes(int n, int m) {
  const size_t nn = (size_t)n * n, nm = (size_t)n * m;
  size_t quad = std::max<size_t>(8 * nn, 11 * nn) * sizeof(T);
  size_t cond = ((size_t)m * m + (size_t)m * 2 * n + 2 * nm + nn) * sizeof(double);
  size_t lf = (2 * nn + 2 * nn + nn + nm + nn + nm + (size_t)m * m + (size_t)m * (n + m) + nm + nn) * sizeof(T);
  return std::max(quad, std::max(cond, lf));
}

// Launch the whole factor + solve for working type T on `st`.
template <typename T>
static int launch_all(PlanObj &P, Bufs<T> bf, Timer &tm, hipStream_t st) {
  const PlanHost &h = P.host;
  const int n = h.n, m = h.m;
  const size_t lds = lds_matrix_bytes<T>(n, m);
  const unsigned NB = (unsigned)h.N;
  tm.begin(RCR_K_CONDENSE);
  hipLaunchKernelGGL(k_condense<T>, dim3(NB), dim3(64), lds, st, bf);
  tm.end();
  tm.begin(RCR_K_QUAD_CONTRACT);
  for (int64_t t = 0; t < h.levels(); ++t) {
    const int64_t cnt = h.lvl_off[t + 1] - h.lvl_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_quad_level<T>, dim3((unsigned)cnt), dim3(64), lds, st, bf, P.dev.ops, h.lvl_off[t]);
  }
  tm.end();
  tm.begin(RCR_K_QUAD_EXPAND);
  for (int64_t t = 0; t < h.expand_levels(); ++t) {
    const int64_t cnt = h.exp_off[t + 1] - h.exp_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_quad_expand<T>, dim3((unsigned)cnt), dim3(64), lds, st, bf, P.dev.exp_ops, h.exp_off[t]);
  }
  tm.end();
  tm.begin(RCR_K_LOCAL_FACTOR);
  hipLaunchKernelGGL(k_local_factor<T>, dim3(NB), dim3(64), lds, st, bf);
  tm.end();
  tm.begin(RCR_K_TCOMPOSE);
  for (int64_t t = 0; t < h.state_levels(); ++t) {
    const int64_t cnt = h.tc_off[t + 1] - h.tc_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_tcompose<T>, dim3((unsigned)cnt), dim3(64), 2 * n * n * sizeof(T), st, bf, P.dev.tc_ops, h.tc_off[t]);
  }
  tm.end();
  const unsigned VB = blocks_for(h.N, TEAMS_PER_BLOCK);
  tm.begin(RCR_K_RHS_INIT);
  hipLaunchKernelGGL(k_rhs_init<T>, dim3(VB), dim3(256), 0, st, bf);
  tm.end();
  tm.begin(RCR_K_AFF_CONTRACT);
  for (int64_t t = 0; t < h.levels(); ++t) {
    const int64_t cnt = h.lvl_off[t + 1] - h.lvl_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_aff_level<T>, dim3(blocks_for(cnt, TEAMS_PER_BLOCK)), dim3(256), 0, st, bf, P.dev.ops, h.lvl_off[t], cnt);
  }
  tm.end();
  tm.begin(RCR_K_AFF_EXPAND);
  for (int64_t t = 0; t < h.expand_levels(); ++t) {
    const int64_t cnt = h.exp_off[t + 1] - h.exp_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_aff_expand<T>, dim3(blocks_for(cnt, TEAMS_PER_BLOCK)), dim3(256), 0, st, bf, P.dev.exp_ops, h.exp_off[t], cnt);
  }
  tm.end();
  tm.begin(RCR_K_LOCAL_AFFINE);
  hipLaunchKernelGGL(k_local_affine<T>, dim3(VB), dim3(256), 0, st, bf);
  tm.end();
  tm.begin(RCR_K_STATE_CONTRACT);
  for (int64_t t = 0; t < h.state_levels(); ++t) {
    const int64_t cnt = h.tc_off[t + 1] - h.tc_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_state_level<T>, dim3(blocks_for(cnt, TEAMS_PER_BLOCK)), dim3(256), 0, st, bf, P.dev.tc_ops, h.tc_off[t], cnt);
  }
  tm.end();
  tm.begin(RCR_K_STATE_EXPAND);
  for (int64_t t = 0; t < h.sexp_levels(); ++t) {
    const int64_t cnt = h.sx_off[t + 1] - h.sx_off[t];
    if (cnt > 0) hipLaunchKernelGGL(k_state_expand<T>, dim3(blocks_for(cnt, TEAMS_PER_BLOCK)), dim3(256), 0, st, bf, P.dev.sx_ops, h.sx_off[t], cnt);
  }
  tm.end();
  tm.begin(RCR_K_RECOVER);
  hipLaunchKernelGGL(k_recover<T>, dim3(VB), dim3(256), 0, st, bf);
  tm.end();
  HIPCK(hipGetLastError());
  return RCR_OK;
}

static int launch_residual(PlanObj &P, const rcr_problem &in, const double *x, const double *u,
                           const double *y, hipStream_t st) {
  const PlanHost &h = P.host;
  hipLaunchKernelGGL(k_kkt_residual, dim3(blocks_for(h.N, TEAMS_PER_BLOCK)), dim3(256), 0, st, h.N, h.n, h.m,
                     (int)h.root, in.Q, in.q, in.c, in.Delta, in.R, in.S, in.r, in.A, in.B, x, u, y,
                     P.dev.parent, P.dev.child_off, P.dev.child_idx, P.resid);
  HIPCK(hipGetLastError());
  return RCR_OK;
}

template <typename T>
static Bufs<T> make_bufs(PlanObj &P, const WsLayout &L, void *ws, const rcr_problem &in, rcr_solution &out) {
  const PlanHost &h = P.host;
  T *base = reinterpret_cast<T *>(ws);
  Bufs<T> bf;
  bf.n = h.n;
  bf.m = h.m;
  bf.root = (int)h.root;
  bf.N = h.N;
  bf.Q = in.Q; bf.q = in.q; bf.c = in.c; bf.De = in.Delta;
  bf.R = in.R; bf.S = in.S; bf.r = in.r; bf.A = in.A; bf.B = in.B;
  bf.U = base + L.U; bf.EA = base + L.EA; bf.EC = base + L.EC; bf.EP = base + L.EP; bf.CT = base + L.CT;
  bf.Finv = base + L.Finv; bf.W = base + L.W; bf.Ginv = base + L.Ginv; bf.Acl = base + L.Acl; bf.Tm = base + L.Tm;
  bf.h = base + L.h; bf.cv = base + L.cv; bf.z = base + L.z; bf.p = base + L.p; bf.kff = base + L.kff; bf.b = base + L.b;
  bf.parent = P.dev.parent;
  bf.status = P.status;
  return bf;
}

int solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt, hipStream_t st) {
  std::lock_guard<std::mutex> lock(P.mu);
  int rc = plan_upload(P);
  if (rc) return rc;
  const int prec = opt.precision;
  if (prec != RCR_FP64) return RCR_BAD_OPTION;  // MIXED32 is dispatched by solve_mixed
  const WsLayout L = workspace_layout(P.host, prec);
  void *ws = opt.workspace;
  if (ws) {
    if ((size_t)opt.workspace_bytes < L.total_bytes) return RCR_SMALL_WORKSPACE;
  } else {
    if (P.ws_bytes[prec] < L.total_bytes) {
      if (P.ws[prec]) (void)hipFree(P.ws[prec]);
      P.ws[prec] = nullptr;
      P.ws_bytes[prec] = 0;
      if (hipMalloc(&P.ws[prec], L.total_bytes) != hipSuccess) return RCR_OOM;
      P.ws_bytes[prec] = L.total_bytes;
    }
    ws = P.ws[prec];
  }
  Bufs<double> bf = make_bufs<double>(P, L, ws, in, out);
  bf.sq = in.q;
  bf.sr = in.r;
  bf.sc = in.c;
  bf.PW = out.P;
  bf.Kw = out.K;
  bf.xw = out.x;
  bf.uw = out.u;
  bf.yw = out.lam;

  Timer tm;
  tm.P = &P;
  tm.st = st;
  tm.on = opt.kernel_ms != nullptr;
  const bool use_graph = (opt.executor == RCR_EXEC_GRAPH) && !tm.on;
  if (use_graph) {
    GraphKey key;
    memset(&key, 0, sizeof(key));
    const void *ptrs[16] = {in.Q, in.q, in.c, in.Delta, in.R, in.S, in.r, in.A, in.B,
                            out.K, out.P, out.x, out.u, out.lam, ws, (const void *)(intptr_t)prec};
    memcpy(key.p, ptrs, sizeof(ptrs));
    auto it = P.graphs.find(key);
    if (it == P.graphs.end()) {
      hipStream_t cs;
      HIPCK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g;
      HIPCK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, cs, P.status, P.resid);
      Timer off;
      int lrc = launch_all<double>(P, bf, off, cs);
      hipError_t ce = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (lrc) return lrc;
      HIPCK(ce);
      hipGraphExec_t ge;
      hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCK(ie);
      it = P.graphs.emplace(key, ge).first;
    }
    HIPCK(hipGraphLaunch(it->second, st));
  } else {
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, P.status, P.resid);
    rc = launch_all<double>(P, bf, tm, st);
    if (rc) return rc;
  }
  if (opt.kkt_residual) {
    rc = launch_residual(P, in, out.x, out.u, out.lam, st);
    if (rc) return rc;
  }
  if (opt.check || opt.kkt_residual || tm.on) {
    HIPCK(hipStreamSynchronize(st));
    if (tm.on) {
      for (int c = 0; c < RCR_NUM_KERNEL_CLASSES; ++c) opt.kernel_ms[c] = 0.f;
      for (auto &sp : tm.spans) {
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, sp.second.first, sp.second.second));
        opt.kernel_ms[sp.first] += ms;
      }
    }
    if (opt.kkt_residual) HIPCK(hipMemcpy(opt.kkt_residual, P.resid, sizeof(double), hipMemcpyDeviceToHost));
    if (opt.check) {
      int stw = 0;
      HIPCK(hipMemcpy(&stw, P.status, sizeof(int), hipMemcpyDeviceToHost));
      if (stw & ST_NOT_PD) return RCR_NOT_PD;
      if (stw & ST_SINGULAR) return RCR_SINGULAR;
      if (stw & ST_NONFINITE) return RCR_NONFINITE;
    }
  }
  return RCR_OK;
}

}  // namespace rcr
