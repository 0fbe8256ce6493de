// Block products on the float64 matrix cores for the wide layout (NB in
// {12, 16}), with v_mfma_f64_16x16x4_f64: a 16 x 16 x 16 product is NB / 4
// instructions whose operands each lane fetches as one element per
// instruction, instead of a row and a column quarter per product from LDS.
// Blocks of dimension NB < 16 are zero-padded to 16 by masking.
//
// Lane layout of the instruction (lane l, k-block kb):
//   A operand  A[l % 16][4 kb + l / 16]
//   B operand  B[4 kb + l / 16][l % 16]
//   result     D[l / 16 + 4 v][l % 16],  v = 0..3
// so a lane owns column l % 16 and rows l / 16, l / 16 + 4, ... of a product.
// Products accumulate in float64 for both working types.
#pragma once

#include "wide.hpp"

namespace rcr {

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int mf_col() { return (int)(threadIdx.x & 15); }
__device__ __forceinline__ int mf_row(int v) { return (int)((threadIdx.x & 63) >> 4) + 4 * v; }

__device__ __forceinline__ dv4 mf_zero() {
  dv4 z = {0.0, 0.0, 0.0, 0.0};
  return z;
}

// Identity of order nb in the result layout.
__device__ __forceinline__ dv4 mf_ident(int nb) {
  dv4 d;
  const int c = mf_col();
#pragma unroll
  for (int v = 0; v < 4; ++v) d[v] = (mf_row(v) == c && c < nb) ? 1.0 : 0.0;
  return d;
}

// Load / store a block in the result layout: element (row, col) at
// p[row * ld + col] for row < nr, col < nc (zero elsewhere on load).
template <typename S>
__device__ __forceinline__ dv4 mf_load(const S *__restrict__ p, int ld, int nr, int nc) {
  dv4 d;
  const int c = mf_col();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = mf_row(v);
    d[v] = (r < nr && c < nc) ? (double)p[r * ld + c] : 0.0;
  }
  return d;
}

template <typename D>
__device__ __forceinline__ void mf_store(D *__restrict__ p, int ld, const dv4 &x, int nr, int nc) {
  const int c = mf_col();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = mf_row(v);
    if (r < nr && c < nc) p[r * ld + c] = (D)x[v];
  }
}

// 1 / sqrt(s) for s > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - s y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// x rounded to the working type T and back, per component (what storing x as T
// and loading it again gives).
template <typename T>
__device__ __forceinline__ dv4 mf_round(const dv4 &x) {
  dv4 d;
#pragma unroll
  for (int v = 0; v < 4; ++v) d[v] = (double)(T)x[v];
  return d;
}

// acc + op(A) op(B) for NB x NB blocks (TA / TB: use the transpose), rows and
// columns at or beyond NB read as zero.
template <int NB, bool TA, bool TB, typename SA, typename SB>
__device__ __forceinline__ dv4 mf_mm(dv4 acc, const SA *A, int lda, const SB *B, int ldb) {
  const int l = (int)(threadIdx.x & 63), i = l & 15, kk = l >> 4;
#pragma unroll
  for (int kb = 0; kb < NB / 4; ++kb) {
    const int k = 4 * kb + kk;
    const double a = (i < NB) ? (double)(TA ? A[k * lda + i] : A[i * lda + k]) : 0.0;
    const double b = (i < NB) ? (double)(TB ? B[i * ldb + k] : B[k * ldb + i]) : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// 0.5 (X + X^T) in the result layout, X an NB x NB block in LDS (stride ld)
// that the caller has synchronised.
template <typename T>
__device__ __forceinline__ dv4 mf_sym(const T *X, int ld, int nb) {
  dv4 d;
  const int c = mf_col();
  const int cc = c < nb ? c : nb - 1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = mf_row(v), rr = r < nb ? r : nb - 1;
    d[v] = 0.5 * ((double)X[rr * ld + cc] + (double)X[cc * ld + rr]);
  }
  return d;
}

}  // namespace rcr
