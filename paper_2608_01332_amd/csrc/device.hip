// HIP kernels (gfx950) and the launch sequence of one factor + solve.
//
// Mapping.  Every primitive runs on a team of TW lanes (team.hpp): lane r
// owns row r of each n x n block (padded to NB in {4, 6, 8, 12, 16}) in
// registers, blocks read by other lanes are broadcast from the team's LDS,
// nonsymmetric solves (I + C U, S = I + C_l Pt, F = I + Delta P) use
// Gauss-Jordan elimination with partial pivoting and the SPD solves (R_e, G_e)
// use float64 Cholesky.  Node and edge data are structure-of-arrays with one
// contiguous block per node or edge slot.
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
#include "kernels.hpp"
#include "launch_impl.hpp"

namespace rcr {

#define TEAM 16
#define TEAMS_PER_BLOCK 16

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
  if ((rc = up((void **)&P.dev.koff, h.kind_off.data(), h.kind_off.size() * sizeof(int64_t)))) return rc;
  if ((rc = up((void **)&P.dev.exp_off, h.exp_off.data(), h.exp_off.size() * sizeof(int64_t)))) return rc;
  if ((rc = up((void **)&P.dev.tc_off, h.tc_off.data(), h.tc_off.size() * sizeof(int64_t)))) return rc;
  if ((rc = up((void **)&P.dev.sx_off, h.sx_off.data(), h.sx_off.size() * sizeof(int64_t)))) return rc;
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
  void *ptrs[] = {P.dev.ops,    P.dev.exp_ops, P.dev.tc_ops, P.dev.sx_ops, P.dev.parent, P.dev.child_off,
                  P.dev.child_idx, P.dev.koff,  P.dev.exp_off, P.dev.tc_off, P.dev.sx_off, P.status,
                  P.resid,        P.ws[0],       P.ws[1]};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  P.dev = PlanDev();
  P.status = nullptr;
  P.resid = nullptr;
  P.ws[0] = P.ws[1] = nullptr;
  P.ws_bytes[0] = P.ws_bytes[1] = 0;
}

#define RCR_DECL_NB(NBV)                                                                        \
  extern template int launch_all_m<double, NBV>(PlanObj &, Bufs<double>, Timer &, hipStream_t);
RCR_DECL_NB(4)
RCR_DECL_NB(6)
RCR_DECL_NB(8)
RCR_DECL_NB(12)
RCR_DECL_NB(16)
template <typename T>
static int launch_all(PlanObj &P, Bufs<T> bf, Timer &tm, hipStream_t st) {
  switch (pad_n(bf.n)) {
    case 4: return launch_all_m<T, 4>(P, bf, tm, st);
    case 6: return launch_all_m<T, 6>(P, bf, tm, st);
    case 8: return launch_all_m<T, 8>(P, bf, tm, st);
    case 12: return launch_all_m<T, 12>(P, bf, tm, st);
    default: return launch_all_m<T, 16>(P, bf, tm, st);
  }
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
      for (int c = 0; c < RCR_NUM_KERNEL_CLASSES; ++c) {
        opt.kernel_ms[c] = 0.f;
        if (opt.kernel_launches) opt.kernel_launches[c] = 0;
      }
      for (auto &sp : tm.spans) {
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, sp.second.first, sp.second.second));
        opt.kernel_ms[sp.first] += ms;
        if (opt.kernel_launches) opt.kernel_launches[sp.first] += 1;
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
