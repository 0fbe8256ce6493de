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
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "device.hpp"
#include "kernels.hpp"
#include "launch_impl.hpp"

namespace rcr {


__global__ void k_zero_status(int *st, double *resid) {
  if (threadIdx.x < 4) st[threadIdx.x] = 0;
  if (threadIdx.x == 0) resid[0] = 0.0;
}

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

WsLayout workspace_layout(const PlanHost &ph, int precision) {
  const size_t N = (size_t)ph.N, n = (size_t)ph.n, m = (size_t)ph.m, nn = n * n;
  const size_t S = (size_t)ph.n_edge_slots, NC = (size_t)std::max<int64_t>(ph.n_contrib, 1);
  const size_t es = precision == RCR_FP64 ? 8 : 4;
  WsLayout L;
  size_t cur = WS_HEADER_BYTES;  // per-solve status words and residual accumulator
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
    L.rq = L.rr = L.rc = (size_t)-1;
  } else {
    L.PW = take(N * nn);
    L.Kw = take(N * m * n);
    L.xw = take(N * n);
    L.uw = take(N * m);
    L.yw = take(N * n);
    L.rq = take(N * n);
    L.rr = take(N * m);
    L.rc = take(N * n);
  }
  L.total_bytes = cur;
  return L;
}

// Float64 word counts of the lifted problem and solution per lifted node (d = n + m).
static void lift_words(int d, int m, size_t in_w[9], size_t out_w[5]) {
  const size_t dd = (size_t)d * d, dm = (size_t)d * m, mm = (size_t)m * m;
  const size_t iw[9] = {dd, (size_t)d, (size_t)d, dd, mm, dm, (size_t)m, dd, dm};  // Q q c Delta R S r A B
  const size_t ow[5] = {dm, dd, (size_t)d, (size_t)m, (size_t)d};                  // K P x u lam
  for (int k = 0; k < 9; ++k) in_w[k] = iw[k];
  for (int k = 0; k < 5; ++k) out_w[k] = ow[k];
}

size_t total_workspace_bytes(const PlanHost &ph, int precision) {
  size_t cur = workspace_layout(ph, precision).total_bytes;
  if (!ph.lift_N && ph.rg_n.empty()) return cur;  // lifted and ragged plans stage a uniform problem
  size_t iw[9], ow[5];
  lift_words(ph.n, ph.m, iw, ow);
  for (int k = 0; k < 9; ++k) cur = align_up(cur + iw[k] * 8 * (size_t)ph.N, 256);
  for (int k = 0; k < 5; ++k) cur = align_up(cur + ow[k] * 8 * (size_t)ph.N, 256);
  return cur;
}

static inline int *ws_status(void *ws) { return reinterpret_cast<int *>(ws); }
static inline double *ws_resid(void *ws) { return reinterpret_cast<double *>(static_cast<char *>(ws) + 256); }

// Pinned staging buffers of plan uploads, reused across uploads: a fresh
// pageable buffer per upload pays first-touch page faults on the host and a
// staged pageable copy.  Every pooled buffer holds STAGE_BYTES; the pool grows
// to STAGE_MAX buffers and is never freed (freeing pinned memory waits for the
// device, which would stall the solves on other streams).  Pinning a new
// buffer takes tens of milliseconds and holds up other HIP calls of the
// process, so beyond STAGE_MAX uploads at once, and for uploads larger than a
// buffer, the upload stages through ordinary heap memory instead.
namespace {
constexpr size_t STAGE_BYTES = size_t(32) << 20;
constexpr int STAGE_MAX = 4;
struct StagePool {
  std::mutex mu;
  std::vector<char *> free_bufs;
  int made = 0;
};
StagePool &stage_pool() {
  static StagePool *pool = new StagePool();
  return *pool;
}
// A pooled buffer, or nullptr when none is free and the pool is full.
char *stage_take() {
  StagePool &sp = stage_pool();
  {
    std::lock_guard<std::mutex> lock(sp.mu);
    if (!sp.free_bufs.empty()) {
      char *b = sp.free_bufs.back();
      sp.free_bufs.pop_back();
      return b;
    }
    if (sp.made >= STAGE_MAX) return nullptr;
    ++sp.made;
  }
  void *b = nullptr;
  if (hipHostMalloc(&b, STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
    std::lock_guard<std::mutex> lock(sp.mu);
    --sp.made;
    return nullptr;
  }
  return static_cast<char *>(b);
}
void stage_give(char *b) {
  StagePool &sp = stage_pool();
  std::lock_guard<std::mutex> lock(sp.mu);
  sp.free_bufs.push_back(b);
}
}  // namespace

// Device memory of the library (plan copies, plan-owned workspaces, residual
// buffers) comes from one stream-ordered pool per GPU that keeps up to
// POOL_KEEP_BYTES of freed memory mapped for reuse.  With a release threshold of
// zero (the default pool's), each allocation after a free maps fresh pages,
// which serialises with the other device allocations of the process; a serving
// loop uploads a plan per request.  The pools live until the process ends.
namespace {
constexpr uint64_t POOL_KEEP_BYTES = uint64_t(4) << 30;
constexpr int POOL_MAX_DEVICES = 64;
std::mutex pool_mu;
hipMemPool_t pools[POOL_MAX_DEVICES] = {};
}  // namespace

hipError_t dev_alloc(void **p, size_t bytes, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipStreamGetDevice(st, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= POOL_MAX_DEVICES) return hipMallocAsync(p, bytes, st);
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(pool_mu);
    if (!pools[dev]) {
      hipMemPoolProps props = {};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      if ((e = hipMemPoolCreate(&pool, &props)) != hipSuccess) return e;
      uint64_t keep = POOL_KEEP_BYTES;
      if ((e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return e;
      }
      pools[dev] = pool;
    }
    pool = pools[dev];
  }
  return hipMallocFromPoolAsync(p, bytes, pool, st);
}

// Byte sizes of the pieces of a plan's device copy, in their order in the
// allocation (each piece starts on a 256-byte boundary); returns the total.
constexpr int PLAN_PIECES = 18;
static size_t plan_pieces(const PlanHost &h, size_t bytes[PLAN_PIECES], size_t at[PLAN_PIECES]) {
  const int64_t NC = std::max<int64_t>(h.N, 1);
  const size_t b[PLAN_PIECES] = {
      h.ops.size() * sizeof(OpRec),
      h.exp_ops.size() * sizeof(Op4),
      h.tc_ops.size() * sizeof(Op4),
      h.sx_ops.size() * sizeof(Op4),
      h.parent32.size() * sizeof(int32_t),
      (size_t)(h.N + 1) * sizeof(int32_t),                   // child offsets
      (size_t)NC * sizeof(int32_t),                          // child ids
      (size_t)(h.N / (RES_HUB + 1) + 1) * sizeof(int32_t),  // hubs
      h.kind_off.size() * sizeof(int64_t),
      h.exp_off.size() * sizeof(int64_t),
      h.tc_off.size() * sizeof(int64_t),
      h.sx_off.size() * sizeof(int64_t),
      h.lift_plus.size() * sizeof(int32_t),
      h.rg_n.size() * sizeof(int32_t),
      h.rg_m.size() * sizeof(int32_t),
      h.rg_off.size() * sizeof(int64_t),
      (size_t)NC * sizeof(int32_t),  // U liveness per node
      (size_t)NC * sizeof(int32_t),  // edge slots condensed on their own
  };
  size_t total = 0;
  for (int k = 0; k < PLAN_PIECES; ++k) {
    bytes[k] = b[k];
    at[k] = total;
    total = align_up(total + std::max<size_t>(b[k], 16), 256);
  }
  return total;
}

size_t plan_device_bytes(const PlanHost &h) {
  size_t b[PLAN_PIECES], at[PLAN_PIECES];
  return plan_pieces(h, b, at);
}

// The plan's integer arrays live in one device allocation, made and filled in
// the order of `st` and released in stream order after the last solve that
// used them (no device-wide synchronisation on destroy).
int plan_upload(PlanObj &P, hipStream_t st) {
  if (P.dev.base) return RCR_OK;
  const PlanHost &h = P.host;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  P.dev.device = dev;
  struct Piece {
    void **dst;
    const void *src;  // nullptr: the child lists, written in place
  };
  const Piece pieces[PLAN_PIECES] = {
      {(void **)&P.dev.ops, h.ops.data()},
      {(void **)&P.dev.exp_ops, h.exp_ops.data()},
      {(void **)&P.dev.tc_ops, h.tc_ops.data()},
      {(void **)&P.dev.sx_ops, h.sx_ops.data()},
      {(void **)&P.dev.parent, h.parent32.data()},
      {(void **)&P.dev.child_off, nullptr},
      {(void **)&P.dev.child_idx, nullptr},
      {(void **)&P.dev.hubs, nullptr},
      {(void **)&P.dev.koff, h.kind_off.data()},
      {(void **)&P.dev.exp_off, h.exp_off.data()},
      {(void **)&P.dev.tc_off, h.tc_off.data()},
      {(void **)&P.dev.sx_off, h.sx_off.data()},
      {(void **)&P.dev.lift_plus, h.lift_plus.data()},
      {(void **)&P.dev.rg_n, h.rg_n.data()},
      {(void **)&P.dev.rg_m, h.rg_m.data()},
      {(void **)&P.dev.rg_off, h.rg_off.data()},
      {(void **)&P.dev.uabs, nullptr},
      {(void **)&P.dev.rest, nullptr},
  };
  constexpr int NP = PLAN_PIECES;
  const int64_t NC = std::max<int64_t>(h.N, 1);
  size_t bytes[NP], at[NP];
  const size_t total = plan_pieces(h, bytes, at);
  char *stage = total <= STAGE_BYTES ? stage_take() : nullptr;
  const bool pooled = stage != nullptr;
  std::unique_ptr<char[]> heap;
  if (!pooled) {
    heap.reset(new (std::nothrow) char[total]);
    stage = heap.get();
  }
  if (!stage) return RCR_OOM;
  for (int k = 0; k < NP; ++k) {
    if (pieces[k].src && bytes[k]) memcpy(stage + at[k], pieces[k].src, bytes[k]);
    const size_t pad = std::max<size_t>(bytes[k], 16);
    if (pieces[k].src && pad > bytes[k]) memset(stage + at[k] + bytes[k], 0, pad - bytes[k]);
  }
  {  // children of each node in increasing id: node i owns cidx[coff[i] .. coff[i + 1])
    int32_t *coff = reinterpret_cast<int32_t *>(stage + at[5]);
    int32_t *cidx = reinterpret_cast<int32_t *>(stage + at[6]);
    const int32_t *par = h.parent32.data();
    const int64_t N = h.N;
    memset(cidx, 0, (size_t)NC * sizeof(int32_t));
    // count node p's children at coff[p + 2] (the last node's count is never needed
    // as a start); after the prefix sum coff[p + 1] is the start of p, and the
    // scatter advances it to the end of p, which is the start of p + 1
    memset(coff, 0, (size_t)(N + 1) * sizeof(int32_t));
    for (int64_t j = 0; j < N; ++j)
      if (par[j] >= 0 && par[j] + 2 <= N) coff[par[j] + 2]++;
    for (int64_t i = 2; i <= N; ++i) coff[i] += coff[i - 1];
    for (int64_t j = 0; j < N; ++j)
      if (par[j] >= 0) cidx[coff[par[j] + 1]++] = (int32_t)j;
    // nodes whose child terms the residual sums in a workgroup of their own
    // (at most N / (RES_HUB + 1) of them: the children are distinct nodes)
    int32_t *hubs = reinterpret_cast<int32_t *>(stage + at[7]);
    int64_t nh = 0;
    hubs[0] = 0;
    for (int64_t i = 0; i < N; ++i)
      if (coff[i + 1] - coff[i] > RES_HUB) hubs[nh++] = (int32_t)i;
    P.dev.n_hubs = nh;
  }
  {  // flags of the device records and the lists of the fused first level (flags_and_lists)
    OpRec *dops = reinterpret_cast<OpRec *>(stage + at[0]);
    Op4 *dexp = reinterpret_cast<Op4 *>(stage + at[1]);
    int32_t *uabs = reinterpret_cast<int32_t *>(stage + at[16]);
    int32_t *rest = reinterpret_cast<int32_t *>(stage + at[17]);
    const size_t nops = h.ops.size(), nexp = h.exp_ops.size();
    const int64_t N = h.N;
    memset(uabs, 0, (size_t)NC * sizeof(int32_t));
    // ops are sorted by level: the first absorb of a node is the first one met
    for (size_t i = 0; i < nops; ++i) {
      OpRec &o = dops[i];
      int32_t f = 0;
      if (o.kind == OP_ABSORB) {
        if (!uabs[o.a]) f |= OPF_FIRST_ABSORB;
        uabs[o.a] = 1;
      }
      o.round = f;
    }
    for (size_t i = 0; i < nops; ++i) {
      OpRec &o = dops[i];
      if ((o.kind == OP_RAKE || o.kind == OP_COMPRESS) && uabs[o.a]) o.round |= OPF_U_LIVE;
    }
    for (size_t i = 0; i < nexp; ++i) dexp[i].d = uabs[dexp[i].a] ? OPF_U_LIVE : 0;
    // level 1 can be fused with the condensation when it holds only rakes and
    // compresses whose edges are original slots (the first round's)
    bool ok = h.levels() >= 1 && h.kind_off.size() >= 5 && h.kind_off[1] == h.kind_off[2] &&
              h.kind_off[2] == h.kind_off[3];
    std::vector<char> used(ok ? (size_t)N : 0, 0);
    for (int64_t i = ok ? h.kind_off[0] : 0; ok && i < h.kind_off[4]; ++i) {
      const OpRec &o = h.ops[(size_t)i];
      if (o.kind == OP_RAKE) {
        ok = o.b == o.a && o.a < N;
        if (ok) used[(size_t)o.a] = 1;
      } else if (o.kind == OP_COMPRESS) {
        ok = o.b == o.a && o.a < N && o.c >= 0 && o.c < N;
        if (ok) used[(size_t)o.a] = used[(size_t)o.c] = 1;
      } else {
        ok = false;
      }
    }
    int64_t nr = 0;
    if (ok)
      for (int64_t v = 0; v < N; ++v)
        if (h.parent32[(size_t)v] >= 0 && !used[(size_t)v]) rest[nr++] = (int32_t)v;
    P.dev.l1_fusable = ok;
    P.dev.n_rest = nr;
  }
  char *base = nullptr;
  if (dev_alloc((void **)&base, total, st) != hipSuccess) {
    if (pooled) stage_give(stage);
    return RCR_OOM;
  }
  for (int k = 0; k < NP; ++k) *pieces[k].dst = base + at[k];
  P.dev.base = base;
  P.dev.bytes = total;
  // the staging buffer goes back to the pool on return, and solves on other
  // streams may use the arrays: wait for the copy
  hipError_t e = hipMemcpyAsync(base, stage, total, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && !P.last_done) e = hipEventCreateWithFlags(&P.last_done, hipEventDisableTiming);
  if (pooled) stage_give(stage);
  if (e != hipSuccess) {
    fprintf(stderr, "rcr: plan upload failed: %s\n", hipGetErrorString(e));
    return RCR_HIP_ERROR;
  }
  return RCR_OK;
}

// A graph is destroyed only after its latest replay has completed (its `done`
// event, or the event recorded after a timed sequence's last graph).
static void destroy_graph(GraphEntry &e) {
  if (e.done) {
    (void)hipEventSynchronize(e.done);
    (void)hipEventDestroy(e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  e = GraphEntry();
}

static void destroy_timed(TimedGraph &t) {
  if (!t.events.empty()) (void)hipEventSynchronize(t.events.back());
  for (hipGraphExec_t g : t.execs) (void)hipGraphExecDestroy(g);
  for (hipEvent_t e : t.events) (void)hipEventDestroy(e);
  t = TimedGraph();
}

// Make room for one more entry in a graph cache: the least recently used
// entry goes once the cache holds GRAPH_CACHE_CAP entries.
template <typename Map, typename Destroy>
static void evict_lru(Map &cache, Destroy destroy) {
  while (cache.size() >= GRAPH_CACHE_CAP) {
    auto victim = cache.begin();
    for (auto it = cache.begin(); it != cache.end(); ++it)
      if (it->second.tick < victim->second.tick) victim = it;
    destroy(victim->second);
    cache.erase(victim);
  }
}

void drop_graphs(PlanObj &P) {
  for (auto &kv : P.graphs) destroy_graph(kv.second);
  P.graphs.clear();
  for (auto &kv : P.timed) destroy_timed(kv.second);
  P.timed.clear();
}

size_t graph_cache_size(const PlanObj &P) { return P.graphs.size() + P.timed.size(); }

// One stream of the library's own per GPU (non-blocking, default priority) on
// which plans release their device memory after their last solve.  The legacy
// default stream would order those frees with all other blocking work of the
// process, and a serving loop releases a plan per completed group.
namespace {
std::mutex rel_mu;
hipStream_t rel_streams[POOL_MAX_DEVICES] = {};
}  // namespace

static hipStream_t release_stream(int dev) {
  if (dev < 0 || dev >= POOL_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(rel_mu);
  if (!rel_streams[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess) rel_streams[dev] = st;
    if (cur != dev) (void)hipSetDevice(cur);
  }
  return rel_streams[dev];
}

void plan_release_device(PlanObj &P) {
  drop_graphs(P);
  for (hipEvent_t e : P.events) (void)hipEventDestroy(e);
  P.events.clear();
  // release after the last solve that used the plan (its completion event), in
  // the order of the library's release stream, without blocking the host
  void *ptrs[] = {P.dev.base, P.ws[0], P.ws[1], P.resid_buf};
  bool any = false;
  for (void *p : ptrs) any = any || p;
  int dev = P.dev.device;
  if (any && dev < 0 && hipGetDevice(&dev) != hipSuccess) dev = -1;
  hipStream_t rs = any ? release_stream(dev) : nullptr;
  if (any && P.last_done) (void)hipStreamWaitEvent(rs, P.last_done, 0);
  for (void *p : ptrs)
    if (p) (void)hipFreeAsync(p, rs);
  if (P.last_done) (void)hipEventDestroy(P.last_done);
  P.last_done = nullptr;
  P.dev = PlanDev();
  P.ws[0] = P.ws[1] = nullptr;
  P.ws_bytes[0] = P.ws_bytes[1] = 0;
  P.resid_buf = nullptr;
}

#define RCR_DECL_NB(NBV)                                                                                 \
  extern template int launch_phase_m<double, NBV>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int); \
  extern template int launch_phase_m<float, NBV>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
RCR_DECL_NB(4)
RCR_DECL_NB(6)
RCR_DECL_NB(8)
RCR_DECL_NB(12)
RCR_DECL_NB(16)

// phase 0: factor (Algorithm 1, Steps 2-3); phase 1: solve one right-hand side (Steps 4-6)
template <typename T>
static int launch_phase(PlanObj &P, Bufs<T> bf, Timer &tm, hipStream_t st, int phase) {
  switch (pad_n(bf.n)) {
    case 4: return launch_phase_m<T, 4>(P, bf, tm, st, phase);
    case 6: return launch_phase_m<T, 6>(P, bf, tm, st, phase);
    case 8: return launch_phase_m<T, 8>(P, bf, tm, st, phase);
    case 12: return launch_phase_m<T, 12>(P, bf, tm, st, phase);
    default: return launch_phase_m<T, 16>(P, bf, tm, st, phase);
  }
}

// ---- element-wise helpers of the mixed-precision path
template <typename A, typename B>
__global__ __launch_bounds__(256) void k_cast(const A *__restrict__ a, B *__restrict__ b, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) b[i] = (B)a[i];
}

// b += a (correction of the float64 iterate by a float32 step)
__global__ __launch_bounds__(256) void k_accumulate(const float *__restrict__ a, double *__restrict__ b, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    b[i] += (double)a[i];
}

static unsigned grid_for(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

// KKT residual blocks of eq. (kkt) in float64, one team of lanes per node v, written
// as the right-hand side of the correction solve (q' = r_x, r' = r_u, c'_root = r_root,
// c'_v = r_dyn) when rq is non-null; the max-abs residual is accumulated into out.
// Lane r < n forms the stationarity and dynamics rows r, lane r < m the control
// row r.  Every operand vector and row is fetched with all its loads issued at
// once (gather over the padded sizes NB, MB), so a node costs a few memory
// round trips (one per child for the child terms), not one per entry.  The
// grid strides over the nodes; each workgroup folds its lanes' maxima and
// issues one atomic, so the maximum does not serialise on one address.

// Max-abs fold of the residual rows that keeps a NaN: fmax returns its non-NaN
// operand, so a NaN reaching only some rows would otherwise be dropped.
__device__ __forceinline__ double fold_max(double a, double b) {
  return (a != a || b != b) ? INFINITY : fmax(a, b);
}

// Lanes per node of the residual kernel: 8 when both padded sizes fit (no
// lane idle at n, m <= 8), else 16.
template <int NB, int MB>
constexpr int res_team() {
  return NB <= 8 && MB <= 8 ? 8 : 16;
}

// The child terms of stationarity row rn of node v: for child j,
// (S_j u_j)[rn] + (A_j^T lambda_j)[rn], added to s.
template <int NB, int MB>
__device__ __forceinline__ double child_terms(int64_t j, int n, int m, int rn, const double *S, const double *u,
                                              const double *A, const double *y, double s) {
  const int nn = n * n, nm = n * m;
  double sj[MB], uj[MB], aj[NB], yj[NB];
  gather(sj, m, [&](int k) { return S[j * nm + rn * m + k]; });
  gather(uj, m, [&](int k) { return u[j * m + k]; });
  gather(aj, n, [&](int k) { return A[j * nn + k * n + rn]; });
  gather(yj, n, [&](int k) { return y[j * n + k]; });
  s = dot_n(sj, uj, m, s);
  return dot_n(aj, yj, n, s);
}

// HUB: node v has more than RES_HUB children, whose terms (row r) the caller
// has summed into csum; otherwise they are summed here in child order, and a
// node with more than RES_HUB children is skipped (returns 0, writes nothing).
template <typename OT, int NB, int MB, bool HUB = false>
__device__ __forceinline__ double residual_rhs(int64_t v, int n, int m, const double *Q, const double *q,
                                               const double *c, const double *De, const double *R, const double *S,
                                               const double *rr, const double *A, const double *B, const double *x,
                                               const double *u, const double *y, const int32_t *parent,
                                               const int32_t *coff, const int32_t *cidx, OT *rq, OT *rr_out, OT *rc,
                                               double csum = 0.0) {
  constexpr int TW = res_team<NB, MB>();
  const int r = threadIdx.x & (TW - 1);
  const int nn = n * n, nm = n * m;
  const int rn = r < n ? r : n - 1, rm = r < m ? r : m - 1;
  const int64_t pv = parent[v];
  const bool isroot = pv < 0;
  const int64_t pi = isroot ? v : pv;  // a valid row for the parent's loads
  double xv[NB], yv[NB], xp[NB], uv[MB], qr[NB], dr[NB], ar[NB], br[MB];
  gather(xv, n, [&](int k) { return x[v * n + k]; });
  gather(yv, n, [&](int k) { return y[v * n + k]; });
  gather(xp, n, [&](int k) { return x[pi * n + k]; });
  gather(uv, m, [&](int k) { return u[v * m + k]; });
  gather(qr, n, [&](int k) { return Q[v * nn + rn * n + k]; });
  gather(dr, n, [&](int k) { return De[v * nn + rn * n + k]; });
  gather(ar, n, [&](int k) { return A[v * nn + rn * n + k]; });
  gather(br, m, [&](int k) { return B[v * nm + rn * m + k]; });
  double sx[NB], bx[NB], rx[MB];  // control row r: S[:, r], B[:, r], R[r, :]
  gather(sx, n, [&](int k) { return S[v * nm + k * m + rm]; });
  gather(bx, n, [&](int k) { return B[v * nm + k * m + rm]; });
  gather(rx, m, [&](int k) { return R[v * m * m + rm * m + k]; });
  double s = q[v * n + rn] - y[v * n + rn];
  s = dot_n(qr, xv, n, s);
  if constexpr (HUB) {
    s += csum;
  } else {
    const int32_t t0 = coff[v], t1 = coff[v + 1];
    if (t1 - t0 > RES_HUB) return 0.0;  // a hub: k_residual_hub covers the node
    for (int32_t t = t0; t < t1; ++t) s = child_terms<NB, MB>(cidx[t], n, m, rn, S, u, A, y, s);
  }
  double worst = 0.0;
  if (r < n) worst = fold_max(worst, fabs(s));
  double t = c[v * n + rn] - x[v * n + rn];
  if (isroot) {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) t = fma(-dr[k], yv[k], t);
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < n) t = fma(-dr[k], yv[k], fma(ar[k], xp[k], t));
    t = dot_n(br, uv, m, t);
  }
  if (r < n) {
    worst = fold_max(worst, fabs(t));
    if (rq) {
      rq[v * n + r] = (OT)s;
      rc[v * n + r] = (OT)t;
    }
  }
  if (r < m) {
    double tu = 0.0;
    if (!isroot) {
      tu = rr[v * m + r];
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < n) tu = fma(bx[k], yv[k], fma(sx[k], xp[k], tu));
      tu = dot_n(rx, uv, m, tu);
    }
    worst = fold_max(worst, fabs(tu));
    if (rq) rr_out[v * m + r] = (OT)tu;
  }
  return worst;
}

template <typename OT, int NB, int MB>
__global__ __launch_bounds__(256) void k_residual_rhs(int64_t N, int n, int m, const double *Q, const double *q,
                                                      const double *c, const double *De, const double *R,
                                                      const double *S, const double *rr, const double *A,
                                                      const double *B, const double *x, const double *u,
                                                      const double *y, const int32_t *parent, const int32_t *coff,
                                                      const int32_t *cidx, OT *rq, OT *rr_out, OT *rc, double *out) {
  constexpr int TW = res_team<NB, MB>(), TPB = 256 / TW;
  __shared__ double wmax[256 / 64];
  double worst = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x / TW; v < N; v += (int64_t)gridDim.x * TPB) {
    const double w =
        (n == NB && m == MB)  // unpadded: every bound a compile-time constant
            ? residual_rhs<OT, NB, MB>(v, NB, MB, Q, q, c, De, R, S, rr, A, B, x, u, y, parent, coff, cidx, rq,
                                       rr_out, rc)
            : residual_rhs<OT, NB, MB>(v, n, m, Q, q, c, De, R, S, rr, A, B, x, u, y, parent, coff, cidx, rq,
                                       rr_out, rc);
    worst = fmax(worst, w);
  }
  for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    double w = wmax[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) w = fmax(w, wmax[i]);
    if (w > 0.0) atomicMax(reinterpret_cast<unsigned long long *>(out), (unsigned long long)__double_as_longlong(w));
  }
}

// The nodes with more than RES_HUB children, one workgroup each: team k sums
// the terms of children k, k + teams, ... in that order, the partial sums are
// added in team order, and team 0 forms the node's residual rows.  The order
// is fixed by the launch, so results do not vary between runs.
template <typename OT, int NB, int MB>
__global__ __launch_bounds__(256) void k_residual_hub(int64_t N, int n, int m, const double *Q, const double *q,
                                                      const double *c, const double *De, const double *R,
                                                      const double *S, const double *rr, const double *A,
                                                      const double *B, const double *x, const double *u,
                                                      const double *y, const int32_t *parent, const int32_t *coff,
                                                      const int32_t *cidx, const int32_t *hubs, OT *rq, OT *rr_out,
                                                      OT *rc, double *out) {
  constexpr int TW = res_team<NB, MB>(), TEAMS = 256 / TW;
  __shared__ double part[256];
  __shared__ double wmax[256 / 64];
  const int64_t v = hubs[blockIdx.x];
  const int k = threadIdx.x / TW, r = threadIdx.x & (TW - 1);
  const bool exact = n == NB && m == MB;
  const int rn = r < n ? r : n - 1;
  double s = 0.0;
  const int32_t te = coff[v + 1];
  int32_t t = coff[v] + k;
  int64_t j = t < te ? cidx[t] : 0;
  while (t < te) {
    // the next child's id is fetched with this child's operands, not after them
    const int32_t tn = t + TEAMS;
    const int64_t jn = tn < te ? cidx[tn] : 0;
    s = exact ? child_terms<NB, MB>(j, NB, MB, rn, S, u, A, y, s) : child_terms<NB, MB>(j, n, m, rn, S, u, A, y, s);
    t = tn;
    j = jn;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  double worst = 0.0;
  if (k == 0) {
    double csum = part[r];
    for (int i = 1; i < TEAMS; ++i) csum += part[i * TW + r];
    worst = exact ? residual_rhs<OT, NB, MB, true>(v, NB, MB, Q, q, c, De, R, S, rr, A, B, x, u, y, parent, coff,
                                                    cidx, rq, rr_out, rc, csum)
                  : residual_rhs<OT, NB, MB, true>(v, n, m, Q, q, c, De, R, S, rr, A, B, x, u, y, parent, coff,
                                                    cidx, rq, rr_out, rc, csum);
  }
  for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    double w = wmax[0];
    for (int i = 1; i < 256 / 64; ++i) w = fmax(w, wmax[i]);
    if (w > 0.0) atomicMax(reinterpret_cast<unsigned long long *>(out), (unsigned long long)__double_as_longlong(w));
  }
}

template <typename OT, int NB>
static void launch_residual_nb(const PlanHost &h, const rcr_problem &in, const rcr_solution &out, OT *rq, OT *rr,
                               OT *rc, const PlanObj &P, double *resid, hipStream_t st) {
  const dim3 g(std::min<unsigned>(blocks_for(h.N, 256 / res_team<NB, 16>()), 4096u)), b(256);
#define RCR_RES_ARGS                                                                                           \
  h.N, h.n, h.m, in.Q, in.q, in.c, in.Delta, in.R, in.S, in.r, in.A, in.B, out.x, out.u, out.lam, P.dev.parent, \
      P.dev.child_off, P.dev.child_idx, rq, rr, rc, resid
  switch (pad_m(h.m)) {
    case 4: hipLaunchKernelGGL((k_residual_rhs<OT, NB, 4>), g, b, 0, st, RCR_RES_ARGS); break;
    case 8: hipLaunchKernelGGL((k_residual_rhs<OT, NB, 8>), g, b, 0, st, RCR_RES_ARGS); break;
    default: hipLaunchKernelGGL((k_residual_rhs<OT, NB, 16>), g, b, 0, st, RCR_RES_ARGS); break;
  }
#undef RCR_RES_ARGS
  if (P.dev.n_hubs > 0) {
    const dim3 gh((unsigned)P.dev.n_hubs), bh(256);
#define RCR_HUB_ARGS                                                                                           \
  h.N, h.n, h.m, in.Q, in.q, in.c, in.Delta, in.R, in.S, in.r, in.A, in.B, out.x, out.u, out.lam, P.dev.parent, \
      P.dev.child_off, P.dev.child_idx, P.dev.hubs, rq, rr, rc, resid
    switch (pad_m(h.m)) {
      case 4: hipLaunchKernelGGL((k_residual_hub<OT, NB, 4>), gh, bh, 0, st, RCR_HUB_ARGS); break;
      case 8: hipLaunchKernelGGL((k_residual_hub<OT, NB, 8>), gh, bh, 0, st, RCR_HUB_ARGS); break;
      default: hipLaunchKernelGGL((k_residual_hub<OT, NB, 16>), gh, bh, 0, st, RCR_HUB_ARGS); break;
    }
#undef RCR_HUB_ARGS
  }
}

template <typename OT>
static void launch_residual_rhs(PlanObj &P, const rcr_problem &in, const rcr_solution &out, OT *rq, OT *rr, OT *rc,
                                double *resid, hipStream_t st) {
  const PlanHost &h = P.host;
  switch (pad_n(h.n)) {
    case 4: launch_residual_nb<OT, 4>(h, in, out, rq, rr, rc, P, resid, st); break;
    case 6: launch_residual_nb<OT, 6>(h, in, out, rq, rr, rc, P, resid, st); break;
    case 8: launch_residual_nb<OT, 8>(h, in, out, rq, rr, rc, P, resid, st); break;
    case 12: launch_residual_nb<OT, 12>(h, in, out, rq, rr, rc, P, resid, st); break;
    default: launch_residual_nb<OT, 16>(h, in, out, rq, rr, rc, P, resid, st); break;
  }
}

template <typename T>
static Bufs<T> make_bufs(PlanObj &P, const WsLayout &L, void *ws, const rcr_problem &in) {
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
  bf.uabs = P.dev.uabs;
  bf.status = ws_status(ws);
  return bf;
}

// Working buffers of a factor (K, P: the caller's float64 outputs) and, when io
// is given, of the solve of one right-hand side.  Float64 works in the caller's
// arrays; float32 in the workspace copies (right-hand side, K, P, x, u, lam).
template <typename T>
static Bufs<T> bufs_for(PlanObj &P, const WsLayout &L, void *ws, const rcr_problem &in, double *K, double *Pm,
                        const RhsIO *io) {
  Bufs<T> bf = make_bufs<T>(P, L, ws, in);
  if constexpr (sizeof(T) == sizeof(double)) {
    bf.PW = Pm;
    bf.Kw = K;
    if (io) {
      bf.sq = io->q;
      bf.sr = io->r;
      bf.sc = io->c;
      bf.xw = io->x;
      bf.uw = io->u;
      bf.yw = io->lam;
    }
  } else {
    T *base = reinterpret_cast<T *>(ws);
    bf.sq = base + L.rq;
    bf.sr = base + L.rr;
    bf.sc = base + L.rc;
    bf.PW = base + L.PW;
    bf.Kw = base + L.Kw;
    bf.xw = base + L.xw;
    bf.uw = base + L.uw;
    bf.yw = base + L.yw;
  }
  return bf;
}

// The problem a residual or correction sees: the matrices of `in`, the
// right-hand side (q, r, c) of `io`.
static rcr_problem with_rhs(const rcr_problem &in, const RhsIO &io) {
  rcr_problem p = in;
  p.q = io.q;
  p.r = io.r;
  p.c = io.c;
  return p;
}

static rcr_solution sol_of(const RhsIO &io, double *K, double *Pm) { return rcr_solution{K, Pm, io.x, io.u, io.lam}; }

// MIXED32: the float32 copy of a right-hand side that the solve passes read.
static void cast_rhs(PlanObj &P, const WsLayout &L, void *ws, const RhsIO &io, Timer &tm, hipStream_t st) {
  const PlanHost &h = P.host;
  const int64_t Nn = h.N * h.n, Nm = h.N * h.m;
  float *base = reinterpret_cast<float *>(ws);
  tm.begin(RCR_K_RESIDUAL);
  LAUNCH(tm, (k_cast<double, float>), dim3(grid_for(Nn)), dim3(256), 0, st, io.q, base + L.rq, Nn);
  LAUNCH(tm, (k_cast<double, float>), dim3(grid_for(Nm)), dim3(256), 0, st, io.r, base + L.rr, Nm);
  LAUNCH(tm, (k_cast<double, float>), dim3(grid_for(Nn)), dim3(256), 0, st, io.c, base + L.rc, Nn);
}

// MIXED32, after the float32 solve of io's right-hand side: x, u, lam in float64,
// then `refine` correction solves on the float64 KKT residual of eq. (kkt)
// (q' = r_x, r' = r_u, c'_root = r_root, c'_j = r_dyn), each reusing the factor.
static int finish_mixed(PlanObj &P, const rcr_problem &in, const RhsIO &io, int refine, Bufs<float> bf,
                        const WsLayout &L, void *ws, Timer &tm, hipStream_t st) {
  const PlanHost &h = P.host;
  const int64_t Nn = h.N * h.n, Nm = h.N * h.m;
  float *base = reinterpret_cast<float *>(ws);
  tm.begin(RCR_K_RESIDUAL);
  LAUNCH(tm, (k_cast<float, double>), dim3(grid_for(Nn)), dim3(256), 0, st, bf.xw, io.x, Nn);
  LAUNCH(tm, (k_cast<float, double>), dim3(grid_for(Nm)), dim3(256), 0, st, bf.uw, io.u, Nm);
  LAUNCH(tm, (k_cast<float, double>), dim3(grid_for(Nn)), dim3(256), 0, st, bf.yw, io.lam, Nn);
  const rcr_problem pin = with_rhs(in, io);
  const rcr_solution sol = sol_of(io, nullptr, nullptr);
  for (int it = 0; it < refine; ++it) {
    tm.begin(RCR_K_RESIDUAL);
    tm.pre();
    launch_residual_rhs<float>(P, pin, sol, base + L.rq, base + L.rr, base + L.rc, ws_resid(ws), st);
    tm.post();
    const int rc = launch_phase<float>(P, bf, tm, st, 1);
    if (rc) return rc;
    tm.begin(RCR_K_RESIDUAL);
    LAUNCH(tm, k_accumulate, dim3(grid_for(Nn)), dim3(256), 0, st, bf.xw, io.x, Nn);
    LAUNCH(tm, k_accumulate, dim3(grid_for(Nm)), dim3(256), 0, st, bf.uw, io.u, Nm);
    LAUNCH(tm, k_accumulate, dim3(grid_for(Nn)), dim3(256), 0, st, bf.yw, io.lam, Nn);
  }
  HIPCK(hipGetLastError());
  return RCR_OK;
}

// MIXED32: the float32 K, P of the factor into the caller's float64 arrays.
static void cast_factor_out(PlanObj &P, const WsLayout &L, void *ws, double *K, double *Pm, Timer &tm,
                            hipStream_t st) {
  const PlanHost &h = P.host;
  const int64_t Nnn = h.N * h.n * h.n, Nmn = h.N * h.m * h.n;
  float *base = reinterpret_cast<float *>(ws);
  tm.begin(RCR_K_RESIDUAL);
  LAUNCH(tm, (k_cast<float, double>), dim3(grid_for(Nmn)), dim3(256), 0, st, base + L.Kw, K, Nmn);
  LAUNCH(tm, (k_cast<float, double>), dim3(grid_for(Nnn)), dim3(256), 0, st, base + L.PW, Pm, Nnn);
}

// The whole launch sequence of one rcr_solve on `st` (directly, or while a
// graph is captured): the factor and the solve of the problem's own
// right-hand side, the two phases sharing it (RCR_PHASE_FIRST_RHS).
static int launch_sequence(PlanObj &P, const rcr_problem &in, const rcr_solution &out, const rcr_solve_options &opt,
                           const WsLayout &L, void *ws, Timer &tm, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, ws_status(ws), ws_resid(ws));
  const RhsIO io{in.q, in.r, in.c, out.x, out.u, out.lam};
  if (opt.precision == RCR_FP64) {
    Bufs<double> bf = bufs_for<double>(P, L, ws, in, out.K, out.P, &io);
    int rc = launch_phase<double>(P, bf, tm, st, 0 | RCR_PHASE_FIRST_RHS | RCR_PHASE_ONE_RHS);
    if (!rc) rc = launch_phase<double>(P, bf, tm, st, 1 | RCR_PHASE_FIRST_RHS | RCR_PHASE_ONE_RHS);
    return rc;
  }
  // MIXED32: float32 factor and solves; float64 R/G Cholesky and compress (I + C P)
  // solve inside the kernels; float64 residual, correction right-hand side and update.
  cast_rhs(P, L, ws, io, tm, st);
  Bufs<float> bf = bufs_for<float>(P, L, ws, in, out.K, out.P, &io);
  int rc = launch_phase<float>(P, bf, tm, st, 0 | RCR_PHASE_FIRST_RHS);
  if (!rc) rc = launch_phase<float>(P, bf, tm, st, 1 | RCR_PHASE_FIRST_RHS);
  if (!rc) rc = finish_mixed(P, in, io, opt.refine_steps, bf, L, ws, tm, st);
  if (rc) return rc;
  cast_factor_out(P, L, ws, out.K, out.P, tm, st);
  HIPCK(hipGetLastError());
  return RCR_OK;
}

// Algorithm 1, Steps 2-3 only: the factor stays in the workspace (and in the
// caller's K, P), ready for any number of right-hand sides.
static int factor_sequence(PlanObj &P, const rcr_problem &in, double *K, double *Pm, int prec, const WsLayout &L,
                           void *ws, Timer &tm, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, ws_status(ws), ws_resid(ws));
  if (prec == RCR_FP64) return launch_phase<double>(P, bufs_for<double>(P, L, ws, in, K, Pm, nullptr), tm, st, 0);
  const int rc = launch_phase<float>(P, bufs_for<float>(P, L, ws, in, K, Pm, nullptr), tm, st, 0);
  if (rc) return rc;
  cast_factor_out(P, L, ws, K, Pm, tm, st);
  HIPCK(hipGetLastError());
  return RCR_OK;
}

// Algorithm 1, Steps 4-6 for each of k right-hand sides, in order, on the
// factor in the workspace (K, Pm: the factor's float64 outputs).
static int rhs_sequence(PlanObj &P, const rcr_problem &in, const double *K, const double *Pm, int32_t k,
                        const RhsIO *ios, int prec, int refine, const WsLayout &L, void *ws, Timer &tm,
                        hipStream_t st) {
  double *Kd = const_cast<double *>(K), *Pd = const_cast<double *>(Pm);  // read only by the solve passes
  for (int32_t i = 0; i < k; ++i) {
    int rc;
    if (prec == RCR_FP64) {
      rc = launch_phase<double>(P, bufs_for<double>(P, L, ws, in, Kd, Pd, &ios[i]), tm, st, 1);
    } else {
      cast_rhs(P, L, ws, ios[i], tm, st);
      Bufs<float> bf = bufs_for<float>(P, L, ws, in, Kd, Pd, &ios[i]);
      rc = launch_phase<float>(P, bf, tm, st, 1);
      if (!rc) rc = finish_mixed(P, in, ios[i], refine, bf, L, ws, tm, st);
    }
    if (rc) return rc;
  }
  HIPCK(hipGetLastError());
  return RCR_OK;
}

// Replay the launch sequence `seq(timer, stream)` from the plan's graph cache
// under `key`, capturing it into a graph on a miss.
template <typename F>
static int replay_graph(PlanObj &P, const GraphKey &key, hipStream_t st, F &&seq) {
  auto it = P.graphs.find(key);
  if (it == P.graphs.end()) {
    hipStream_t cs;
    HIPCK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (be != hipSuccess) {
      (void)hipStreamDestroy(cs);
      HIPCK(be);
    }
    Timer off;
    const int lrc = seq(off, cs);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (lrc || ce != hipSuccess) {
      if (ce == hipSuccess && g) (void)hipGraphDestroy(g);
      if (lrc) return lrc;
      HIPCK(ce);
    }
    GraphEntry e;
    const hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCK(ie);
    if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGraphExecDestroy(e.exec);
      return RCR_HIP_ERROR;
    }
    evict_lru(P.graphs, destroy_graph);
    it = P.graphs.emplace(key, e).first;
  }
  it->second.tick = ++P.tick;
  HIPCK(hipGraphLaunch(it->second.exec, st));
  HIPCK(hipEventRecord(it->second.done, st));
  return RCR_OK;
}

static GraphKey key_of(std::initializer_list<const void *> ptrs, int64_t tag) {
  GraphKey k;
  k.reserve(ptrs.size() + 1);
  k.push_back((uintptr_t)tag);
  for (const void *p : ptrs) k.push_back((uintptr_t)p);
  return k;
}

// Device memory of a call: the caller's workspace, or the plan-owned one of
// this precision (made on first use, in the order of `st`).
static int take_workspace(PlanObj &P, const rcr_solve_options &opt, size_t need_solver, size_t need_total,
                          hipStream_t st, void *&ws) {
  const int prec = opt.precision;
  ws = opt.workspace;
  if (ws) {
    if ((size_t)opt.workspace_bytes < need_solver) return RCR_SMALL_WORKSPACE;
    return RCR_OK;
  }
  if (P.ws[prec] && P.ws_bytes[prec] < need_total) {
    (void)hipFreeAsync(P.ws[prec], st);
    P.ws[prec] = nullptr;
  }
  if (!P.ws[prec]) {
    if (dev_alloc(&P.ws[prec], need_total, st) != hipSuccess) return RCR_OOM;
    P.ws_bytes[prec] = need_total;
  }
  ws = P.ws[prec];
  return RCR_OK;
}

// Device time and launch counts per kernel class from a per-launch Timer.
static int report_timer(const Timer &tm, const TimedGraph *tg, const rcr_solve_options &opt) {
  for (int c = 0; c < RCR_NUM_KERNEL_CLASSES; ++c) {
    opt.kernel_ms[c] = 0.f;
    if (opt.kernel_launches) opt.kernel_launches[c] = 0;
  }
  if (tg) {
    for (size_t i = 0; i < tg->execs.size(); ++i) {
      if (tg->cls[i] < 0) continue;
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, tg->events[i], tg->events[i + 1]));
      opt.kernel_ms[tg->cls[i]] += ms;
    }
  }
  for (auto &sp : tm.spans) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, sp.second.first, sp.second.second));
    opt.kernel_ms[sp.first] += ms;
  }
  if (opt.kernel_launches)
    for (int c = 0; c < RCR_NUM_KERNEL_CLASSES; ++c) opt.kernel_launches[c] = tg ? tg->launches[c] : tm.launches[c];
  return RCR_OK;
}

// After a call's launches: optional residual, completion event, optional
// synchronisation with the status and residual read back.
static int finish_call(PlanObj &P, void *ws, const rcr_solve_options &opt, Timer &tm, const TimedGraph *tg,
                       const std::vector<std::pair<rcr_problem, rcr_solution>> &resid_of, hipStream_t st) {
  if (opt.kkt_residual) {
    tm.begin(RCR_K_RESIDUAL);
    // the residual of the returned iterates (the refinement's accumulator is reset first)
    tm.gap();
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, ws_status(ws) + 8, ws_resid(ws));
    for (const auto &ps : resid_of)
      launch_residual_rhs<double>(P, ps.first, ps.second, nullptr, nullptr, nullptr, ws_resid(ws), st);
    HIPCK(hipGetLastError());
  }
  if (!P.last_done) HIPCK(hipEventCreateWithFlags(&P.last_done, hipEventDisableTiming));
  HIPCK(hipEventRecord(P.last_done, st));
  if (opt.check || opt.kkt_residual || tm.on) {
    HIPCK(hipStreamSynchronize(st));
    if (tm.on) {
      const int rc = report_timer(tm, tg, opt);
      if (rc) return rc;
    }
    double resid = 0.0;
    int stw = 0;
    HIPCK(hipMemcpyAsync(&resid, ws_resid(ws), sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(&stw, ws_status(ws), sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (opt.kkt_residual) *opt.kkt_residual = resid;
    if (opt.check) {
      if (stw & ST_NOT_PD) return RCR_NOT_PD;
      if (stw & ST_SINGULAR) return RCR_SINGULAR;
      if (stw & ST_NONFINITE) return RCR_NONFINITE;
    }
  }
  return RCR_OK;
}

// Timed replay (kernel_ms with the graph executor): the sequence is captured
// as one graph per run of same-class launches, replayed with HIP events
// between them, so a class's launches run back to back as in a plain replay.
static int timed_replay(PlanObj &P, const GraphKey &key, const rcr_problem &in, const rcr_solution &out,
                        const rcr_solve_options &opt, const WsLayout &L, void *ws, hipStream_t st,
                        const TimedGraph *&tg) {
  auto it = P.timed.find(key);
  if (it == P.timed.end()) {
    struct Cap {
      hipStream_t cs;
      TimedGraph rec;
      int cur = -1;
      hipError_t err = hipSuccess;
      void end_run() {  // close the capture of the current run (empty runs are dropped)
        hipGraph_t g;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (e != hipSuccess) {
          err = e;
          return;
        }
        size_t nn = 0;
        if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess && nn > 0) {
          hipGraphExec_t ge;
          e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          if (e == hipSuccess) {
            rec.execs.push_back(ge);
            rec.cls.push_back(cur);
          } else {
            err = e;
          }
        }
        (void)hipGraphDestroy(g);
      }
      static void split(void *self, int c) {
        Cap *k = static_cast<Cap *>(self);
        if (k->err != hipSuccess) return;
        k->end_run();
        if (k->err == hipSuccess) k->err = hipStreamBeginCapture(k->cs, hipStreamCaptureModeThreadLocal);
        k->cur = c;
      }
    } cap;
    HIPCK(hipStreamCreateWithFlags(&cap.cs, hipStreamNonBlocking));
    const hipError_t be = hipStreamBeginCapture(cap.cs, hipStreamCaptureModeThreadLocal);
    if (be != hipSuccess) {
      (void)hipStreamDestroy(cap.cs);
      HIPCK(be);
    }
    Timer tc;
    tc.P = &P;
    tc.st = cap.cs;
    tc.on = true;
    tc.split = &Cap::split;
    tc.split_arg = &cap;
    const int lrc = launch_sequence(P, in, out, opt, L, ws, tc, cap.cs);
    if (cap.err == hipSuccess) cap.end_run();
    (void)hipStreamDestroy(cap.cs);
    for (int c = 0; c < RCR_NUM_KERNEL_CLASSES; ++c) cap.rec.launches[c] = tc.launches[c];
    bool ok = !lrc && cap.err == hipSuccess;
    for (size_t i = 0; ok && i <= cap.rec.execs.size(); ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) ok = false;
      else cap.rec.events.push_back(e);
    }
    if (!ok) {
      for (hipGraphExec_t g : cap.rec.execs) (void)hipGraphExecDestroy(g);
      for (hipEvent_t e : cap.rec.events) (void)hipEventDestroy(e);
      if (lrc) return lrc;
      HIPCK(cap.err);
      return RCR_HIP_ERROR;
    }
    evict_lru(P.timed, destroy_timed);
    it = P.timed.emplace(key, cap.rec).first;
  }
  it->second.tick = ++P.tick;
  tg = &it->second;
  HIPCK(hipEventRecord(tg->events[0], st));
  for (size_t i = 0; i < tg->execs.size(); ++i) {
    HIPCK(hipGraphLaunch(tg->execs[i], st));
    HIPCK(hipEventRecord(tg->events[i + 1], st));
  }
  return RCR_OK;
}

int solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt, hipStream_t st) {
  std::lock_guard<std::mutex> lock(P.mu);
  int rc = plan_upload(P, st);
  if (rc) return rc;
  const int prec = opt.precision;
  const WsLayout L = workspace_layout(P.host, prec);
  void *ws = nullptr;
  if ((rc = take_workspace(P, opt, L.total_bytes, total_workspace_bytes(P.host, prec), st, ws))) return rc;
  if (ws == P.ws[prec]) P.ws_factor[prec] = false;  // a solve leaves no factor for rcr_solve_rhs
  Timer tm;
  tm.P = &P;
  tm.st = st;
  tm.on = opt.kernel_ms != nullptr;
  const TimedGraph *tg = nullptr;
  const GraphKey key = key_of({in.Q, in.q, in.c, in.Delta, in.R, in.S, in.r, in.A, in.B, out.K, out.P, out.x,
                               out.u, out.lam, ws},
                              1 + 16 * prec + 256 * (int64_t)opt.refine_steps);
  if (opt.executor == RCR_EXEC_GRAPH && tm.on) {
    rc = timed_replay(P, key, in, out, opt, L, ws, st, tg);
  } else if (opt.executor == RCR_EXEC_GRAPH) {
    rc = replay_graph(P, key, st, [&](Timer &t, hipStream_t cs) { return launch_sequence(P, in, out, opt, L, ws, t, cs); });
  } else {
    rc = launch_sequence(P, in, out, opt, L, ws, tm, st);
  }
  if (rc) return rc;
  return finish_call(P, ws, opt, tm, tg, {{in, out}}, st);
}

int factor(PlanObj &P, const rcr_problem &in, double *K, double *Pm, const rcr_solve_options &opt,
           hipStream_t st) {
  std::lock_guard<std::mutex> lock(P.mu);
  int rc = plan_upload(P, st);
  if (rc) return rc;
  const int prec = opt.precision;
  const WsLayout L = workspace_layout(P.host, prec);
  void *ws = nullptr;
  if ((rc = take_workspace(P, opt, L.total_bytes, total_workspace_bytes(P.host, prec), st, ws))) return rc;
  Timer tm;
  tm.P = &P;
  tm.st = st;
  tm.on = opt.kernel_ms != nullptr;
  if (opt.executor == RCR_EXEC_GRAPH && !tm.on) {
    const GraphKey key = key_of({in.Q, in.Delta, in.R, in.S, in.A, in.B, K, Pm, ws}, 2 + 16 * prec);
    rc = replay_graph(P, key, st, [&](Timer &t, hipStream_t cs) {
      return factor_sequence(P, in, K, Pm, prec, L, ws, t, cs);
    });
  } else {
    rc = factor_sequence(P, in, K, Pm, prec, L, ws, tm, st);
  }
  if (rc) return rc;
  if (ws == P.ws[prec]) P.ws_factor[prec] = true;
  rcr_solve_options o = opt;
  o.kkt_residual = nullptr;  // no iterate yet
  return finish_call(P, ws, o, tm, nullptr, {}, st);
}

int solve_rhs(PlanObj &P, const rcr_problem &in, const double *K, const double *Pm, int32_t k, const RhsIO *ios,
              const rcr_solve_options &opt, hipStream_t st) {
  std::lock_guard<std::mutex> lock(P.mu);
  int rc = plan_upload(P, st);
  if (rc) return rc;
  const int prec = opt.precision;
  const WsLayout L = workspace_layout(P.host, prec);
  void *ws = opt.workspace ? opt.workspace : P.ws[prec];
  if (!opt.workspace && !P.ws_factor[prec]) return RCR_BAD_OPTION;  // no factor of this precision in the plan's workspace
  if (opt.workspace && (size_t)opt.workspace_bytes < L.total_bytes) return RCR_SMALL_WORKSPACE;
  Timer tm;
  tm.P = &P;
  tm.st = st;
  tm.on = opt.kernel_ms != nullptr;
  if (opt.executor == RCR_EXEC_GRAPH && !tm.on) {
    GraphKey key = key_of({in.Q, in.Delta, in.R, in.S, in.A, in.B, K, Pm, ws},
                          3 + 16 * prec + 256 * (int64_t)opt.refine_steps);
    for (int32_t i = 0; i < k; ++i)
      for (const void *p : {(const void *)ios[i].q, (const void *)ios[i].r, (const void *)ios[i].c,
                            (const void *)ios[i].x, (const void *)ios[i].u, (const void *)ios[i].lam})
        key.push_back((uintptr_t)p);
    rc = replay_graph(P, key, st, [&](Timer &t, hipStream_t cs) {
      return rhs_sequence(P, in, K, Pm, k, ios, prec, opt.refine_steps, L, ws, t, cs);
    });
  } else {
    rc = rhs_sequence(P, in, K, Pm, k, ios, prec, opt.refine_steps, L, ws, tm, st);
  }
  if (rc) return rc;
  std::vector<std::pair<rcr_problem, rcr_solution>> rs;
  if (opt.kkt_residual)
    for (int32_t i = 0; i < k; ++i) rs.push_back({with_rhs(in, ios[i]), sol_of(ios[i], nullptr, nullptr)});
  return finish_call(P, ws, opt, tm, nullptr, rs, st);
}

// ------------------------------------------------------------ adjoint
// Gradients of a scalar loss L with respect to the matrices of the problem,
// from the forward solution (x, u, y) and the adjoint vector a = (a_x, a_u, a_y)
// (the solve of the seeds dL/dx, dL/du, dL/dy, which is also dL/d(q, r, c)).
// With M the symmetric KKT matrix of eq. (kkt) and M (x, u, y) = -(q, r, c),
// dL = a^T dM (x, u, y), and dM pairs each block with its place in eq. (kkt):
//   dQ_i = a_x,i x_i^T          (Q_i x_i in the stationarity of x_i)
//   dDelta_j = -a_y,j y_j^T     (-Delta_j y_j in the dynamics into j / root)
//   dR_e = a_u,e u_e^T          (R_e u_e in the control stationarity)
//   dS_e = a_x,i u_e^T + x_i a_u,e^T          (M_e u_e and M_e^T x_i)
//   dA_e = a_y,j x_i^T + y_j a_x,i^T          (A_e x_i and A_e^T y_j)
//   dB_e = a_y,j u_e^T + y_j a_u,e^T          (B_e u_e and B_e^T y_j)
// for e = (i, j) in edge slot j; the root's edge slot is written as zero.
// One thread per output entry; a null output is skipped.
__global__ __launch_bounds__(256) void k_adjoint_grads(int64_t N, int n, int m, const int32_t *__restrict__ parent,
                                                       const double *__restrict__ x, const double *__restrict__ u,
                                                       const double *__restrict__ y, const double *__restrict__ ax,
                                                       const double *__restrict__ au, const double *__restrict__ ay,
                                                       double *dQ, double *dD, double *dR, double *dS, double *dA,
                                                       double *dB) {
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  const int64_t per = 3 * nn + mm + 2 * nm;  // entries of dQ, dDelta, dA, dR, dS, dB per node
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * per; t += stride) {
    const int64_t v = t / per;
    int64_t e = t - v * per;
    const int64_t pi = parent[v];
    const bool edge = pi >= 0;
    if (e < nn) {
      const int a = (int)(e / n), b = (int)(e % n);
      if (dQ) dQ[v * nn + e] = ax[v * n + a] * x[v * n + b];
      continue;
    }
    e -= nn;
    if (e < nn) {
      const int a = (int)(e / n), b = (int)(e % n);
      if (dD) dD[v * nn + e] = -ay[v * n + a] * y[v * n + b];
      continue;
    }
    e -= nn;
    if (e < nn) {
      const int a = (int)(e / n), b = (int)(e % n);
      if (dA) dA[v * nn + e] = edge ? fma(ay[v * n + a], x[pi * n + b], y[v * n + a] * ax[pi * n + b]) : 0.0;
      continue;
    }
    e -= nn;
    if (e < mm) {
      const int a = (int)(e / m), b = (int)(e % m);
      if (dR) dR[v * mm + e] = edge ? au[v * m + a] * u[v * m + b] : 0.0;
      continue;
    }
    e -= mm;
    if (e < nm) {
      const int a = (int)(e / m), b = (int)(e % m);
      if (dS) dS[v * nm + e] = edge ? fma(ax[pi * n + a], u[v * m + b], x[pi * n + a] * au[v * m + b]) : 0.0;
      continue;
    }
    e -= nm;
    {
      const int a = (int)(e / m), b = (int)(e % m);
      if (dB) dB[v * nm + e] = edge ? fma(ay[v * n + a], u[v * m + b], y[v * n + a] * au[v * m + b]) : 0.0;
    }
  }
}

int adjoint(PlanObj &P, const rcr_problem &in, const rcr_solution &fwd, const double *gx, const double *gu,
            const double *gy, const rcr_gradient &g, const rcr_solve_options &opt, hipStream_t st) {
  // a = the solve of the seeds (the KKT matrix is symmetric), written to dq, dr, dc
  const RhsIO io{gx, gu, gy, g.q, g.r, g.c};
  int rc = solve_rhs(P, in, fwd.K, fwd.P, 1, &io, opt, st);
  if (rc) return rc;
  if (!(g.Q || g.Delta || g.R || g.S || g.A || g.B)) return RCR_OK;
  std::lock_guard<std::mutex> lock(P.mu);
  const PlanHost &h = P.host;
  const int64_t per = 3 * (int64_t)h.n * h.n + (int64_t)h.m * h.m + 2 * (int64_t)h.n * h.m;
  hipLaunchKernelGGL(k_adjoint_grads, dim3(grid_for(h.N * per)), dim3(256), 0, st, h.N, h.n, h.m, P.dev.parent,
                     fwd.x, fwd.u, fwd.lam, io.x, io.u, io.lam, g.Q, g.Delta, g.R, g.S, g.A, g.B);
  HIPCK(hipGetLastError());
  HIPCK(hipEventRecord(P.last_done, st));
  if (opt.check || opt.kkt_residual) HIPCK(hipStreamSynchronize(st));
  return RCR_OK;
}

// Max-abs KKT residual of eq. (kkt) for a given iterate (float64, synchronises).
int kkt_residual(PlanObj &P, const rcr_problem &in, const rcr_solution &sol, const rcr_solve_options &opt,
                 hipStream_t st) {
  std::lock_guard<std::mutex> lock(P.mu);
  int rc = plan_upload(P, st);
  if (rc) return rc;
  void *ws = opt.workspace;
  if (ws) {
    if ((size_t)opt.workspace_bytes < WS_HEADER_BYTES) return RCR_SMALL_WORKSPACE;
  } else {
    if (!P.resid_buf && dev_alloc((void **)&P.resid_buf, WS_HEADER_BYTES, st) != hipSuccess) return RCR_OOM;
    ws = P.resid_buf;
  }
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, ws_status(ws), ws_resid(ws));
  launch_residual_rhs<double>(P, in, sol, nullptr, nullptr, nullptr, ws_resid(ws), st);
  HIPCK(hipGetLastError());
  if (!P.last_done) HIPCK(hipEventCreateWithFlags(&P.last_done, hipEventDisableTiming));
  HIPCK(hipEventRecord(P.last_done, st));
  double resid = 0.0;
  HIPCK(hipMemcpyAsync(&resid, ws_resid(ws), sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  *opt.kkt_residual = resid;
  return RCR_OK;
}

// ------------------------------------------------------------ batched solve
// rcr_batch_solve: k trees, each with its own problem and solution buffers,
// solved with the merged plan of their forest.  The trees' inputs are gathered
// into contiguous staging arrays in the workspace (tree t at its node offset),
// the merged launch sequence runs on them, and the outputs are scattered back;
// the gather and the scatter are one launch each, driven by a table of copy
// chunks that is uploaded with the call.
namespace {
constexpr int BATCH_IN = 9, BATCH_OUT = 5;
constexpr int64_t COPY_CHUNK = 32768;  // words per copy chunk (one workgroup each)

struct CopyChunk {
  const double *src;
  double *dst;
  int64_t words;
  int64_t pad;
};

// Words per node of each staged field: Q q c Delta R S r A B, then K P x u lam.
void batch_words(int n, int m, int64_t w[BATCH_IN + BATCH_OUT]) {
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  const int64_t v[BATCH_IN + BATCH_OUT] = {nn, n, n, nn, mm, nm, m, nn, nm, nm, nn, n, m, n};
  for (int f = 0; f < BATCH_IN + BATCH_OUT; ++f) w[f] = v[f];
}

// Copy chunks of one direction over all trees and fields.
int64_t batch_chunks(const PlanHost &B, int f0, int f1) {
  int64_t w[BATCH_IN + BATCH_OUT];
  batch_words(B.n, B.m, w);
  const int64_t T = (int64_t)B.tree_off.size() - 1;
  int64_t c = 0;
  for (int f = f0; f < f1; ++f)
    for (int64_t t = 0; t < T; ++t) c += (w[f] * (B.tree_off[t + 1] - B.tree_off[t]) + COPY_CHUNK - 1) / COPY_CHUNK;
  return c;
}

struct BatchLayout {
  size_t stage[BATCH_IN + BATCH_OUT];  // byte offsets of the staged fields
  size_t table;                        // byte offset of the chunk table (gather, then scatter)
  int64_t n_gather, n_scatter;
  size_t total;
};

BatchLayout batch_layout(const PlanHost &B, int precision) {
  BatchLayout L;
  size_t cur = workspace_layout(B, precision).total_bytes;
  int64_t w[BATCH_IN + BATCH_OUT];
  batch_words(B.n, B.m, w);
  for (int f = 0; f < BATCH_IN + BATCH_OUT; ++f) {
    L.stage[f] = cur;
    cur = align_up(cur + (size_t)w[f] * (size_t)B.N * sizeof(double), 256);
  }
  L.n_gather = batch_chunks(B, 0, BATCH_IN);
  L.n_scatter = batch_chunks(B, BATCH_IN, BATCH_IN + BATCH_OUT);
  L.table = cur;
  cur = align_up(cur + (size_t)(L.n_gather + L.n_scatter) * sizeof(CopyChunk), 256);
  L.total = cur;
  return L;
}

__global__ __launch_bounds__(256) void k_copy_chunks(const CopyChunk *__restrict__ ch, int64_t nch) {
  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const CopyChunk k = ch[c];
    for (int64_t i = threadIdx.x; i < k.words; i += 4 * 256) {
      double a[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t q = i + j * 256;
        a[j] = q < k.words ? k.src[q] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t q = i + j * 256;
        if (q < k.words) k.dst[q] = a[j];
      }
    }
  }
}

// Pinned host buffers for the chunk tables, reused once the copy that read
// them has completed (their event); the list grows to the number of tables in
// flight and is never freed.
struct PinSlot {
  char *buf = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
std::mutex pin_mu;
std::vector<PinSlot> &pin_free() {
  static std::vector<PinSlot> *v = new std::vector<PinSlot>();
  return *v;
}
int pin_take(size_t need, PinSlot &out) {
  {
    std::lock_guard<std::mutex> lock(pin_mu);
    auto &fl = pin_free();
    for (size_t i = 0; i < fl.size(); ++i)
      if (fl[i].bytes >= need && hipEventQuery(fl[i].done) == hipSuccess) {
        out = fl[i];
        fl.erase(fl.begin() + (long)i);
        return RCR_OK;
      }
  }
  PinSlot s;
  s.bytes = std::max<size_t>(need, size_t(1) << 20);
  if (hipHostMalloc((void **)&s.buf, s.bytes, hipHostMallocDefault) != hipSuccess) return RCR_OOM;
  if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return RCR_HIP_ERROR;
  out = s;
  return RCR_OK;
}
void pin_give(const PinSlot &s, hipStream_t st) {
  (void)hipEventRecord(s.done, st);
  std::lock_guard<std::mutex> lock(pin_mu);
  pin_free().push_back(s);
}
}  // namespace

size_t batch_workspace_bytes(const PlanHost &B, int precision) { return batch_layout(B, precision).total; }

int batch_solve(PlanObj &Bp, int32_t k, const rcr_problem *in, rcr_solution *out, const rcr_solve_options &opt,
                hipStream_t st) {
  const PlanHost &h = Bp.host;
  const int64_t T = h.tree_off.empty() ? 1 : (int64_t)h.tree_off.size() - 1;
  if (k != T || h.tree_off.empty()) return RCR_BAD_OPTION;
  const int prec = opt.precision;
  const BatchLayout BL = batch_layout(h, prec);
  const size_t solver = workspace_layout(h, prec).total_bytes;
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(Bp.mu);
    int rc = plan_upload(Bp, st);
    if (rc) return rc;
    if ((rc = take_workspace(Bp, opt, BL.total, BL.total, st, ws))) return rc;
  }
  char *wsb = static_cast<char *>(ws);
  double *stg[BATCH_IN + BATCH_OUT];
  for (int f = 0; f < BATCH_IN + BATCH_OUT; ++f) stg[f] = reinterpret_cast<double *>(wsb + BL.stage[f]);
  int64_t w[BATCH_IN + BATCH_OUT];
  batch_words(h.n, h.m, w);
  const int64_t nch = BL.n_gather + BL.n_scatter;
  PinSlot pin;
  int rc = pin_take((size_t)nch * sizeof(CopyChunk), pin);
  if (rc) return rc;
  CopyChunk *tab = reinterpret_cast<CopyChunk *>(pin.buf);
  int64_t c = 0;
  for (int f = 0; f < BATCH_IN + BATCH_OUT; ++f)
    for (int64_t t = 0; t < T; ++t) {
      const int64_t off = h.tree_off[t], words = w[f] * (h.tree_off[t + 1] - off);
      double *tree_buf;
      switch (f) {
        case 0: tree_buf = const_cast<double *>(in[t].Q); break;
        case 1: tree_buf = const_cast<double *>(in[t].q); break;
        case 2: tree_buf = const_cast<double *>(in[t].c); break;
        case 3: tree_buf = const_cast<double *>(in[t].Delta); break;
        case 4: tree_buf = const_cast<double *>(in[t].R); break;
        case 5: tree_buf = const_cast<double *>(in[t].S); break;
        case 6: tree_buf = const_cast<double *>(in[t].r); break;
        case 7: tree_buf = const_cast<double *>(in[t].A); break;
        case 8: tree_buf = const_cast<double *>(in[t].B); break;
        case 9: tree_buf = out[t].K; break;
        case 10: tree_buf = out[t].P; break;
        case 11: tree_buf = out[t].x; break;
        case 12: tree_buf = out[t].u; break;
        default: tree_buf = out[t].lam; break;
      }
      double *staged = stg[f] + off * w[f];
      for (int64_t q = 0; q < words; q += COPY_CHUNK) {
        const int64_t len = std::min<int64_t>(COPY_CHUNK, words - q);
        tab[c++] = f < BATCH_IN ? CopyChunk{tree_buf + q, staged + q, len, 0} : CopyChunk{staged + q, tree_buf + q, len, 0};
      }
    }
  CopyChunk *dtab = reinterpret_cast<CopyChunk *>(wsb + BL.table);
  const hipError_t ce = hipMemcpyAsync(dtab, tab, (size_t)nch * sizeof(CopyChunk), hipMemcpyHostToDevice, st);
  pin_give(pin, st);
  HIPCK(ce);
  auto grid = [](int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 65535))); };
  hipLaunchKernelGGL(k_copy_chunks, grid(BL.n_gather), dim3(256), 0, st, dtab, BL.n_gather);
  HIPCK(hipGetLastError());
  const rcr_problem sin{stg[0], stg[1], stg[2], stg[3], stg[4], stg[5], stg[6], stg[7], stg[8]};
  rcr_solution sout{stg[9], stg[10], stg[11], stg[12], stg[13]};
  rcr_solve_options o = opt;
  o.workspace = ws;
  o.workspace_bytes = (int64_t)solver;
  rc = solve(Bp, sin, sout, o, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_copy_chunks, grid(BL.n_scatter), dim3(256), 0, st, dtab + BL.n_gather, BL.n_scatter);
  HIPCK(hipGetLastError());
  std::lock_guard<std::mutex> lock(Bp.mu);
  HIPCK(hipEventRecord(Bp.last_done, st));
  return RCR_OK;
}


// ------------------------------------------------------ no-allocation solve
// rcr_solve_noalloc: rcr_solve on a workspace that is a static device array
// (one per GPU, NOALLOC_SCRATCH_BYTES, held until the process ends), for
// callers that cannot allocate.  Its address is looked up once per device with
// that device current; the host-side name of the array is never handed to a
// kernel or a copy.  Every call on a GPU shares that GPU's array: overlapping
// calls race, and each call starts by clearing its status words and residual
// accumulator with a fill kernel (no other part of the workspace needs to start
// at zero).  Nothing here allocates: the plan's device copy and completion
// event must exist (rcr_plan_upload), only the per-level executor is allowed
// (capturing a graph allocates) and no timing events are made.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static int scratch_address(int dev, void *&ptr) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return RCR_NO_DEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fprintf(stderr, "rcr: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev, hipGetErrorString(e));
      return RCR_HIP_ERROR;
    }
    scratch_ptr[dev] = p;
  }
  ptr = scratch_ptr[dev];
  return RCR_OK;
}

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

int solve_noalloc(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
                  hipStream_t st) {
  if (opt.executor != RCR_EXEC_LEVELS || opt.kernel_ms || opt.kernel_launches || opt.workspace) return RCR_BAD_OPTION;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lock(P.mu);
    if (!P.dev.base || !P.last_done || P.dev.device != dev) return RCR_BAD_OPTION;  // rcr_plan_upload first
  }
  if (workspace_layout(P.host, opt.precision).total_bytes > NOALLOC_SCRATCH_BYTES) return RCR_SMALL_WORKSPACE;
  void *ptr = nullptr;
  const int rc = scratch_address(dev, ptr);
  if (rc) return rc;
  rcr_solve_options o = opt;
  o.workspace = ptr;
  o.workspace_bytes = (int64_t)NOALLOC_SCRATCH_BYTES;
  return solve(P, in, out, o, st);
}

// ------------------------------------------------------------ autotuning
// Time every candidate launch mapping with HIP events on `st` and keep the
// fastest (the per-level executor is used, so no graph is captured).
int tune(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt, hipStream_t st,
         LaunchCfg &best, float &best_ms) {
  rcr_solve_options o = opt;
  o.executor = RCR_EXEC_LEVELS;
  o.check = 0;
  o.kkt_residual = nullptr;
  o.kernel_ms = nullptr;
  o.kernel_launches = nullptr;
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  const LaunchCfg keep = P.cfg;
  best_ms = -1.f;
  int rc = RCR_OK;
  auto trial = [&](const LaunchCfg &c) {
    {
      std::lock_guard<std::mutex> lock(P.mu);
      P.cfg = c;
    }
    if ((rc = solve(P, in, out, o, st))) return;  // warm-up
    float ms = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess) rc = RCR_HIP_ERROR;
    for (int k = 0; k < 3 && !rc; ++k) rc = solve(P, in, out, o, st);
    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = RCR_HIP_ERROR;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = RCR_HIP_ERROR;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = RCR_HIP_ERROR;
    if (rc) return;
    ms /= 3.f;
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  };
  // The quadratic mapping only changes the factor's launches and the vector
  // mapping only the solve's, so they are tuned one after the other: first
  // the quadratic tail (off or 1, 2, 4, 8 rounds), then, with the best of
  // those, the vector tails (off, or 2, 4, 8 rounds of 8 or 16 wavefronts).
  LaunchCfg c = keep;
  for (int qr : {-1, 1, 2, 4, 8}) {
    if (rc) break;
    c.quad_tail_rounds = qr;
    trial(c);
  }
  if (!rc) c = best;
  if (!rc) {
    c.vec_tail_rounds = -1;
    trial(c);
  }
  for (int vr : {2, 4, 8})
    for (int vw : {8, 16}) {
      if (rc) break;
      c.vec_tail_rounds = vr;
      c.vec_tail_waves = vw;
      trial(c);
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lock(P.mu);
  P.cfg = rc ? keep : best;
  drop_graphs(P);
  return rc;
}

// ------------------------------------------------------------ exact lifting
struct LiftedPtrs {
  double *Q, *q, *c, *De, *R, *S, *r, *A, *B;
};

// Lifted data of a node-control problem (Prop. 2), one wavefront per lifted
// node v: v < N is the predecision node of native node v, v >= N the decision
// node of native node parent'(v).
//   predecision node i^-:  Q' = diag(Q_i, 0), q' = (q_i, 0), c' = (c_i, 0),
//     Delta' = diag(Delta_i, 0); its edge from pa(i)^+ is the uncertainty
//     edge of eq. (uncertainty-edge): A' = [[A_i, B_i], [0, 0]], B' = 0,
//     dummy control cost R' = I, S' = 0, r' = 0 (inert at the root: A' = 0)
//   decision node i^+:  zero costs and offsets; its edge from i^- is the
//     decision edge of eq. (decision-edge): A' = [[I, 0], [0, 0]], B' = [0; I],
//     R' = R_i, S' = [M_i; 0], r' = r_i
__global__ __launch_bounds__(256) void k_lift(int64_t N, int64_t NL, int n, int m, const int32_t *__restrict__ lparent,
                                              rcr_native_problem in, LiftedPtrs o) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= NL) return;
  const int d = n + m;
  const bool pre = v < N;
  const int64_t i = pre ? v : (int64_t)lparent[v];
  const bool unc = pre && lparent[v] >= 0;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  const int64_t dd = (int64_t)d * d, dm = (int64_t)d * m;
  for (int e = lane; e < d * d; e += 64) {
    const int a = e / d, b = e % d;
    const bool xx = pre && a < n && b < n;
    o.Q[v * dd + e] = xx ? in.Q[i * nn + a * n + b] : 0.0;
    o.De[v * dd + e] = xx ? in.Delta[i * nn + a * n + b] : 0.0;
    double av = 0.0;
    if (unc && a < n) av = b < n ? in.A[i * nn + a * n + b] : in.B[i * nm + a * m + (b - n)];
    if (!pre && a == b && a < n) av = 1.0;
    o.A[v * dd + e] = av;
  }
  for (int e = lane; e < d; e += 64) {
    o.q[v * d + e] = (pre && e < n) ? in.q[i * n + e] : 0.0;
    o.c[v * d + e] = (pre && e < n) ? in.c[i * n + e] : 0.0;
  }
  for (int e = lane; e < m * m; e += 64) o.R[v * mm + e] = pre ? ((e / m == e % m) ? 1.0 : 0.0) : in.R[i * mm + e];
  for (int e = lane; e < d * m; e += 64) {
    const int a = e / m, b = e % m;
    o.S[v * dm + e] = (!pre && a < n) ? in.M[i * nm + a * m + b] : 0.0;
    o.B[v * dm + e] = (!pre && a >= n && a - n == b) ? 1.0 : 0.0;
  }
  for (int e = lane; e < m; e += 64) o.r[v * m + e] = pre ? 0.0 : in.r[i * m + e];
}

// Native solution from the lifted one: x_i, lam_i = the first n entries of the
// lifted state and multiplier of i^-, v_i = the control of the decision edge
// into i^+ (zero at leaves).
__global__ __launch_bounds__(256) void k_project(int64_t N, int n, int m, const int32_t *__restrict__ plus,
                                                 const double *__restrict__ xl, const double *__restrict__ ul,
                                                 const double *__restrict__ yl, double *x, double *vv, double *lam) {
  const int d = n + m;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * n; t += stride) {
    const int64_t i = t / n;
    const int a = (int)(t % n);
    x[t] = xl[i * d + a];
    lam[t] = yl[i * d + a];
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * m; t += stride) {
    const int64_t i = t / m;
    const int b = (int)(t % m);
    const int32_t k = plus[i];
    vv[t] = k >= 0 ? ul[(int64_t)k * m + b] : 0.0;
  }
}

// The uniform float64 problem and solution that lifted and ragged plans stage
// after the solver's workspace (9 problem arrays, then 5 solution arrays).
static void staged_ptrs(const PlanHost &h, void *ws, int prec, double *ptr[14]) {
  size_t iw[9], ow[5];
  lift_words(h.n, h.m, iw, ow);
  size_t cur = workspace_layout(h, prec).total_bytes;
  for (int k = 0; k < 14; ++k) {
    ptr[k] = reinterpret_cast<double *>(static_cast<char *>(ws) + cur);
    cur = align_up(cur + (k < 9 ? iw[k] : ow[k - 9]) * 8 * (size_t)h.N, 256);
  }
}

// Ragged problems (node v of state dimension nv = rg_n[v], the edge into it of
// control dimension mv = rg_m[v], the parent's dimension np) padded to the
// uniform n, m: every block sits in the top-left corner of its padded block,
// zeros elsewhere, except the control cost, padded with the identity.  The
// padded coordinates decouple (their rows of the dynamics give x = 0, of the
// stationarities y = 0 and u = 0) and the standing assumptions still hold, so
// the padded solution restricted to the real coordinates is the solution,
// and P, K are the padded ones' top-left blocks.  One wavefront per node.
// Offsets off[f * (N + 1) + v] locate v's block of field f in the packed arrays.
__global__ __launch_bounds__(256) void k_ragged_pack(int64_t N, int n, int m, const int32_t *__restrict__ parent,
                                                     const int32_t *__restrict__ rn, const int32_t *__restrict__ rm,
                                                     const int64_t *__restrict__ off, rcr_problem in, LiftedPtrs o) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= N) return;
  const int64_t N1 = N + 1;
  const int nv = rn[v], mv = rm[v], pv = parent[v], np = pv >= 0 ? rn[pv] : 0;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  for (int e = lane; e < n * n; e += 64) {
    const int a = e / n, b = e % n;
    const bool xx = a < nv && b < nv;
    o.Q[v * nn + e] = xx ? in.Q[off[0 * N1 + v] + a * nv + b] : 0.0;
    o.De[v * nn + e] = xx ? in.Delta[off[3 * N1 + v] + a * nv + b] : 0.0;
    o.A[v * nn + e] = (a < nv && b < np) ? in.A[off[7 * N1 + v] + a * np + b] : 0.0;
  }
  for (int e = lane; e < n; e += 64) {
    o.q[v * n + e] = e < nv ? in.q[off[1 * N1 + v] + e] : 0.0;
    o.c[v * n + e] = e < nv ? in.c[off[2 * N1 + v] + e] : 0.0;
  }
  for (int e = lane; e < m * m; e += 64) {
    const int a = e / m, b = e % m;
    o.R[v * mm + e] = (a < mv && b < mv) ? in.R[off[4 * N1 + v] + a * mv + b] : (a == b ? 1.0 : 0.0);
  }
  for (int e = lane; e < n * m; e += 64) {
    const int a = e / m, b = e % m;
    o.S[v * nm + e] = (a < np && b < mv) ? in.S[off[5 * N1 + v] + a * mv + b] : 0.0;
    o.B[v * nm + e] = (a < nv && b < mv) ? in.B[off[8 * N1 + v] + a * mv + b] : 0.0;
  }
  for (int e = lane; e < m; e += 64) o.r[v * m + e] = e < mv ? in.r[off[6 * N1 + v] + e] : 0.0;
}

// The real blocks of the padded solution into the caller's packed arrays.
__global__ __launch_bounds__(256) void k_ragged_unpack(int64_t N, int n, int m, const int32_t *__restrict__ parent,
                                                       const int32_t *__restrict__ rn, const int32_t *__restrict__ rm,
                                                       const int64_t *__restrict__ off, rcr_solution po,
                                                       rcr_solution out) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= N) return;
  const int64_t N1 = N + 1;
  const int nv = rn[v], mv = rm[v], pv = parent[v], np = pv >= 0 ? rn[pv] : 0;
  for (int e = lane; e < nv * nv; e += 64) out.P[off[10 * N1 + v] + e] = po.P[v * n * n + (e / nv) * n + e % nv];
  for (int e = lane; e < mv * np; e += 64) out.K[off[9 * N1 + v] + e] = po.K[v * m * n + (e / np) * n + e % np];
  for (int e = lane; e < nv; e += 64) {
    out.x[off[11 * N1 + v] + e] = po.x[v * n + e];
    out.lam[off[13 * N1 + v] + e] = po.lam[v * n + e];
  }
  for (int e = lane; e < mv; e += 64) out.u[off[12 * N1 + v] + e] = po.u[v * m + e];
}

int ragged_solve(PlanObj &P, const rcr_problem &in, rcr_solution &out, const rcr_solve_options &opt,
                 hipStream_t st) {
  const PlanHost &h = P.host;
  if (h.rg_n.empty()) return RCR_BAD_OPTION;
  const int prec = opt.precision;
  void *ws = opt.workspace;
  const size_t need = total_workspace_bytes(h, prec);
  {
    std::lock_guard<std::mutex> lock(P.mu);
    int rc = plan_upload(P, st);
    if (rc) return rc;
    if ((rc = take_workspace(P, opt, need, need, st, ws))) return rc;
  }
  double *ptr[14];
  staged_ptrs(h, ws, prec, ptr);
  const LiftedPtrs lp{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], ptr[7], ptr[8]};
  const dim3 g((unsigned)((h.N + 3) / 4)), b(256);
  hipLaunchKernelGGL(k_ragged_pack, g, b, 0, st, h.N, h.n, h.m, P.dev.parent, P.dev.rg_n, P.dev.rg_m, P.dev.rg_off,
                     in, lp);
  HIPCK(hipGetLastError());
  const rcr_problem pin{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], ptr[7], ptr[8]};
  rcr_solution pout{ptr[9], ptr[10], ptr[11], ptr[12], ptr[13]};
  rcr_solve_options o2 = opt;
  o2.workspace = ws;
  o2.workspace_bytes = (int64_t)workspace_layout(h, prec).total_bytes;
  int rc = solve(P, pin, pout, o2, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_ragged_unpack, g, b, 0, st, h.N, h.n, h.m, P.dev.parent, P.dev.rg_n, P.dev.rg_m,
                     P.dev.rg_off, pout, out);
  HIPCK(hipGetLastError());
  std::lock_guard<std::mutex> lock(P.mu);
  HIPCK(hipEventRecord(P.last_done, st));
  return RCR_OK;
}

int lift_solve(PlanObj &P, const rcr_native_problem &in, rcr_native_solution &out, const rcr_solve_options &opt,
               hipStream_t st) {
  const PlanHost &h = P.host;
  if (!h.lift_N) return RCR_BAD_OPTION;
  const int prec = opt.precision;
  void *ws = opt.workspace;
  const size_t need = total_workspace_bytes(h, prec);
  {
    std::lock_guard<std::mutex> lock(P.mu);
    int rc = plan_upload(P, st);
    if (rc) return rc;
    if (ws) {
      if ((size_t)opt.workspace_bytes < need) return RCR_SMALL_WORKSPACE;
    } else {
      if (!P.ws[prec]) {
        if (dev_alloc(&P.ws[prec], need, st) != hipSuccess) return RCR_OOM;
        P.ws_bytes[prec] = need;
      }
      ws = P.ws[prec];
    }
  }
  const size_t solver_bytes = workspace_layout(h, prec).total_bytes;
  size_t iw[9], ow[5];
  lift_words(h.n, h.m, iw, ow);
  double *ptr[14];
  size_t cur = solver_bytes;
  for (int k = 0; k < 14; ++k) {
    ptr[k] = reinterpret_cast<double *>(static_cast<char *>(ws) + cur);
    cur = align_up(cur + (k < 9 ? iw[k] : ow[k - 9]) * 8 * (size_t)h.N, 256);
  }
  const LiftedPtrs lp{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], ptr[7], ptr[8]};
  const int64_t NL = h.N, N = h.lift_N;
  const int n = h.lift_n, m = h.m;
  hipLaunchKernelGGL(k_lift, dim3((unsigned)((NL + 3) / 4)), dim3(256), 0, st, N, NL, n, m, P.dev.parent, in, lp);
  HIPCK(hipGetLastError());
  rcr_problem lin{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], ptr[7], ptr[8]};
  rcr_solution lout{ptr[9], ptr[10], ptr[11], ptr[12], ptr[13]};
  rcr_solve_options o2 = opt;
  o2.workspace = ws;
  o2.workspace_bytes = (int64_t)solver_bytes;
  int rc = solve(P, lin, lout, o2, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_project, dim3(grid_for(N * std::max(n, m))), dim3(256), 0, st, N, n, m, P.dev.lift_plus,
                     lout.x, lout.u, lout.lam, out.x, out.v, out.lam);
  HIPCK(hipGetLastError());
  std::lock_guard<std::mutex> lock(P.mu);
  HIPCK(hipEventRecord(P.last_done, st));
  return RCR_OK;
}

}  // namespace rcr
