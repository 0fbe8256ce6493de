// Device-side planner: the program of dplan.hpp on one workgroup of 1024
// threads (16 wavefronts of one CU), so planning a new topology occupies one CU
// while solves run on the others, and the plan's schedules come back to the
// host in two copies.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "device.hpp"
#include "dplan.hpp"

namespace rcr {
namespace dplan {
namespace {

// Every thread of the workgroup runs the program; each() is one phase.
struct GpuExec {
  template <class F>
  __device__ void each(F f) {
    f((int)threadIdx.x);
    __syncthreads();
  }
  template <class F>
  __device__ bool any(F f) {
    return __syncthreads_or(f((int)threadIdx.x) ? 1 : 0) != 0;
  }
  template <class F>
  __device__ int32_t maxall(F f) {
    __shared__ int32_t m;
    const int32_t v = f((int)threadIdx.x);
    if (threadIdx.x == 0) m = INT_MIN;
    __syncthreads();
    atomicMax(&m, v);
    __syncthreads();
    const int32_t r = m;
    __syncthreads();
    return r;
  }
  // Exclusive scan of a[0 .. THREADS) in place (a wavefront scan by lane
  // shuffles, then the 16 wavefront totals); returns the total.
  __device__ uint32_t scan(uint32_t *a) {
    __shared__ uint32_t wsum[THREADS / 64];
    __shared__ uint32_t tot;
    const int t = (int)threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t v = a[t];
    uint32_t s = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(s, (unsigned)o);
      if (lane >= o) s += y;
    }
    if (lane == 63) wsum[w] = s;
    __syncthreads();
    if (t == 0) {
      uint32_t acc = 0;
      for (int i = 0; i < THREADS / 64; ++i) {
        const uint32_t c = wsum[i];
        wsum[i] = acc;
        acc += c;
      }
      tot = acc;
    }
    __syncthreads();
    a[t] = s - v + wsum[w];
    const uint32_t r = tot;
    __syncthreads();
    return r;
  }
  // scan() for 64-bit values.
  __device__ uint64_t scan64(uint64_t *a) {
    __shared__ uint64_t wsum[THREADS / 64];
    __shared__ uint64_t tot;
    const int t = (int)threadIdx.x, lane = t & 63, w = t >> 6;
    const uint64_t v = a[t];
    uint64_t s = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(s, (unsigned)o);
      if (lane >= o) s += y;
    }
    if (lane == 63) wsum[w] = s;
    __syncthreads();
    if (t == 0) {
      uint64_t acc = 0;
      for (int i = 0; i < THREADS / 64; ++i) {
        const uint64_t c = wsum[i];
        wsum[i] = acc;
        acc += c;
      }
      tot = acc;
    }
    __syncthreads();
    a[t] = s - v + wsum[w];
    const uint64_t r = tot;
    __syncthreads();
    return r;
  }
  __device__ void atomic_add(int32_t *p, int32_t v) { atomicAdd(p, v); }

  // Wavefront w takes a contiguous range of the indices in steps of 64 (lane l
  // the step's l-th index, so loads are coalesced) and ranks its lanes by
  // ballot; U steps are loaded before any is ranked.
  static constexpr int NW = THREADS / 64, U = 4;
  __device__ static void wave_range(int64_t n, int64_t &b, int64_t &e) {
    const int64_t steps = (n + 63) >> 6, per = (steps + NW - 1) / NW;
    b = (int64_t)(threadIdx.x >> 6) * per * 64;
    e = b + per * 64 < n ? b + per * 64 : n;
  }

  template <class P, class W>
  __device__ uint32_t compact(const Arena &, int64_t n, P pred, W write) {
    __shared__ uint32_t woff[NW + 1];
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const uint64_t lt = __lanemask_lt();
    int64_t b, e;
    wave_range(n, b, e);
    uint32_t c = 0;
    for (int64_t i0 = b; i0 < e; i0 += 64 * U) {
      bool f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 64 * u + lane;
        f[u] = i < e && pred(i);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) c += (uint32_t)__popcll(__ballot(f[u]));
    }
    if (lane == 0) woff[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t s = 0;
      for (int k = 0; k < NW; ++k) {
        const uint32_t v = woff[k];
        woff[k] = s;
        s += v;
      }
      woff[NW] = s;
    }
    __syncthreads();
    uint32_t o = woff[w];
    for (int64_t i0 = b; i0 < e; i0 += 64 * U) {
      bool f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 64 * u + lane;
        f[u] = i < e && pred(i);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t m = __ballot(f[u]);
        if (f[u]) write(i0 + 64 * u + lane, o + (uint32_t)__popcll(m & lt));
        o += (uint32_t)__popcll(m);
      }
    }
    const uint32_t total = woff[NW];
    __syncthreads();
    return total;
  }

  // One stable pass on digit (k >> sh) & 15: per-wavefront digit counts, a
  // digit-major scan, then each step's lanes ranked among the lanes of the same
  // digit (four ballots) and the group's offset advanced by its lowest lane.
  __device__ void radix_pass(const Arena &, int64_t n, int sh, const uint32_t *kk, const uint32_t *vv, uint32_t *kd,
                             uint32_t *vd) {
    __shared__ uint32_t off[16 * NW];  // [digit][wavefront]
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const uint64_t lt = __lanemask_lt();
    if (threadIdx.x < 16 * NW) off[threadIdx.x] = 0;
    __syncthreads();
    int64_t b, e;
    wave_range(n, b, e);
    for (int64_t i0 = b; i0 < e; i0 += 64 * U) {
      uint32_t dg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 64 * u + lane;
        dg[u] = i < e ? (kk[i] >> sh) & 15 : 16;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (dg[u] < 16) atomicAdd(&off[dg[u] * NW + w], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t s = 0;
      for (int k = 0; k < 16 * NW; ++k) {
        const uint32_t v = off[k];
        off[k] = s;
        s += v;
      }
    }
    __syncthreads();
    for (int64_t i0 = b; i0 < e; i0 += 64 * U) {
      uint32_t kb[U], vb[U];
      bool act[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + 64 * u + lane;
        act[u] = i < e;
        kb[u] = act[u] ? kk[i] : 0;
        vb[u] = act[u] ? vv[i] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t d = (kb[u] >> sh) & 15;
        uint64_t peers = __ballot(act[u]);
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
          const bool one = (d >> bit) & 1;
          const uint64_t bb = __ballot(act[u] && one);
          peers &= one ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        uint32_t base = 0;
        if (act[u]) base = off[d * NW + w];
        if (act[u]) {
          kd[base + rank] = kb[u];
          vd[base + rank] = vb[u];
        }
        if (act[u] && rank == 0) off[d * NW + w] = base + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
  }
};

__global__ void __launch_bounds__(THREADS) k_device_plan(Arena a) {
  GpuExec x;
  const int32_t rc = program(x, a);
  if (threadIdx.x == 0) a.stats[S_STATUS] = rc;
}

}  // namespace
}  // namespace dplan

int device_plan(const int64_t *parent, int64_t N, int n, int m, hipStream_t st, PlanHost &P) {
  using namespace dplan;
  if (!parent) return RCR_NULL_ARG;
  if (N < 1 || n < 1 || m < 1 || n > RCR_MAX_DIM || m > RCR_MAX_DIM) return RCR_BAD_DIMS;
  if (N > (int64_t)(INT32_MAX / 2 - 16)) return RCR_BAD_DIMS;
  Arena a;
  const size_t bytes = carve(a, nullptr, N, THREADS);
  char *base = nullptr;
  if (dev_alloc((void **)&base, bytes, st) != hipSuccess) return RCR_OOM;
  carve(a, base, N, THREADS);
  a.parent = parent;
  hipLaunchKernelGGL(k_device_plan, dim3(1), dim3(THREADS), 0, st, a);
  hipError_t e = hipGetLastError();
  HostOut h;
  if (e == hipSuccess) e = hipMemcpyAsync(h.stats, a.stats, sizeof(h.stats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int rc = e == hipSuccess ? (int)h.stats[S_STATUS] : RCR_HIP_ERROR;
  if (rc == 0) {
    const OutSizes z = out_sizes(h.stats);
    h.par32.resize((size_t)N);
    h.ops.resize(z.ops);
    h.lvl_off.resize(z.lvl);
    h.kind_off.resize(z.kind);
    h.exp_ops.resize(z.exp);
    h.exp_off.resize(z.exp_off);
    h.tc_ops.resize(z.tc);
    h.tc_off.resize(z.tc_off);
    h.sx_ops.resize(z.sx);
    h.sx_off.resize(z.sx_off);
    struct Piece {
      void *dst;
      const void *src;
      size_t bytes;
    } pieces[] = {{h.par32.data(), a.par32, h.par32.size() * sizeof(int32_t)},
                  {h.ops.data(), a.ops, h.ops.size() * sizeof(OpRec)},
                  {h.lvl_off.data(), a.lvl_off, h.lvl_off.size() * sizeof(int64_t)},
                  {h.kind_off.data(), a.kind_off, h.kind_off.size() * sizeof(int64_t)},
                  {h.exp_ops.data(), a.exp_ops, h.exp_ops.size() * sizeof(Op4)},
                  {h.exp_off.data(), a.exp_off, h.exp_off.size() * sizeof(int64_t)},
                  {h.tc_ops.data(), a.tc_ops, h.tc_ops.size() * sizeof(Op4)},
                  {h.tc_off.data(), a.tc_off, h.tc_off.size() * sizeof(int64_t)},
                  {h.sx_ops.data(), a.sx_ops, h.sx_ops.size() * sizeof(Op4)},
                  {h.sx_off.data(), a.sx_off, h.sx_off.size() * sizeof(int64_t)}};
    for (const Piece &p : pieces)
      if (e == hipSuccess && p.bytes) e = hipMemcpyAsync(p.dst, p.src, p.bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = RCR_HIP_ERROR;
  }
  (void)hipFreeAsync(base, st);
  if (e != hipSuccess) fprintf(stderr, "rcr: device planner failed: %s\n", hipGetErrorString(e));
  if (rc == 0) fill_plan(h, N, n, m, P);
  return rc;
}

}  // namespace rcr
