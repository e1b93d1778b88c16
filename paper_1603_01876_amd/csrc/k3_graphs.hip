// k3_graphs.hip -- K3 (Sec. IV.D) for many independent small graphs in one
// persistent launch, captured once into a hipGraph and replayed.
//
// Each 1024-thread workgroup takes whole graphs from an atomic queue
// (descriptors uploaded largest first) and runs the full K3 of a graph on
// its own: the initial vector r = rand ./ norm(r,1) (same counter-based
// draws and exact integer sum as pp_init_r), then `iters` damped
// iterations.  r and y live in LDS, so every gather r[u] is an LDS read and
// only the graph's CSR streams from L2/HBM.  Rows are split between threads
// by a merge-path partition of the graph's (row ends, non-zeros), computed
// once per graph; rows cut between threads are completed with a segmented
// scan over the workgroup.  sum(r) is an FP64 block reduction in a fixed
// order.  Workgroups never wait on each other: a workgroup exits when the
// queue is empty.
#include <mutex>
#include <vector>

#include "pp_common.hpp"

#pragma clang fp contract(off)

namespace pp {

namespace {

constexpr int kT = 1024;           // threads per workgroup
constexpr int kW = kT / kWave;     // waves per workgroup

struct AccD {
  double s;
  __device__ __forceinline__ void add(double x) { s += x; }
  __device__ __forceinline__ double value() const { return s; }
};
__device__ __forceinline__ AccD merge(AccD a, AccD b) { return AccD{a.s + b.s}; }
__device__ __forceinline__ AccD shfl_up_acc(AccD a, int o) { return AccD{__shfl_up(a.s, o, kWave)}; }
__device__ __forceinline__ AccD shfl_acc(AccD a, int src) { return AccD{__shfl(a.s, src, kWave)}; }

struct AccF {
  float s, e;
  __device__ __forceinline__ void add(float x) {
    const float t = s + x;
    const float z = t - s;
    const float err = (s - (t - z)) + (x - z);
    s = t;
    e += err;
  }
  __device__ __forceinline__ float value() const { return s + e; }
};
__device__ __forceinline__ AccF merge(AccF a, AccF b) {
  AccF r = a;
  r.add(b.s);
  r.e += b.e;
  return r;
}
__device__ __forceinline__ AccF shfl_up_acc(AccF a, int o) {
  return AccF{__shfl_up(a.s, o, kWave), __shfl_up(a.e, o, kWave)};
}
__device__ __forceinline__ AccF shfl_acc(AccF a, int src) {
  return AccF{__shfl(a.s, src, kWave), __shfl(a.e, src, kWave)};
}

template <typename V>
struct GForm;
template <>
struct GForm<double> {
  using Acc = AccD;
  __device__ static double finish(AccD a, double c, double t) { return c * a.value() + t; }
};
template <>
struct GForm<float> {
  using Acc = AccF;
  __device__ static float finish(AccF a, double c, double t) {
    return float(c * double(a.value()) + t);
  }
};

// Fixed-order sum over the 1024 threads (shuffle tree, then 16 wave sums in
// index order); valid in every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  for (int i = 0; i < kW; ++i) r += sh[i];
  __syncthreads();
  return r;
}

constexpr int kU = 4;                  // merge items per lane per round
constexpr int kRound = kWave * kU;     // merge items per wave round

// Orders a wave's LDS writes before its later reads of other lanes' data
// (a wave's LDS operations complete in issue order; this keeps the
// compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
using GPtr = const T __attribute__((address_space(1))) *;
template <typename T>
using GPtrW = T __attribute__((address_space(1))) *;

// Every descriptor has been checked on the host before the launch (n in
// [1, lds_n], nnz >= 0, the arrays present), so each graph fits the
// workgroup's two LDS vectors.
template <typename V>
__global__ __launch_bounds__(kT) void k_graphs(const pp_graph *__restrict__ graphs, int32_t ngraphs,
                                               int32_t iters, double c, uint32_t *queue,
                                               int32_t lds_n) {
  // queue[0]: index of the next graph to take.
  using Acc = typename GForm<V>::Acc;
  extern __shared__ __align__(16) uint8_t smem[];
  V *xa = reinterpret_cast<V *>(smem);
  V *ya = xa + lds_n;
  __shared__ int32_t s_g;
  __shared__ double s_dred[kW];
  __shared__ unsigned long long s_ured[kW];
  __shared__ int32_t s_re[kW][kRound];   // row ends of each wave's round
  __shared__ Acc s_tail[kW], s_head[kW];
  __shared__ int32_t s_first[kW], s_last[kW], s_hdone[kW];
  __shared__ int32_t s_wi[kW + 1], s_wj[kW + 1];

  const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  for (;;) {
    if (tid == 0) s_g = int32_t(atomicAdd(queue, 1u));
    __syncthreads();
    const int32_t g = s_g;
    __syncthreads();
    if (g >= ngraphs) break;
    const pp_graph G = graphs[g];
    const int32_t n = int32_t(G.n), nnz = int32_t(G.nnz);
    // The descriptor's pointers are generic; these views tell the compiler
    // they are device (global) memory, so their reads are global loads
    // rather than flat ones (which also wait on the LDS counter).
    const GPtr<int32_t> rp = (GPtr<int32_t>)(G.row_ptr);
    const GPtr<int32_t> col = (GPtr<int32_t>)(G.col);
    const GPtr<V> val = (GPtr<V>)(G.val);
    const GPtrW<double> sums = (GPtrW<double>)(G.sums);
    V *x = xa, *y = ya;

    // Initial vector: 24-bit draws, exact integer sum, one division each.
    const uint32_t k0 = uint32_t(G.seed), k1 = uint32_t(G.seed >> 32);
    unsigned long long part = 0;
    for (int32_t i = tid; i < n; i += kT)
      part += philox10(U4{uint32_t(i), 0u, 0u, 2u}, k0, k1).x >> 8;
    const unsigned long long K = block_sum(part, s_ured);
    for (int32_t i = tid; i < n; i += kT) {
      const uint32_t ki = philox10(U4{uint32_t(i), 0u, 0u, 2u}, k0, k1).x >> 8;
      x[i] = V(K ? double(ki) / double(K) : 1.0 / double(n));
    }
    __syncthreads();
    double ps = 0.0;
    for (int32_t i = tid; i < n; i += kT) ps += double(x[i]);
    double s = block_sum(ps, s_dred);
    if (tid == 0 && sums) sums[0] = s;
    const double w = (1.0 - c) / double(n);

    // Each wave takes a contiguous range of the merge sequence (row ends and
    // non-zeros), fixed for all iterations, and walks it in rounds of
    // kRound items: the round's row ends go to LDS (coalesced reads), each
    // lane takes kU consecutive items of the round (a merge-path search in
    // the round's row ends) with its column/value reads adjacent to its
    // neighbours', and a segmented scan across the wave completes the rows
    // that span lanes.  The row left open at the end of a round is carried
    // into the next; rows that span waves are completed after one barrier.
    const int32_t tot = n + nnz;
    const int32_t per = (tot + kW - 1) / kW;
    if (tid <= kW) {
      const int32_t d = tid * per < tot ? tid * per : tot;
      int32_t lo = d - nnz > 0 ? d - nnz : 0, hi = d < n ? d : n;
      while (lo < hi) {
        const int32_t m = (lo + hi) >> 1;
        if (rp[m + 1] <= d - m - 1)
          lo = m + 1;
        else
          hi = m;
      }
      s_wi[tid] = lo;
      s_wj[tid] = d - lo;
    }
    __syncthreads();
    const int32_t wi0 = s_wi[wv], wj0 = s_wj[wv];
    const int32_t dw0 = wi0 + wj0, dw1 = s_wi[wv + 1] + s_wj[wv + 1];
    // The wave starts inside a row that earlier waves began.
    const bool mid = wi0 < n && wj0 > rp[wi0];
    int32_t *re = s_re[wv];

    for (int32_t it = 0; it < iters; ++it) {
      const double tk = w * s;
      double ysum = 0.0;
      int32_t ri = wi0, rj = wj0;   // coordinate (row, non-zero) of the round's start
      Acc carry{};                  // row ri's partial from earlier rounds of this wave
      Acc head{};                   // the wave's part of row wi0 when mid (completed here)
      bool hdone = false;
      for (int32_t d = dw0; d < dw1; d += kRound) {
        const int32_t cnt = dw1 - d < kRound ? dw1 - d : kRound;
        // Row ends of rows ri, ri + 1, ... as non-zero offsets from rj
        // (rows past the graph never end).  Reads unconditional.
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int32_t q = u * kWave + lane;
          const int32_t row = ri + q < n ? ri + q : n - 1;
          const int32_t e = rp[row + 1] - rj;
          re[q] = ri + q < n ? e : INT32_MAX;
        }
        wave_sync();
        // This lane's items [o, o + nit) of the round and its start.
        const int32_t o = lane * kU < cnt ? lane * kU : cnt;
        const int32_t nit = cnt - o < kU ? cnt - o : kU;
        int32_t lo = 0, hi = o;
        while (lo < hi) {
          const int32_t m = (lo + hi) >> 1;
          if (re[m] <= o - m - 1)
            lo = m + 1;
          else
            hi = m;
        }
        int32_t ti = ri + lo, tj = rj + (o - lo);
        int32_t cw[kU];
        V vw[kU];
        if (nnz > 0) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int32_t q = tj + u < nnz ? tj + u : nnz - 1;
            cw[u] = col[q];
            vw[u] = val[q];
          }
        }
        Acc acc{}, first{};
        int32_t first_row = -1;
        int32_t left = nit;
        auto row_end = [&]() {
          if (first_row < 0) {
            first_row = ti;
            first = acc;
          } else {
            const V yv = GForm<V>::finish(acc, c, tk);
            y[ti] = yv;
            ysum += double(yv);
          }
          acc = Acc{};
          ++ti;
          --left;
        };
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          while (left > 0 && re[ti - ri] <= tj - rj) row_end();
          if (left > 0) {
            acc.add(x[cw[u]] * vw[u]);
            ++tj;
            --left;
          }
        }
        while (left > 0 && re[ti - ri] <= tj - rj) row_end();
        // Lane 0 starts in row ri, which earlier rounds may have begun.
        if (lane == 0) {
          if (first_row >= 0)
            first = merge(carry, first);
          else
            acc = merge(carry, acc);
        }
        // Segmented scan of the open rows' partials across the wave.
        const int32_t key = ti;
        Acc v = acc;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
          const Acc vu = shfl_up_acc(v, off);
          const int32_t ku = __shfl_up(key, off, kWave);
          if (lane >= off && ku == key) v = merge(vu, v);
        }
        const Acc pv = shfl_up_acc(v, 1);
        const int32_t pk = __shfl_up(key, 1, kWave);
        if (first_row >= 0) {
          const Acc sum = lane > 0 && pk == first_row ? merge(pv, first) : first;
          if (mid && first_row == wi0) {
            head = sum;   // earlier waves hold the rest of this row
            hdone = true;
          } else {
            const V yv = GForm<V>::finish(sum, c, tk);
            y[first_row] = yv;
            ysum += double(yv);
          }
        }
        carry = shfl_acc(v, kWave - 1);
        ri = __shfl(ti, kWave - 1, kWave);
        rj = __shfl(tj, kWave - 1, kWave);
        wave_sync();   // every lane is done with re before the next round
      }
      // Wave tails and heads; rows that span waves.
      if (hdone) s_head[wv] = head;
      const uint64_t hb = __ballot(hdone);
      if (lane == 0) {
        s_tail[wv] = carry;
        s_first[wv] = wi0;
        s_last[wv] = ri;
        s_hdone[wv] = hb != 0ull;
      }
      __syncthreads();
      if (lane == 0 && s_hdone[wv]) {
        Acc before{};
        for (int q = wv - 1; q >= 0; --q) {
          if (s_last[q] != wi0) break;
          before = merge(s_tail[q], before);
          if (s_first[q] != wi0) break;
        }
        const V yv = GForm<V>::finish(merge(before, s_head[wv]), c, tk);
        y[wi0] = yv;
        ysum += double(yv);
      }
      s = block_sum(ysum, s_dred);   // contains __syncthreads: y complete
      if (tid == 0 && sums) sums[it + 1] = s;
      V *t = x;
      x = y;
      y = t;
    }
    const GPtrW<V> r = (GPtrW<V>)(G.r);
    for (int32_t i = tid; i < n; i += kT) r[i] = x[i];
    __syncthreads();
  }
}

__global__ void k_zero_queue(uint32_t *q) {
  if (threadIdx.x == 0) q[0] = 0u;
}

// Cached hipGraph per launch configuration.  The graph holds two kernel
// nodes (queue reset, persistent kernel) whose arguments point into the
// caller's workspace; the descriptor table is copied there before every
// launch or replay, so a replay reads the batch of the current call.
struct GraphEntry {
  const void *ws;
  hipStream_t stream;
  int32_t ngraphs, iters, lds_n, grid;
  pp_dtype dt;
  double c;
  hipGraphExec_t exec;
};
std::vector<GraphEntry> g_cache;

int lds_limit() {
  static int limit = -1;
  if (limit < 0) {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      limit = v;
    else
      limit = 65536;
  }
  return limit;
}

int cu_count() {
  static int cus = -1;
  if (cus < 0) {
    int dev = 0, v = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cus = v;
    else
      cus = 256;
  }
  return cus;
}

constexpr size_t kStaticLds = 24 * 1024;  // reductions, scan tails, s_pre

}  // namespace

// Scratch of the allocation-free entry point: the queue counter and the
// descriptor table of up to kStaticGraphs graphs, laid out as the workspace
// of launch_graphs (graphs_ws_bytes).  Every GPU holds its own copy for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr int32_t kStaticGraphs = 1 << 16;
constexpr size_t kStaticScratch = 512 + size_t(kStaticGraphs) * sizeof(pp_graph);
static __device__ __align__(256) uint8_t scratch[kStaticScratch];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch, looked up once per device.
pp_status static_scratch(void **out) {
  int dev = -1;
  PP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PP_EHIP, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PP_EHIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PP_OK;
}

}  // namespace

int32_t graphs_static_max() { return kStaticGraphs; }

pp_status launch_graphs_static(int32_t ngraphs, const pp_graph *graphs, int64_t max_n,
                               pp_dtype dt, int32_t iters, double c, hipStream_t s) {
  if (ngraphs < 1 || ngraphs > kStaticGraphs)
    return fail(PP_ERANGE, "pp_pagerank_graphs_noalloc: %d graphs, at most %d", ngraphs,
                kStaticGraphs);
  void *ws = nullptr;
  const pp_status st = static_scratch(&ws);
  if (st != PP_OK) return st;
  // Direct launches only: the kernels take the scratch as their workspace.
  return launch_graphs(ngraphs, graphs, max_n, dt, iters, c, 0, ws, kStaticScratch, s);
}

size_t graphs_ws_bytes(int32_t ngraphs) {
  Carve c(nullptr);
  c.take<uint32_t>(4);
  c.take<pp_graph>(size_t(ngraphs < 1 ? 1 : ngraphs));
  return c.bytes();
}

int64_t graphs_max_n(pp_dtype dt) {
  const size_t vb = dt == PP_F64 ? 8 : 4;
  const int64_t room = int64_t(lds_limit()) - int64_t(kStaticLds);
  return room > 0 ? room / int64_t(2 * vb) / 64 * 64 : 0;
}

pp_status launch_graphs(int32_t ngraphs, const pp_graph *graphs, int64_t max_n, pp_dtype dt,
                        int32_t iters, double c, int32_t use_graph, void *ws, size_t ws_bytes,
                        hipStream_t s) {
  if (ws_bytes < graphs_ws_bytes(ngraphs)) return fail(PP_EWORKSPACE, "graphs workspace too small");
  Carve cv(ws);
  uint32_t *queue = cv.take<uint32_t>(4);
  pp_graph *table = cv.take<pp_graph>(size_t(ngraphs));
  const int32_t lds_n = int32_t((max_n + 63) / 64 * 64);
  const size_t dyn = size_t(2) * lds_n * (dt == PP_F64 ? 8 : 4);
  const int grid = ngraphs < cu_count() ? ngraphs : cu_count();
  // The dynamic LDS limit is raised once per value type to the largest
  // batch any call may run (graphs_max_n), never lowered, so a hipGraph
  // recorded earlier with a larger size stays launchable.
  static bool raised[2] = {false, false};
  const int room = int(size_t(2) * graphs_max_n(dt) * (dt == PP_F64 ? 8 : 4));
  if (!raised[dt == PP_F64 ? 0 : 1]) {
    if (dt == PP_F64)
      PP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graphs<double>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, room));
    else
      PP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graphs<float>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, room));
    raised[dt == PP_F64 ? 0 : 1] = true;
  }
  // The descriptor table (host memory, checked by the caller) goes into the
  // workspace ahead of the launch; graph replays read it from there.
  PP_HIP(hipMemcpyAsync(table, graphs, size_t(ngraphs) * sizeof(pp_graph), hipMemcpyHostToDevice,
                        s));

  auto enqueue = [&](hipStream_t st) -> pp_status {
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, queue);
    if (dt == PP_F64)
      hipLaunchKernelGGL(k_graphs<double>, dim3(grid), dim3(kT), dyn, st, table, ngraphs, iters,
                         c, queue, lds_n);
    else
      hipLaunchKernelGGL(k_graphs<float>, dim3(grid), dim3(kT), dyn, st, table, ngraphs, iters,
                         c, queue, lds_n);
    PP_LAUNCHED("k_graphs");
    return PP_OK;
  };
  if (!use_graph) return enqueue(s);

  for (GraphEntry &e : g_cache) {
    if (e.ws == ws && e.stream == s && e.ngraphs == ngraphs &&
        e.iters == iters && e.lds_n == lds_n && e.grid == grid && e.dt == dt && e.c == c) {
      PP_HIP(hipGraphLaunch(e.exec, s));
      return PP_OK;
    }
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  PP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  pp_status st = enqueue(s);
  hipError_t e_end = hipStreamEndCapture(s, &graph);
  if (st != PP_OK) return st;
  if (e_end != hipSuccess) return check_hip(e_end, "hipStreamEndCapture");
  hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e_inst != hipSuccess) return check_hip(e_inst, "hipGraphInstantiate");
  if (g_cache.size() >= 8) {
    (void)hipGraphExecDestroy(g_cache.front().exec);
    g_cache.erase(g_cache.begin());
  }
  g_cache.push_back(GraphEntry{ws, s, ngraphs, iters, lds_n, grid, dt, c, exec});
  PP_HIP(hipGraphLaunch(exec, s));
  return PP_OK;
}

}  // namespace pp
