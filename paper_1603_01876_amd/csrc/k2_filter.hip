// k2_filter.hip -- K2, the filter (Sec. IV.C): count matrix, in-degree,
// supernode and leaf column removal, out-degree, row normalisation, written
// out as CSR(A^T) for the pull-form PageRank of K3.
//
// The K1 output is ordered by u.  A stable radix sort of it by v gives the
// lexicographic (v, u) order: equal (u,v) pairs are adjacent (their run
// length is the count A(u,v)), each column v of A is a contiguous run (its
// length is d_in[v]), and column removal becomes the removal of whole runs.
// Every reduction is an integer one (counts, max, integer atomics), so the
// result is bit-identical run to run and independent of scheduling:
//   1. radix-sort (v<<32|u) by v; the first pass also checks the input
//   2. vstart[w]  = first position of column w in the sorted list
//   3. d_in[w]    = vstart[w+1] - vstart[w];  mx = max d_in (atomicMax)
//   4. keep bitmap: d_in != mx and d_in != 1 (both on the same d_in)
//   5. d_out[u]   = all edges per u, on the u-ordered input: per-wave
//                   run lengths, one integer atomic per run
//   6. compaction: per-tile counts of kept distinct pairs; every edge into
//                   a removed column takes one from d_out[u] (d_out is then
//                   the kept edges per u); scan, emit col = u, val = count /
//                   d_out[u] (IEEE FP64 division, FP32 stores the rounded
//                   quotient) and row_ptr.
// Step 5 reads only u; the keep bitmap is read in v order in step 6, where
// consecutive entries share its words, instead of once per edge at random.
#include "pp_common.hpp"

namespace pp {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;  // 4096 sorted entries per tile
constexpr int kWaves = kThreads / kWave;
constexpr int kWaveKeys = kTile / kWaves;

__device__ __forceinline__ int32_t vof(uint64_t key) { return int32_t(key >> 32); }
__device__ __forceinline__ int32_t uof(uint64_t key) { return int32_t(key & 0xFFFFFFFFull); }

__device__ __forceinline__ bool kept(const uint64_t *keepw, int32_t w) {
  return (keepw[w >> 6] >> (w & 63)) & 1ull;
}

// The previous lane's 64-bit value, and lane 63's: a wave reads 64
// consecutive sorted positions per round, so the key at p - 1 is the
// previous lane's, or for lane 0 the previous round's lane 63.
__device__ __forceinline__ uint64_t from_lane_below(uint64_t x) {
  const uint32_t lo = uint32_t(__shfl_up(int(uint32_t(x)), 1, kWave));
  const uint32_t hi = uint32_t(__shfl_up(int(uint32_t(x >> 32)), 1, kWave));
  return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t from_lane63(uint64_t x) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), 63));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), 63));
  return (uint64_t(hi) << 32) | lo;
}

// vstart[w] = first sorted position with v >= w, for w = 0..n.
__global__ __launch_bounds__(kThreads) void k_vstart(const uint64_t *__restrict__ P, int64_t m,
                                                     int32_t n, int32_t *__restrict__ vstart) {
  // A wave takes kWaveKeys consecutive keys, kPerThread rounds of 64; every
  // read is issued first (index clamped), then the rounds are processed.
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(w) * kWaveKeys;
  int32_t vv[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane;
    vv[r] = vof(P[p < m ? p : m - 1]);
  }
  const int32_t vbefore = base > 0 ? vof(P[(base < m ? base : m) - 1]) : -1;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane;
    const int32_t v = vv[r];
    const int32_t up = __shfl_up(v, 1, kWave);
    const int32_t last = __shfl(r > 0 ? vv[r > 0 ? r - 1 : 0] : 0, kWave - 1, kWave);
    if (p < m) {
      const int32_t vp = lane > 0 ? up : (r > 0 ? last : vbefore);
      for (int32_t q = vp + 1; q <= v; ++q) vstart[q] = int32_t(p);
      if (p == m - 1)
        for (int32_t q = v + 1; q <= n; ++q) vstart[q] = int32_t(m);
    }
  }
}

__global__ __launch_bounds__(256) void k_din(const int32_t *__restrict__ vstart, int32_t n,
                                             int32_t *__restrict__ d_in, int32_t *mx) {
  int32_t best = 0;
  const int64_t stride = int64_t(gridDim.x) * 256;
  for (int64_t w = int64_t(blockIdx.x) * 256 + threadIdx.x; w < n; w += stride) {
    const int32_t d = vstart[w + 1] - vstart[w];
    d_in[w] = d;
    best = d > best ? d : best;
  }
  best = wave_max(best);
  // One address for the whole grid: update it only when this wave's maximum
  // exceeds it (it settles early, so few waves write it).
  if (lane_id() == 0 && best > __hip_atomic_load(mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(mx, best);
}

// One 64-bit word per wave: bit (w mod 64) set iff column w survives.
__global__ __launch_bounds__(256) void k_keepbits(const int32_t *__restrict__ d_in, int32_t n,
                                                  const int32_t *mx, uint64_t *__restrict__ keepw) {
  const int32_t top = *mx;
  const int64_t stride = int64_t(gridDim.x) * 256;
  const int64_t nw = (int64_t(n) + 63) / 64 * 64;
  for (int64_t w = int64_t(blockIdx.x) * 256 + threadIdx.x; w < nw; w += stride) {
    bool keep = false;
    if (w < n) {
      const int32_t d = d_in[w];
      keep = d != top && d != 1;
    }
    const uint64_t bits = __ballot(keep);
    if (lane_id() == 0) keepw[w >> 6] = bits;
  }
}

// d_out[u] += number of edges of u, over the u-ordered input.  A wave
// covers 64 consecutive edges; each run of equal u inside it is counted by
// the run's first lane with one popcount and one atomic add.
__global__ __launch_bounds__(kThreads) void k_dout(const int64_t *__restrict__ u, int64_t m,
                                                   int32_t *__restrict__ d_out) {
  // Tiles as in k_vstart: all reads first, then one 64-edge round at a time.
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(w) * kWaveKeys;
  int32_t us[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane;
    us[r] = int32_t(u[p < m ? p : m - 1]);
  }
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const bool valid = base + r * kWave + lane < m;
    const int32_t uu = valid ? us[r] : -1;
    const int32_t up = __shfl_up(uu, 1, kWave);
    const bool head = valid && (lane == 0 || up != uu);
    const uint64_t heads = __ballot(head);
    const uint64_t flags = __ballot(valid);
    if (head) {
      const uint64_t after = heads & ~((2ull << lane) - 1ull);   // heads above this lane
      const uint64_t upto = after ? (after & (~after + 1ull)) - 1ull : ~0ull;
      const uint64_t seg = upto & ~((1ull << lane) - 1ull);
      atomicAdd(&d_out[uu], __popcll(flags & seg));
    }
  }
}

// Per tile: number of kept distinct (v,u) pairs.  Every edge into a removed
// column (counted with its multiplicity) takes one from d_out[u].
__global__ __launch_bounds__(kThreads) void k_compact_count(const uint64_t *__restrict__ P,
                                                            int64_t m,
                                                            const uint64_t *__restrict__ keepw,
                                                            uint32_t *__restrict__ tile_cnt,
                                                            int32_t *__restrict__ d_out) {
  __shared__ uint32_t sh[4];
  const int w = threadIdx.x / kWave;
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(w) * kWaveKeys;
  uint32_t c = 0;
  uint64_t carry = 0;   // key of the previous round's lane 63
  // Every read first (index clamped; keys past the end are not counted).
  uint64_t keys[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane_id();
    keys[r] = P[p < m ? p : m - 1];
  }
  const uint64_t before = base > 0 ? P[(base < m ? base : m) - 1] : ~0ull;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane_id();
    const uint64_t key = p < m ? keys[r] : 0ull;
    const uint64_t below = from_lane_below(key);
    const uint64_t prev = lane_id() > 0 ? below : r > 0 ? carry : p > 0 && p <= m ? before : ~0ull;
    carry = from_lane63(key);
    if (p < m) {
      const bool distinct = p == 0 || prev != key;
      if (kept(keepw, vof(key)))
        c += distinct ? 1u : 0u;
      else
        atomicSub(&d_out[uof(key)], 1);
    }
  }
  const uint32_t tot = block_sum256(c, sh);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = tot;
}

// Out-degrees narrowed to 16 bits (65535 = read the full value), a table
// half the size of d_out for the emit's scattered reads: twice the
// vertices per cache line, and small enough to stay in the Infinity Cache.
__global__ __launch_bounds__(256) void k_narrow(const int32_t *__restrict__ d_out, int32_t n,
                                                uint16_t *__restrict__ d16) {
  for (int32_t u = blockIdx.x * 256 + threadIdx.x; u < n; u += gridDim.x * 256) {
    const int32_t d = d_out[u];
    d16[u] = uint16_t(d >= 0 && d < 65535 ? d : 65535);
  }
}

__device__ __forceinline__ int32_t dout_get(HotTab h, const uint16_t *__restrict__ d16,
                                            const int32_t *__restrict__ d_out, int32_t u) {
  const uint32_t m = hot_mix(uint32_t(u));
  const uint32_t e = h.tab[m & h.mask];
  if (((e ^ m) & ~h.mask) == 0u && (e & h.mask) != h.mask) return int32_t(e & h.mask);
  const uint32_t d = d16[u];
  return d != 65535u ? int32_t(d) : d_out[u];
}

template <typename V>
__global__ __launch_bounds__(kThreads) void k_compact_emit(
    const uint64_t *__restrict__ P, int64_t m, int32_t n, const uint64_t *__restrict__ keepw,
    const int32_t *__restrict__ d_out, const uint16_t *__restrict__ d16, HotTab hot,
    const uint32_t *__restrict__ tile_off, int32_t *__restrict__ row_ptr, int32_t *__restrict__ col,
    V *__restrict__ val) {
  __shared__ uint32_t wave_tot[kWaves];
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const int64_t base = int64_t(blockIdx.x) * kTile + int64_t(w) * kWaveKeys;
  uint64_t keys[kPerThread];
  uint64_t ball[kPerThread];
  uint32_t run = 0;
  uint64_t first_prev = ~0ull;   // key at base - 1 (lane 0 only)
  if (lane == 0 && base > 0 && base <= m) first_prev = P[base - 1];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane;
    const uint64_t key = p < m ? P[p] : 0ull;
    const uint64_t below = from_lane_below(key);
    const uint64_t prev = lane > 0 ? below : r > 0 ? from_lane63(keys[r - 1]) : first_prev;
    bool f = false;
    if (p < m) {
      const bool distinct = p == 0 || prev != key;
      f = distinct && kept(keepw, vof(key));
    }
    keys[r] = key;
    ball[r] = __ballot(f);
    run += uint32_t(__popcll(ball[r]));
  }
  if (lane == 0) wave_tot[w] = run;
  __syncthreads();
  uint32_t before = tile_off[blockIdx.x];
  for (int v = 0; v < w; ++v) before += wave_tot[v];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t p = base + r * kWave + lane;
    const uint64_t below = from_lane_below(keys[r]);
    const uint64_t prevk = lane > 0 ? below : r > 0 ? from_lane63(keys[r - 1]) : first_prev;
    if (p < m) {
      const uint64_t key = keys[r];
      const bool f = (ball[r] >> lane) & 1ull;
      const uint32_t excl = before + uint32_t(__popcll(ball[r] & lanes_below()));
      const int32_t v = vof(key);
      if (f) {
        const int32_t u = uof(key);
        int64_t q = p + 1;
        while (q < m && P[q] == key) ++q;
        const double quot = double(q - p) / double(dout_get(hot, d16, d_out, u));
        col[excl] = u;
        val[excl] = V(quot);
      }
      // Row pointers of every column that starts here (empty ones too).
      const int32_t vp = p > 0 ? vof(prevk) : -1;
      for (int32_t j = vp + 1; j <= v; ++j) row_ptr[j] = int32_t(excl);
      if (p == m - 1) {
        const int32_t z = int32_t(excl + (f ? 1u : 0u));
        for (int32_t j = v + 1; j <= n; ++j) row_ptr[j] = z;
      }
    }
    before += uint32_t(__popcll(ball[r]));
  }
}

struct Layout {
  uint64_t *P;
  void *radix_ws;
  size_t radix_bytes;
  int32_t *vstart, *d_in, *d_out;
  uint64_t *keepw;
  uint32_t *tile_cnt, *scan_ws;
  uint64_t *hot;
  int32_t *mx;
  int64_t *z;
  uint32_t *flag;
};

Layout carve(void *ws, int64_t n, int64_t m) {
  Carve c(ws);
  Layout L{};
  const int64_t ntiles = (m + kTile - 1) / kTile;
  L.P = c.take<uint64_t>(size_t(m));
  L.radix_bytes = radix_ws_bytes(m, 31);
  L.radix_ws = c.take<uint8_t>(L.radix_bytes);
  L.vstart = c.take<int32_t>(size_t(n + 1));
  L.d_in = c.take<int32_t>(size_t(n));
  L.d_out = c.take<int32_t>(size_t(n));
  L.keepw = c.take<uint64_t>(size_t((n + 63) / 64));
  L.tile_cnt = c.take<uint32_t>(size_t(ntiles + 1));
  L.scan_ws = c.take<uint32_t>(size_t(scan_ws_elems(ntiles + 1)));
  L.hot = c.take<uint64_t>(hot_bytes(n) / 8);
  L.mx = c.take<int32_t>(1);
  L.z = c.take<int64_t>(1);
  L.flag = c.take<uint32_t>(1);
  return L;
}

}  // namespace

size_t filter_ws_bytes(int64_t n, int64_t m) {
  Carve c(nullptr);
  const int64_t ntiles = (m + kTile - 1) / kTile;
  c.take<uint64_t>(size_t(m));
  c.take<uint8_t>(radix_ws_bytes(m, 31));
  c.take<int32_t>(size_t(n + 1));
  c.take<int32_t>(size_t(n));
  c.take<int32_t>(size_t(n));
  c.take<uint64_t>(size_t((n + 63) / 64));
  c.take<uint32_t>(size_t(ntiles + 1));
  c.take<uint32_t>(size_t(scan_ws_elems(ntiles + 1)));
  c.take<uint64_t>(hot_bytes(n) / 8);
  c.take<int32_t>(1);
  c.take<int64_t>(1);
  c.take<uint32_t>(1);
  return c.bytes();
}

pp_status launch_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                        pp_dtype dt, pp_csr *AT, int32_t *d_in, int32_t *d_out, void *ws,
                        size_t ws_bytes, hipStream_t s) {
  const int64_t n = int64_t(1) << scale;
  if (ws_bytes < filter_ws_bytes(n, m)) return fail(PP_EWORKSPACE, "filter workspace too small");
  Layout L = carve(ws, n, m);
  int32_t *din = d_in ? d_in : L.d_in;
  int32_t *dout = d_out ? d_out : L.d_out;
  pp_status st;

  if (m == 0) {
    if ((st = fill_i32(AT->row_ptr, n + 1, 0, s)) != PP_OK) return st;
    if ((st = fill_i32(din, n, 0, s)) != PP_OK) return st;
    if ((st = fill_i32(dout, n, 0, s)) != PP_OK) return st;
    PP_HIP(hipStreamSynchronize(s));
    AT->nnz = 0;
    return PP_OK;
  }

  // 1. sort by v (stable on the u-ordered input), validating the input.
  if ((st = fill_i32(reinterpret_cast<int32_t *>(L.flag), 1, 0, s)) != PP_OK) return st;
  st = radix_sort(RadixIn{nullptr, v, u}, RadixOut{L.P, nullptr, nullptr}, m, scale, L.radix_ws,
                  L.radix_bytes, n, true, L.flag, s, true);
  if (st != PP_OK) return st;

  // 2-4. column starts, in-degrees, maximum, surviving columns.
  const int n32 = int32_t(n);
  const int64_t ntiles = (m + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_vstart, dim3(unsigned(ntiles)), dim3(kThreads), 0, s, L.P, m, n32,
                     L.vstart);
  if ((st = fill_i32(L.mx, 1, 0, s)) != PP_OK) return st;
  hipLaunchKernelGGL(k_din, dim3(grid_for(n, 256, 256 * 32)), dim3(256), 0, s, L.vstart, n32, din,
                     L.mx);
  hipLaunchKernelGGL(k_keepbits, dim3(grid_for((n + 63) / 64 * 64, 256, 256 * 32)), dim3(256), 0,
                     s, din, n32, L.mx, L.keepw);
  PP_LAUNCHED("k_vstart/k_din/k_keepbits");

  // 5. edges per u from the u-ordered input.
  if ((st = fill_i32(dout, n, 0, s)) != PP_OK) return st;
  hipLaunchKernelGGL(k_dout, dim3(unsigned(ntiles)), dim3(kThreads), 0, s, u, m, dout);
  PP_LAUNCHED("k_dout");

  // 6. compaction into CSR(A^T); removed edges leave d_out here.
  hipLaunchKernelGGL(k_compact_count, dim3(unsigned(ntiles)), dim3(kThreads), 0, s, L.P, m,
                     L.keepw, L.tile_cnt, dout);
  PP_LAUNCHED("k_compact_count");
  if ((st = exscan_u32(L.tile_cnt, L.tile_cnt, ntiles, L.scan_ws, L.z, s)) != PP_OK) return st;
  // d_out is read once per kept pair at random u: the hottest vertices'
  // out-degrees are cached in an L2-sized table in front of it.
  HotTab hot;
  if ((st = hot_build(dout, dout, n32, L.hot, &hot, s)) != PP_OK) return st;
  // The narrowed out-degrees take the column starts' buffer (free by now).
  uint16_t *d16 = reinterpret_cast<uint16_t *>(L.vstart);
  hipLaunchKernelGGL(k_narrow, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, dout, n32, d16);
  PP_LAUNCHED("k_narrow");
  if (dt == PP_F64)
    hipLaunchKernelGGL(k_compact_emit<double>, dim3(unsigned(ntiles)), dim3(kThreads), 0, s, L.P,
                       m, n32, L.keepw, dout, d16, hot, L.tile_cnt, AT->row_ptr, AT->col,
                       static_cast<double *>(AT->val));
  else
    hipLaunchKernelGGL(k_compact_emit<float>, dim3(unsigned(ntiles)), dim3(kThreads), 0, s, L.P,
                       m, n32, L.keepw, dout, d16, hot, L.tile_cnt, AT->row_ptr, AT->col,
                       static_cast<float *>(AT->val));
  PP_LAUNCHED("k_compact_emit");

  int64_t z = 0;
  PP_HIP(hipMemcpyAsync(&z, L.z, sizeof(z), hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  AT->nnz = z;
  return PP_OK;
}

}  // namespace pp
