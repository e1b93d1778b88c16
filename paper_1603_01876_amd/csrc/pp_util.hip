// pp_util.hip -- fills, copies and the device-wide exclusive scan used by the
// sort (digit offsets) and the filter (compaction offsets).
#include "pp_common.hpp"

namespace pp {

// ----------------------------------------------------------------- fills
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n, T value) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    p[i] = value;
}

pp_status fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s) {
  if (n <= 0) return PP_OK;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, value);
  PP_LAUNCHED("fill_i32");
  return PP_OK;
}

pp_status fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t s) {
  if (n <= 0) return PP_OK;
  hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, value);
  PP_LAUNCHED("fill_u64");
  return PP_OK;
}

// ------------------------------------------------------ hot-vertex cache
int hot_log2(int64_t n) {
  int lg = 4;
  while (lg < 17 && (int64_t(4) << lg) < n) ++lg;   // about n / 4 slots
  return lg;
}

// hot_build's table: twice the slots of hot_log2, 32 bits each.
static int hot32_log2(int64_t n) { return hot_log2(n) + 1; }

size_t hot_bytes(int64_t n) { return size_t(8 + 4) << hot32_log2(n); }

__global__ __launch_bounds__(256) void k_hot_max(const int32_t *__restrict__ deg, int32_t n,
                                                 unsigned long long *__restrict__ tab,
                                                 uint32_t mask) {
  for (int32_t u = blockIdx.x * 256 + threadIdx.x; u < n; u += gridDim.x * 256) {
    const int32_t d = deg[u];
    if (d >= 8) {
      // Most vertices lose to a heavier one in their slot: read it first
      // and write only when this key is larger.
      unsigned long long *slot = &tab[hot_mix(uint32_t(u)) & mask];
      const unsigned long long key =
          (static_cast<unsigned long long>(uint32_t(d)) << 32) | uint32_t(u);
      if (key > __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(slot, key);
    }
  }
}

// Winner key (degree << 32 | u) of slot k -> the 32-bit slot: the bits of
// hot_mix(u) above mask, min(full[u], mask) below them; an empty slot is
// all ones.
__global__ __launch_bounds__(256) void k_hot_fill(const int32_t *__restrict__ full,
                                                  const uint64_t *__restrict__ win,
                                                  uint32_t *__restrict__ tab, uint32_t mask) {
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k <= mask; k += gridDim.x * 256) {
    const uint64_t e = win[k];
    const uint32_t u = uint32_t(e);
    if (!e) {
      tab[k] = 0xFFFFFFFFu;
    } else {
      const uint32_t v = uint32_t(full[u]);
      tab[k] = (hot_mix(u) & ~mask) | (v < mask ? v : mask);
    }
  }
}

pp_status hot_select(const int32_t *deg, int32_t n, uint64_t *tab, int lg, hipStream_t s) {
  const uint32_t slots = 1u << lg;
  pp_status st;
  if ((st = fill_u64(tab, slots, 0, s)) != PP_OK) return st;
  if (n > 0)
    hipLaunchKernelGGL(k_hot_max, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, deg, n,
                       reinterpret_cast<unsigned long long *>(tab), slots - 1u);
  PP_LAUNCHED("k_hot_max");
  return PP_OK;
}

pp_status hot_build(const int32_t *deg, const int32_t *full, int32_t n, uint64_t *tab, HotTab *h,
                    hipStream_t s) {
  const int lg = hot32_log2(n);
  const uint32_t slots = 1u << lg;
  pp_status st;
  if ((st = hot_select(deg, n, tab, lg, s)) != PP_OK) return st;
  uint32_t *tab32 = reinterpret_cast<uint32_t *>(tab + slots);
  hipLaunchKernelGGL(k_hot_fill, dim3(grid_for(slots, 256, 1024)), dim3(256), 0, s, full, tab,
                     tab32, slots - 1u);
  PP_LAUNCHED("k_hot_max/k_hot_fill");
  h->tab = tab32;
  h->mask = slots - 1u;
  return PP_OK;
}

__global__ __launch_bounds__(256) void k_copy16(uint4 *dst, const uint4 *src, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    dst[i] = src[i];
}
__global__ __launch_bounds__(256) void k_copy1(uint8_t *dst, const uint8_t *src, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    dst[i] = src[i];
}

// Device-to-device copy by kernel (safe inside captured graphs).
pp_status copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return PP_OK;
  uintptr_t d = reinterpret_cast<uintptr_t>(dst), r = reinterpret_cast<uintptr_t>(src);
  if ((d % 16) == 0 && (r % 16) == 0 && (bytes % 16) == 0) {
    int64_t n = int64_t(bytes / 16);
    hipLaunchKernelGGL(k_copy16, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s,
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n);
  } else {
    int64_t n = int64_t(bytes);
    hipLaunchKernelGGL(k_copy1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s,
                       static_cast<uint8_t *>(dst), static_cast<const uint8_t *>(src), n);
  }
  PP_LAUNCHED("copy_bytes");
  return PP_OK;
}

// ------------------------------------------------------------------ scan
// Reduce-then-scan over tiles of 4096 values (256 threads x 16):
//   1. per-tile sums, 2. one workgroup scans the tile sums in place,
//   3. per-tile scan plus the tile's offset.  No inter-workgroup waiting.
constexpr int kScanPer = 16;
constexpr int kScanTile = 256 * kScanPer;

int64_t scan_ws_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *in, int64_t n,
                                                     uint32_t *tile_sums) {
  __shared__ uint32_t sh[4];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    int64_t k = base + i * 256 + threadIdx.x;
    if (k < n) acc += in[k];
  }
  uint32_t tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place; total -> *total.
__global__ __launch_bounds__(256) void k_scan_tiles(uint32_t *tile_sums, int64_t ntiles,
                                                    int64_t *total) {
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += 256) {
    int64_t k = b + threadIdx.x;
    uint32_t v = k < ntiles ? tile_sums[k] : 0u;
    uint32_t all;
    uint32_t ex = block_exscan256(v, sh, &all);
    if (k < ntiles) tile_sums[k] = carry + ex;
    carry += all;
  }
  if (threadIdx.x == 0 && total) *total = int64_t(carry);
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n,
                                                    const uint32_t *tile_off) {
  __shared__ uint32_t buf[kScanTile + kScanTile / 32];
  __shared__ uint32_t sh[4];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  // Striped coalesced load into LDS (padded to spread banks).
  for (int i = 0; i < kScanPer; ++i) {
    int j = i * 256 + threadIdx.x;
    int64_t k = base + j;
    buf[j + j / 32] = k < n ? in[k] : 0u;
  }
  __syncthreads();
  // Each thread scans 16 consecutive values.
  uint32_t v[kScanPer];
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    int j = threadIdx.x * kScanPer + i;
    v[i] = buf[j + j / 32];
    acc += v[i];
  }
  uint32_t all;
  uint32_t run = block_exscan256(acc, sh, &all) + tile_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    int j = threadIdx.x * kScanPer + i;
    buf[j + j / 32] = run;
    run += v[i];
  }
  __syncthreads();
  for (int i = 0; i < kScanPer; ++i) {
    int j = i * 256 + threadIdx.x;
    int64_t k = base + j;
    if (k < n) out[k] = buf[j + j / 32];
  }
}

pp_status exscan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *ws, int64_t *total,
                     hipStream_t s) {
  if (n <= 0) {
    if (total) {
      hipLaunchKernelGGL(k_fill<uint64_t>, dim3(1), dim3(256), 0, s,
                         reinterpret_cast<uint64_t *>(total), int64_t(1), uint64_t(0));
      PP_LAUNCHED("exscan_u32(empty)");
    }
    return PP_OK;
  }
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles > int64_t(1) << 31) return fail(PP_ERANGE, "scan of %lld values", (long long)n);
  hipLaunchKernelGGL(k_scan_reduce, dim3(unsigned(ntiles)), dim3(256), 0, s, in, n, ws);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, s, ws, ntiles, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(ntiles)), dim3(256), 0, s, in, out, n,
                     static_cast<const uint32_t *>(ws));
  PP_LAUNCHED("exscan_u32");
  return PP_OK;
}

}  // namespace pp
