// k1_radix.hip -- stable LSD radix sort of 64-bit (hi << 32 | lo) keys on the
// low key_bits bits of hi.  K1 sorts the edge list by u with it (Sec. IV.B);
// K2 reuses it to order the u-sorted list by v (Sec. IV.C).
//
// One pass per digit of at most 8 bits (the S label bits are split evenly
// over ceil(S/8) passes).  A pass is three launches with no waiting between
// workgroups: per-tile digit counts, a device-wide exclusive scan of the
// digit-major count table, and a scatter that ranks each key inside its
// tile.  A tile is 4096 keys; each of the four waves owns 1024 contiguous
// keys and walks them in 16 rounds of 64, so every load is a contiguous
// 512 B wave access and the rank of a key among equal digits follows the
// input order (stability).  Inside a round the lanes holding the same digit
// are found through per-wave digit mask words in LDS; the lowest such lane
// advances the wave's LDS counter for that digit by the group's population
// count.  Each XCD takes one contiguous range of tiles.
//
// The first pass can read two int64 arrays (packing on the fly) and the
// last pass can write two int64 arrays (unpacking), so K1 reads and writes
// the caller's u/v directly and the intermediate passes move 8 B per key.
#include "pp_common.hpp"

namespace pp {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;                   // 2048, 6144, 8192-key tiles slower
constexpr int kTile = kThreads * kPerThread;     // 4096 keys
constexpr int kWaves = kThreads / kWave;         // 4
constexpr int kWaveKeys = kTile / kWaves;        // 1024

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift, uint32_t dmask) {
  return uint32_t(key >> (32 + shift)) & dmask;
}

template <bool kSep>
__device__ __forceinline__ uint64_t load_key(const RadixIn &in, int64_t i) {
  if constexpr (kSep) {
    return (uint64_t(in.hi[i]) << 32) | (uint64_t(in.lo[i]) & 0xFFFFFFFFull);
  } else {
    return in.packed[i];
  }
}

template <bool kSep>
__device__ __forceinline__ void store_key(const RadixOut &out, int64_t pos, uint64_t key) {
  if constexpr (kSep) {
    out.hi[pos] = int64_t(key >> 32);
    out.lo[pos] = int64_t(key & 0xFFFFFFFFull);
  } else {
    out.packed[pos] = key;
  }
}

// Per-tile digit counts -> counts[d * ntiles + tile].  The digit comes from
// hi alone, so from two int64 arrays only hi is read.
template <bool kSep>
__global__ __launch_bounds__(kThreads) void k_radix_count(RadixIn in, int64_t m, int shift,
                                                          int bits, int64_t ntiles,
                                                          uint32_t *__restrict__ counts) {
  __shared__ uint32_t wh[kWaves][256];
  for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) (&wh[0][0])[i] = 0u;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int64_t tile = xcd_block(blockIdx.x, ntiles);
  const int64_t base = tile * kTile + int64_t(w) * kWaveKeys;
  const uint32_t dmask = (1u << bits) - 1u;
  // All of the thread's reads first (unconditional, index clamped), so they
  // are in flight together; a read under a per-lane condition would be
  // waited for before the next is issued.
  uint64_t keys[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + r * kWave + lane_id();
    const int64_t ic = i < m ? i : m - 1;
    if constexpr (kSep)
      keys[r] = uint64_t(in.hi[ic]) << 32;
    else
      keys[r] = in.packed[ic];
  }
  // Counts need no order: one LDS add per key into the wave's own bins.
#pragma unroll
  for (int r = 0; r < kPerThread; ++r)
    if (base + r * kWave + lane_id() < m) atomicAdd(&wh[w][digit_of(keys[r], shift, dmask)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d <= int(dmask); d += kThreads)
    counts[int64_t(d) * ntiles + tile] = wh[0][d] + wh[1][d] + wh[2][d] + wh[3][d];
}

// Scatter: every key's position is (digit's global offset for this tile) +
// (keys of that digit in earlier waves) + (its rank in its wave).  The tile
// is first written to LDS in digit order, then read back in that order and
// stored, so consecutive lanes store consecutive addresses of one digit's
// run instead of 64 different buckets per instruction.  With check_n > 0
// (first pass over two int64 arrays) it also validates the raw input: both
// labels in [0, check_n), and with check_sorted lo non-decreasing; flag
// bits 1 / 2 report failures.  Positions depend only on the masked digits
// the count pass saw, so every store stays in range whatever the input.
template <bool kSrcSep, bool kDstSep>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(RadixIn in, RadixOut out, int64_t m,
                                                            int shift, int bits, int64_t ntiles,
                                                            const uint32_t *__restrict__ offsets,
                                                            int64_t check_n, int check_sorted,
                                                            uint32_t *flag) {
  __shared__ uint32_t wh[kWaves][256];
  __shared__ uint32_t s_tile_off[256];   // first slot of each digit in the tile
  __shared__ uint32_t s_glob[256];       // global position of that slot
  __shared__ uint32_t s_scan[4];
  __shared__ uint64_t s_keys[kTile];
  // While the keys are ranked, s_keys holds each wave's 256 digit masks.
  static_assert(kWaves * 256 <= kTile, "digit masks alias the key staging");
  unsigned long long *masks =
      reinterpret_cast<unsigned long long *>(s_keys) + (threadIdx.x / kWave) * 256;
  const uint32_t dmask = (1u << bits) - 1u;
  for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) {
    (&wh[0][0])[i] = 0u;
    s_keys[i] = 0ull;
  }
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int64_t tile = xcd_block(blockIdx.x, ntiles);
  const int64_t tile0 = tile * kTile;
  const int64_t base = tile0 + int64_t(w) * kWaveKeys;
  // All of the thread's reads first (indices clamped into range, so every
  // read is unconditional and they are in flight together), then the ranks.
  uint64_t keys[kPerThread];
  uint32_t rank[kPerThread];
  uint32_t bad = 0;
  if constexpr (kSrcSep) {
    if (check_n > 0) {
      int64_t hv[kPerThread], lv[kPerThread], pv[kPerThread];
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int64_t i = base + r * kWave + lane_id();
        const int64_t ic = i < m ? i : m - 1;
        hv[r] = in.hi[ic];
        lv[r] = in.lo[ic];
        pv[r] = in.lo[ic > 0 ? ic - 1 : 0];
      }
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int64_t i = base + r * kWave + lane_id();
        if (i < m) {
          if (hv[r] < 0 || hv[r] >= check_n || lv[r] < 0 || lv[r] >= check_n) bad |= 1u;
          if (check_sorted && i > 0 && pv[r] > lv[r]) bad |= 2u;
        }
        keys[r] = (uint64_t(hv[r]) << 32) | (uint64_t(lv[r]) & 0xFFFFFFFFull);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int64_t i = base + r * kWave + lane_id();
        keys[r] = load_key<kSrcSep>(in, i < m ? i : m - 1);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
      const int64_t i = base + r * kWave + lane_id();
      keys[r] = load_key<kSrcSep>(in, i < m ? i : m - 1);
    }
  }
#pragma unroll
  for (int r = 0; r < kPerThread; ++r)
    rank[r] = wave_digit_rank_lds(digit_of(keys[r], shift, dmask),
                                  base + r * kWave + lane_id() < m, wh[w], masks);
  if (bad && flag) atomicOr(flag, bad);
  __syncthreads();
  // Per digit: prefix over waves (in place), tile total, then an exclusive
  // scan over digits gives each digit's first slot in the tile.
  const int d = threadIdx.x;   // 256 threads, one digit each
  uint32_t total = 0;
  if (d <= int(dmask)) {
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
      const uint32_t c = wh[v][d];
      wh[v][d] = total;
      total += c;
    }
  }
  uint32_t all;
  const uint32_t first = block_exscan256(total, s_scan, &all);
  if (d <= int(dmask)) {
    s_tile_off[d] = first;
    s_glob[d] = offsets[int64_t(d) * ntiles + tile];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + r * kWave + lane_id();
    if (i < m) {
      const uint32_t dg = digit_of(keys[r], shift, dmask);
      s_keys[s_tile_off[dg] + wh[w][dg] + rank[r]] = keys[r];
    }
  }
  __syncthreads();
  const int64_t valid_in_tile = m - tile0 < kTile ? m - tile0 : kTile;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int slot = r * kThreads + threadIdx.x;
    if (slot < valid_in_tile) {
      const uint64_t key = s_keys[slot];
      const uint32_t dg = digit_of(key, shift, dmask);
      store_key<kDstSep>(out, int64_t(s_glob[dg]) + (slot - s_tile_off[dg]), key);
    }
  }
}

struct Layout {
  uint64_t *buf[2];
  uint32_t *counts;
  uint32_t *scan_ws;
};

Layout carve(void *ws, int64_t m) {
  Carve c(ws);
  Layout L{};
  const int64_t ntiles = (m + kTile - 1) / kTile;
  L.buf[0] = c.take<uint64_t>(size_t(m));
  L.buf[1] = c.take<uint64_t>(size_t(m));
  L.counts = c.take<uint32_t>(size_t(256 * ntiles));
  L.scan_ws = c.take<uint32_t>(size_t(scan_ws_elems(256 * ntiles)));
  return L;
}

size_t layout_bytes(int64_t m) {
  Carve c(nullptr);
  const int64_t ntiles = (m + kTile - 1) / kTile;
  c.take<uint64_t>(size_t(m));
  c.take<uint64_t>(size_t(m));
  c.take<uint32_t>(size_t(256 * ntiles));
  c.take<uint32_t>(size_t(scan_ws_elems(256 * ntiles)));
  return c.bytes();
}

}  // namespace

size_t radix_ws_bytes(int64_t m, int32_t /*key_bits*/) { return layout_bytes(m); }

size_t radix_pingpong_counts(int64_t m) { return size_t(256) * size_t((m + kTile - 1) / kTile); }

pp_status radix_sort_pingpong(uint64_t *a, uint64_t *b, int64_t m, int32_t key_bits,
                              uint32_t *counts, uint32_t *scan_ws, hipStream_t s) {
  if (m <= 0) return PP_OK;
  if (key_bits < 1 || key_bits > 31) return fail(PP_EINVAL, "radix key bits %d", key_bits);
  if (key_bits < 2) key_bits = 2;   // two passes of one bit: the keys end up in a again
  const int64_t ntiles = (m + kTile - 1) / kTile;
  if (ntiles >= (int64_t(1) << 31)) return fail(PP_ERANGE, "too many tiles");
  int npass = (key_bits + 7) / 8;
  npass += npass & 1;
  const int base_bits = key_bits / npass, extra = key_bits % npass;
  int shift = 0;
  uint64_t *src = a, *dst = b;
  const dim3 grid = dim3(static_cast<unsigned>(ntiles)), block = dim3(kThreads);
  for (int p = 0; p < npass; ++p) {
    const int bits = base_bits + (p < extra ? 1 : 0);
    const RadixIn in{src, nullptr, nullptr};
    const RadixOut out{dst, nullptr, nullptr};
    hipLaunchKernelGGL((k_radix_count<false>), grid, block, 0, s, in, m, shift, bits, ntiles,
                       counts);
    PP_LAUNCHED("k_radix_count (pingpong)");
    pp_status st = exscan_u32(counts, counts, (int64_t(1) << bits) * ntiles, scan_ws, nullptr, s);
    if (st != PP_OK) return st;
    hipLaunchKernelGGL((k_radix_scatter<false, false>), grid, block, 0, s, in, out, m, shift,
                       bits, ntiles, counts, int64_t(0), 0, nullptr);
    PP_LAUNCHED("k_radix_scatter (pingpong)");
    shift += bits;
    uint64_t *t = src;
    src = dst;
    dst = t;
  }
  return PP_OK;
}

pp_status radix_sort(RadixIn in, RadixOut out, int64_t m, int32_t key_bits, void *ws,
                     size_t ws_bytes, int64_t check_n, bool check_sorted_lo, uint32_t *flag,
                     hipStream_t s, bool sync_after_first_pass) {
  if (m <= 0) return PP_OK;
  if (key_bits < 1 || key_bits > 31) return fail(PP_EINVAL, "radix key bits %d", key_bits);
  if (ws_bytes < layout_bytes(m)) return fail(PP_EWORKSPACE, "radix workspace too small");
  Layout L = carve(ws, m);
  const int64_t ntiles = (m + kTile - 1) / kTile;
  if (ntiles >= (int64_t(1) << 31)) return fail(PP_ERANGE, "too many tiles");
  const int npass = (key_bits + 7) / 8;
  const int base_bits = key_bits / npass, extra = key_bits % npass;
  int shift = 0;
  const bool check = check_n > 0;
  for (int p = 0; p < npass; ++p) {
    const int bits = base_bits + (p < extra ? 1 : 0);
    const bool first = p == 0, last = p == npass - 1;
    RadixIn src = first ? in : RadixIn{L.buf[(p - 1) & 1], nullptr, nullptr};
    RadixOut dst = last ? out : RadixOut{L.buf[p & 1], nullptr, nullptr};
    const bool src_sep = src.packed == nullptr;
    const bool dst_sep = dst.packed == nullptr;
    const dim3 grid = dim3(static_cast<unsigned>(ntiles)), block = dim3(kThreads);
    if (src_sep)
      hipLaunchKernelGGL((k_radix_count<true>), grid, block, 0, s, src, m, shift, bits, ntiles,
                         L.counts);
    else
      hipLaunchKernelGGL((k_radix_count<false>), grid, block, 0, s, src, m, shift, bits, ntiles,
                         L.counts);
    PP_LAUNCHED("k_radix_count");
    // Digit-major table: only the 2^bits rows this pass wrote are scanned.
    pp_status st = exscan_u32(L.counts, L.counts, (int64_t(1) << bits) * ntiles, L.scan_ws, nullptr, s);
    if (st != PP_OK) return st;
    // The first pass validates the input while it moves it.
    const int64_t cn = first && check ? check_n : 0;
    const int cs = int(check_sorted_lo);
    if (src_sep && dst_sep)
      hipLaunchKernelGGL((k_radix_scatter<true, true>), grid, block, 0, s, src, dst, m, shift,
                         bits, ntiles, L.counts, cn, cs, flag);
    else if (src_sep)
      hipLaunchKernelGGL((k_radix_scatter<true, false>), grid, block, 0, s, src, dst, m, shift,
                         bits, ntiles, L.counts, cn, cs, flag);
    else if (dst_sep)
      hipLaunchKernelGGL((k_radix_scatter<false, true>), grid, block, 0, s, src, dst, m, shift,
                         bits, ntiles, L.counts, int64_t(0), 0, flag);
    else
      hipLaunchKernelGGL((k_radix_scatter<false, false>), grid, block, 0, s, src, dst, m, shift,
                         bits, ntiles, L.counts, int64_t(0), 0, flag);
    PP_LAUNCHED("k_radix_scatter");
    if (first && check && sync_after_first_pass) {
      uint32_t h = 0;
      PP_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
      PP_HIP(hipStreamSynchronize(s));
      if (h & 1u) return fail(PP_EINVAL, "input label outside [0, %lld)", (long long)check_n);
      if (h & 2u) return fail(PP_EINVAL, "input not sorted by start vertex");
    }
    shift += bits;
  }
  return PP_OK;
}

}  // namespace pp
