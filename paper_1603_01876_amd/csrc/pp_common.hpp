// pp_common.hpp -- shared device helpers and host-side plumbing of libpp.so
// (gfx950, wave64).  Internal header: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/pp.h"

namespace pp {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
// Records a message for pp_last_error() and returns the status.
pp_status fail(pp_status st, const char *fmt, ...);
// Checks the launch / runtime status after enqueueing work.
pp_status check_hip(hipError_t e, const char *where);
#define PP_HIP(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) return ::pp::check_hip(e_, #expr);                \
  } while (0)
#define PP_LAUNCHED(where)                                                  \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) return ::pp::check_hip(e_, where);                \
  } while (0)

// ------------------------------------------------------------ workspace
// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures, so pp_workspace_bytes() and the entry points share one layout.
struct Carve {
  uintptr_t base;
  size_t used = 0;
  explicit Carve(void *p) : base(reinterpret_cast<uintptr_t>(p)) {}
  template <typename T>
  T *take(size_t count) {
    const size_t align = 256;
    size_t off = (base + used + align - 1) / align * align - base;
    used = off + count * sizeof(T) + 0;
    return base ? reinterpret_cast<T *>(base + off) : nullptr;
  }
  size_t bytes() const { return used + 256; }
};

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// ------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() {
  return (1ull << lane_id()) - 1ull;
}

// Logical block of workgroup i of g.  Workgroups are dealt to the 8 XCDs in
// turn (workgroup i runs on XCD i mod 8); this gives each XCD one contiguous
// range of blocks, so the short runs that neighbouring blocks store next to
// each other (a digit's keys or counts) meet in one XCD's L2 instead of
// being written back by several.  (Blocks whose reads are the bottleneck
// measured slower this way.)
__device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t g) {
  const int64_t q = g >> 3, r = g & 7, x = i & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

// Rank of this lane's digit d among the earlier lanes of the wave holding
// the same digit, plus the wave's running count wh[d] of that digit from
// earlier calls; advances wh[d] by the digit's lanes in this call.  Digits
// have `bits` (<= 8) bits and are matched with one ballot per bit (the loop
// is unrolled to 8 steps with a uniform guard).  Stable: lanes and calls
// are ranked in order.
__device__ __forceinline__ uint32_t wave_digit_rank(uint32_t d, bool valid, int bits,
                                                    uint32_t *wh) {
  uint64_t match = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b < bits) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      match &= bit ? bal : ~bal;
    }
  }
  const uint64_t below = match & lanes_below();
  uint32_t before = 0;
  if (valid) before = wh[d];
  if (valid && below == 0) wh[d] = before + uint32_t(__popcll(match));
  return before + uint32_t(__popcll(below));
}

// The same rank with the lanes of equal digit found through LDS instead of
// one ballot per digit bit: every lane ORs its own bit into its digit's
// 64-bit word of masks (the wave's own 2^bits words, zero on entry), reads
// the word back (the lanes holding that digit), and the digit's lowest lane
// clears it again.  A wave's LDS instructions execute in order, and the
// fences keep the compiler from moving one lane's clear past another's read.
__device__ __forceinline__ uint32_t wave_digit_rank_lds(uint32_t d, bool valid, uint32_t *wh,
                                                        unsigned long long *masks) {
  if (valid) atomicOr(&masks[d], 1ull << lane_id());
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t match = valid ? uint64_t(masks[d]) : 0ull;
  const uint64_t below = match & lanes_below();
  uint32_t before = 0;
  if (valid) before = wh[d];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (valid && below == 0) {
    wh[d] = before + uint32_t(__popcll(match));
    masks[d] = 0ull;
  }
  return before + uint32_t(__popcll(below));
}

// Philox4x32-10 block (Salmon et al., SC'11): ten rounds; each round
// multiplies counter words 0 and 2 by fixed odd constants, swaps the halves
// across the state and mixes in a key that advances by a Weyl step.
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // Each 32 x 32 -> 64-bit product in one instruction (low and high words).
    const uint64_t pa = uint64_t(0xD2511F53u) * c.x;
    const uint64_t pb = uint64_t(0xCD9E8D57u) * c.z;
    const uint32_t a = uint32_t(pa), ah = uint32_t(pa >> 32);
    const uint32_t b = uint32_t(pb), bh = uint32_t(pb >> 32);
    c = U4{bh ^ c.y ^ k0, b, ah ^ c.w ^ k1, a};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Inclusive wave-wide sum (64 lanes) by shuffles.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Exclusive scan over a 256-thread block.  Returns the exclusive prefix of
// `v` in thread order and writes the block total to *total.  `sh` must hold
// 4 elements of shared memory.  Contains two __syncthreads().
template <typename T>
__device__ __forceinline__ T block_exscan256(T v, T *sh, T *total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sh[w] = x;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T s = sh[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// Deterministic 256-thread block sum (fixed shuffle tree, then fixed
// order over the four waves).  Result valid in every thread.
template <typename T>
__device__ __forceinline__ T block_sum256(T v, T *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  T r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Device-scope loads that bypass non-coherent caches, for values written
// by other workgroups of the same launch.
template <typename T>
__device__ __forceinline__ T load_acquire(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Hot-vertex cache: a small direct-mapped table in front of a per-vertex
// int32 table that a kernel reads at random once per matrix entry.  Random
// reads that miss L2 run about five times slower than ones that hit it,
// whether or not the big table fits the Infinity Cache; the cache is sized
// to stay in one XCD's L2.  Slot m & mask, m = hot_mix(u), holds the vertex
// of highest degree hashed there in 32 bits: the bits of m above mask (which
// with the slot identify u) and below them min(value, mask), mask meaning
// "read the big table" (an empty slot is all ones, which at worst sends a
// lookup to the big table).  A lookup that finds another vertex reads the
// big table too, so results never depend on what the cache holds.  hot_mix
// is the "lowbias32" integer finaliser (C. Wellons, 2018).
struct HotTab {
  const uint32_t *tab;
  uint32_t mask;
};

__device__ __forceinline__ uint32_t hot_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// ------------------------------------------------------ host launchers
// Each .hip file exposes plain host functions that enqueue its kernels.

// fill / copy helpers (pp_util.hip)
pp_status fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s);
pp_status fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t s);
pp_status copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t s);

// Hot-vertex cache (pp_util.hip): hot_log2(n) sizes the selection (about
// n / 4 slots, at most 2^17); hot_build's 32-bit table has twice as many
// slots (at most 2^18, 1 MiB), filled from degrees deg[0..n) (vertices of
// degree < 8 are left out) with values full[u]; hot_bytes(n) is its
// workspace (the winners' 64-bit keys, then the table).
int hot_log2(int64_t n);
size_t hot_bytes(int64_t n);
// hot_select only picks the winners: tab[slot] = (deg[u] << 32 | u) of the
// heaviest u (deg >= 8) hashed to the slot, 0 for an empty slot.
pp_status hot_select(const int32_t *deg, int32_t n, uint64_t *tab, int lg, hipStream_t s);
pp_status hot_build(const int32_t *deg, const int32_t *full, int32_t n, uint64_t *tab,
                    HotTab *h, hipStream_t s);

// Exclusive scan of n uint32 values (in place allowed).  `total` (device,
// may be null) receives the sum as int64.  Workspace from scan_ws_elems().
int64_t scan_ws_elems(int64_t n);
pp_status exscan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *ws,
                     int64_t *total, hipStream_t s);

// K0 (k0_generate.hip)
pp_status launch_generate(const pp_kron_params &p, int64_t *u, int64_t *v, hipStream_t s);

// K1 / K2 radix machinery (k1_radix.hip).  Keys are 64-bit words
// (hi << 32 | lo); a pass orders them stably by bits [32+shift, 32+shift+bits).
struct RadixIn {
  const uint64_t *packed;  // or null: key = hi[i] << 32 | lo[i]
  const int64_t *hi;
  const int64_t *lo;
};
struct RadixOut {
  uint64_t *packed;        // or null: hi[i] = key >> 32, lo[i] = key & mask
  int64_t *hi;
  int64_t *lo;
};
size_t radix_ws_bytes(int64_t m, int32_t key_bits);
// Sorts m keys stably by their hi word's low `key_bits` bits.  If
// check_n > 0 the first pass flags (into *flag, device) any hi or lo outside
// [0, check_n) with bit 0 and, if check_sorted_lo, any lo[i] < lo[i-1]
// with bit 1; the caller decides when to read it.
pp_status radix_sort(RadixIn in, RadixOut out, int64_t m, int32_t key_bits, void *ws,
                     size_t ws_bytes, int64_t check_n, bool check_sorted_lo, uint32_t *flag,
                     hipStream_t s, bool sync_after_first_pass);

// Same ordering with a and b as the only key buffers: an even number of
// passes alternates a -> b -> a, so the sorted keys end in a.  counts holds
// radix_pingpong_counts(m) words, scan_ws scan_ws_elems() of that.
size_t radix_pingpong_counts(int64_t m);
pp_status radix_sort_pingpong(uint64_t *a, uint64_t *b, int64_t m, int32_t key_bits,
                              uint32_t *counts, uint32_t *scan_ws, hipStream_t s);

// K2 (k2_filter.hip)
size_t filter_ws_bytes(int64_t n, int64_t m);
pp_status launch_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                        pp_dtype dt, pp_csr *AT, int32_t *d_in, int32_t *d_out, void *ws,
                        size_t ws_bytes, hipStream_t s);

// CSR(A) from CSR(A^T) (k2_transpose.hip)
size_t transpose_ws_bytes(int64_t n, int64_t z);
pp_status launch_transpose(const pp_csr &AT, pp_dtype dt, pp_csr *A, void *ws, size_t ws_bytes,
                           hipStream_t s);

// K3 (k3_pagerank.hip)
size_t pagerank_ws_bytes(int64_t n, int64_t nnz_cap, pp_dtype dt, int32_t nrhs);
pp_status launch_init_r(int64_t n, int32_t nrhs, uint64_t seed, pp_dtype dt, void *r,
                        void *ws, size_t ws_bytes, hipStream_t s);
pp_status launch_pagerank(const pp_csr &AT, pp_dtype dt, int32_t nrhs, int32_t iters, double c,
                          const int32_t *weights, void *r, double *sums, void *ws, size_t ws_bytes,
                          hipStream_t s);
pp_status launch_pagerank_converge(const pp_csr &AT, pp_dtype dt, int32_t max_iters, double c,
                                   double tol, int32_t mode, const int32_t *d_out,
                                   const int32_t *weights, void *r, double *sums, double *deltas,
                                   int32_t *iters_done, void *ws, size_t ws_bytes, hipStream_t s);
// Edge files (pp_files.hip)
size_t tsv_format_ws_bytes(int64_t m, int32_t nsplit);
size_t tsv_parse_ws_bytes(int64_t nbytes);
pp_status launch_tsv_format(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                            char *text, int64_t cap, int32_t nsplit, int64_t *split_host,
                            void *ws, size_t ws_bytes, hipStream_t s);
pp_status launch_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap,
                           int64_t *u, int64_t *v, int64_t *m_out, void *ws, size_t ws_bytes,
                           hipStream_t s);
pp_status write_text_files(const char *prefix, int32_t nfiles, const char *text,
                           const int64_t *split, int32_t sync, hipStream_t s);
pp_status read_text_files(const char *prefix, int32_t nfiles, char *text, int64_t cap,
                          int64_t *nbytes, hipStream_t s);
// K3 batch of small graphs (k3_graphs.hip)
size_t graphs_ws_bytes(int32_t ngraphs);
int64_t graphs_max_n(pp_dtype dt);
pp_status launch_graphs(int32_t ngraphs, const pp_graph *graphs, int64_t max_n, pp_dtype dt,
                        int32_t iters, double c, int32_t use_graph, void *ws, size_t ws_bytes,
                        hipStream_t s);
int32_t graphs_static_max();
pp_status launch_graphs_static(int32_t ngraphs, const pp_graph *graphs, int64_t max_n,
                               pp_dtype dt, int32_t iters, double c, hipStream_t s);

pp_status set_k3_config(int32_t ipt, int32_t rhs_lanes, int32_t slab_log2, int32_t scaled,
                        int32_t rhs_tile);
void get_k3_config(int32_t *ipt, int32_t *rhs_lanes, int32_t *slab_log2, int32_t *scaled,
                   int32_t *rhs_tile);
int32_t k3_last_layout();
pp_status set_kernel_timing(bool enable);
int32_t kernel_times(float *ms, int32_t cap);

}  // namespace pp
