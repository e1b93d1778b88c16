// k3_pagerank.hip -- K3, PageRank (Sec. IV.D and the Appendix):
//   r_{k+1,j} = c * sum_i r_{k,i} A(i,j) + ((1-c)/N) * sum(r_k),  k = 0..iters-1,
// as a pull-form sparse matrix-vector product on CSR(A^T), plus the
// initial vector r = rand(1,N) ./ norm(r,1).
//
// Load balance: after the filter most rows of A^T are empty and the rest
// follow a power law, so rows are not a unit of work.  The SpMV splits the
// merged sequence of (row ends, non-zeros) into equal pieces (merge-path
// decomposition, Merrill & Garland, SC'16): a workgroup of 256 threads owns
// 256*IPT consecutive items, stages its row ends and its products r[col]*val
// in LDS with coalesced loads, and each thread consumes IPT items of its
// own.  Rows cut by a thread boundary are completed inside the workgroup;
// rows cut by a workgroup boundary leave a carry that a second, small kernel
// adds in workgroup order.  Nothing is summed with floating-point atomics,
// so every result is reproducible bit for bit.
//
// Precision forms: PP_F64 accumulates in FP64.  PP_F32 keeps values, ranks
// and products in FP32 and accumulates each row with a compensated (TwoSum)
// pair; partial pairs are merged with TwoSum too.  In both forms sum(r) is
// reduced in FP64 in a fixed order and the teleport scalar (1-c)/N * sum(r)
// is FP64.  The partition, the carries' row ids and the fix-up flags depend
// only on the matrix, so they are computed once per call.
#include <type_traits>
#include <vector>

#include "pp_common.hpp"

#pragma clang fp contract(off)

namespace pp {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = kThreads * 8;         // SpMM items per workgroup
constexpr int kItemsMin = kThreads * 4;      // smallest SpMV tile (sizes the workspace)
constexpr int kItemsMax = kThreads * 16;     // largest SpMV tile (sizes relabel LDS)

// Launch configuration chosen by the caller (or the autotuner): merge items
// per thread of the SpMV (tile = 256 * ipt items) and lane-group width of
// the SpMM.
struct K3Config {
  int ipt = 8;
  int rhs_lanes = 0;  // 0: next power of two >= nrhs
  int slab_log2 = -1; // 0: one pass over all columns; > 0: slab width 2^slab_log2; -1: auto
  int scaled = 1;     // degree-scaled form of a relabelled, segmented matrix when it verifies
  int rhs_tile = 0;   // SpMM: 0 all right-hand sides per pass; else tiles of this many columns
};
K3Config g_cfg;
// What the most recent pagerank call ran: bit 0 relabelled, bit 1 column
// segmented, bit 2 degree-scaled form (instrumentation).
int32_t g_last_layout = 0;
constexpr int kFinishPer = kThreads;         // spmv workgroups per finish workgroup
constexpr int64_t kSumChunk = kThreads * 64; // entries of r per workgroup of sum(r_0)

// ------------------------------------------------------------ accumulators
struct AccD {
  double s;
  __device__ __forceinline__ void add(double x) { s += x; }
  __device__ __forceinline__ double value() const { return s; }
};
__device__ __forceinline__ AccD merge(AccD a, AccD b) { return AccD{a.s + b.s}; }

// Compensated FP32 sum: s + e approximates the exact sum; every addition is
// Knuth's TwoSum, whose rounding error is carried in e.
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

template <typename V>
struct Form;
// Part: what the segmented iteration stores per (slab, row) pair for the
// combine -- FP64 its sum, FP32 the compensated pair rounded once to float
// (half the bytes; the combine merges the partials with TwoSum again).
template <>
struct Form<double> {
  using Acc = AccD;
  using Part = double;
  __device__ static double finish(AccD a, double c, double t) { return c * a.value() + t; }
  __device__ static Part part(AccD a) { return a.s; }
  __device__ static AccD acc(Part p) { return AccD{p}; }
};
template <>
struct Form<float> {
  using Acc = AccF;
  using Part = float;
  __device__ static float finish(AccF a, double c, double t) {
    return float(c * double(a.value()) + t);
  }
  __device__ static Part part(AccF a) { return a.value(); }
  __device__ static AccF acc(Part p) { return AccF{p, 0.0f}; }
};

// ------------------------------------------------------------- partition
// coord[b] = (rows ended, non-zeros consumed) after the first b*D items of
// the merge of the row-end list rp[1..n] with the non-zero indices.
__global__ __launch_bounds__(256) void k_partition(const int32_t *__restrict__ rp, int32_t n,
                                                   int32_t nnz, int32_t nb, int32_t D,
                                                   int2 *coord) {
  const int64_t total = int64_t(n) + nnz;
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b <= nb; b += gridDim.x * 256) {
    const int64_t diag64 = int64_t(b) * D < total ? int64_t(b) * D : total;
    const int32_t diag = int32_t(diag64);
    int32_t lo = diag - nnz > 0 ? diag - nnz : 0;
    int32_t hi = diag < n ? diag : n;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (rp[mid + 1] <= diag - mid - 1)
        lo = mid + 1;
      else
        hi = mid;
    }
    coord[b] = make_int2(lo, diag - lo);
  }
}

// Static per-block facts: the row left open at the block's end (-1 if none)
// and whether the block completes a row that began in an earlier block.
__global__ __launch_bounds__(256) void k_block_flags(const int32_t *__restrict__ rp, int32_t n,
                                                     int32_t nb, const int2 *__restrict__ coord,
                                                     int32_t *carry_row, uint8_t *closes) {
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256) {
    const int2 c0 = coord[b], c1 = coord[b + 1];
    carry_row[b] = c1.x < n ? c1.x : -1;
    closes[b] = (c0.x < n && rp[c0.x] < c0.y && c1.x > c0.x) ? 1 : 0;
  }
}

// ------------------------------------------------------------------ SpMV
__device__ __forceinline__ AccD shfl_up_acc(AccD a, int o) { return AccD{__shfl_up(a.s, o, kWave)}; }
__device__ __forceinline__ AccF shfl_up_acc(AccF a, int o) {
  return AccF{__shfl_up(a.s, o, kWave), __shfl_up(a.e, o, kWave)};
}

// Entry type of the packed count form: seg_col holds the entry's column
// inside its slab (low 24 bits) and its count (high 8 bits); the slab
// follows from the entry's position (SlabMap).
struct PackedCol {};
template <typename E>
struct EntryVal {
  using type = E;
};
template <>
struct EntryVal<PackedCol> {
  using type = uint32_t;
};
struct SlabMap {
  const int32_t *es;        // first entry of each slab; es[ns] = nnz
  const int2 *tile_slab;    // per workgroup: slab of its first entry, first entry of the next
  int32_t sbits, ns;
};

// With kRaw the rows are (slab, row) pairs of the column-segmented layout
// below: each completed row stores its raw accumulator into part[] instead
// of c * sum + t into y, and no sum(y) is formed.  E is the stored entry
// type: the values (V), or the integer counts (uint8_t) of the
// degree-scaled form, whose x holds r_u / w[u].
template <typename V, int IPT, bool kRaw, typename E = V>
__global__ __launch_bounds__(kThreads) void k_spmv(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const E *__restrict__ val,
    const V *__restrict__ x, V *__restrict__ y, int32_t n, const int2 *__restrict__ coord,
    double c, const double *__restrict__ tele, double *__restrict__ blk_ysum,
    typename Form<V>::Acc *__restrict__ blk_carry, typename Form<V>::Acc *__restrict__ blk_head,
    typename Form<V>::Part *__restrict__ part, SlabMap sm) {
  using Acc = typename Form<V>::Acc;
  constexpr bool kPacked = std::is_same<E, PackedCol>::value;
  constexpr int kD = kThreads * IPT;
  constexpr int kWaves = kThreads / kWave;
  __shared__ int32_t s_end[kD];
  __shared__ V s_prod[kD];
  __shared__ Acc s_pre[kThreads];
  __shared__ Acc s_wtail[kWaves];
  __shared__ int32_t s_wfirst[kWaves], s_wlast[kWaves];
  __shared__ double s_red[4];

  const int b = blockIdx.x, tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  const int2 c0 = coord[b], c1 = coord[b + 1];
  const int32_t i0 = c0.x, j0 = c0.y;
  const int32_t na = c1.x - c0.x, nz = c1.y - c0.y;

  // Stage the workgroup's products r[col]*val and local row ends in LDS.
  // Indices past the end are clamped to the last valid one, so every load
  // is unconditional: a thread issues all IPT column and value loads, then
  // all IPT gathers, before it waits on any of them.
  {
    int32_t cc[IPT], ee[IPT];
    typename EntryVal<E>::type vv[IPT];
    V xv[IPT];
    if (nz > 0) {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int k = r * kThreads + tid;
        const int kk = k < nz ? k : nz - 1;
        if constexpr (kPacked) {
          const int32_t pk = __builtin_nontemporal_load(col + j0 + kk);
          cc[r] = pk & 0xFFFFFF;
          vv[r] = uint32_t(pk) >> 24;
        } else {
          cc[r] = __builtin_nontemporal_load(col + j0 + kk);
          vv[r] = __builtin_nontemporal_load(val + j0 + kk);
        }
      }
      if constexpr (kPacked) {
        // Slab of each entry: the workgroup's first slab unless the entry
        // lies at or past the next slab's start (only at slab boundaries).
        const int2 ts = sm.tile_slab[b];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
          const int k = r * kThreads + tid;
          const int32_t j = j0 + (k < nz ? k : nz - 1);
          int32_t d = ts.x;
          if (j >= ts.y) {
            d = ts.x + 1;
            while (d + 1 < sm.ns && j >= sm.es[d + 1]) ++d;
          }
          cc[r] += d << sm.sbits;
        }
      }
    }
    if (na > 0) {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int k = r * kThreads + tid;
        ee[r] = rp[i0 + 1 + (k < na ? k : na - 1)];
      }
    }
    if (nz > 0) {
#pragma unroll
      for (int r = 0; r < IPT; ++r) xv[r] = x[cc[r]];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int k = r * kThreads + tid;
        if (k < nz) s_prod[k] = xv[r] * V(vv[r]);
      }
    }
    if (na > 0) {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int k = r * kThreads + tid;
        if (k < na) s_end[k] = ee[r] - j0;
      }
    }
  }
  const bool mid_row = i0 < n && rp[i0] < j0;
  const double tk = *tele;
  __syncthreads();

  // This thread's items [d, dend) of the workgroup's merge sequence.
  const int32_t tot = na + nz;
  int32_t d = tid * IPT < tot ? tid * IPT : tot;
  const int32_t dend = d + IPT < tot ? d + IPT : tot;
  int32_t lo = d - nz > 0 ? d - nz : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const int32_t m = (lo + hi) >> 1;
    if (s_end[m] <= d - m - 1)
      lo = m + 1;
    else
      hi = m;
  }
  int32_t ti = lo, tj = d - lo;
  // Raw mode stages its pairs' partials in LDS and stores them together at
  // the end (one coalesced store per 64 pairs instead of one per pair).  A
  // pair is never empty, so when a thread ends the k-th pair it began
  // itself it has consumed at least k + 1 products: the k-th partial goes
  // to s_prod[tj0 + k], a product slot this thread has already read.
  const int32_t tj0 = tj;
  int32_t nstaged = 0;

  Acc acc{}, first{};
  int32_t first_row = -1;
  double ysum = 0.0;
  for (; d < dend; ++d) {
    if (ti < na && s_end[ti] <= tj) {
      if (first_row < 0) {
        first_row = ti;
        first = acc;
      } else if constexpr (kRaw) {
        s_prod[tj0 + nstaged] = Form<V>::part(acc);
        ++nstaged;
      } else {
        const V yv = Form<V>::finish(acc, c, tk);
        y[i0 + ti] = yv;
        ysum += double(yv);
      }
      acc = Acc{};
      ++ti;
    } else {
      acc.add(s_prod[tj]);
      ++tj;
    }
  }

  // Segmented inclusive scan of the threads' open-row partials, keyed by the
  // open row (non-decreasing in thread order, so equal keys are contiguous):
  // shuffles inside each wave, then the tails of earlier waves.
  const int32_t key = i0 + ti;
  Acc v = acc;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const Acc vu = shfl_up_acc(v, o);
    const int32_t ku = __shfl_up(key, o, kWave);
    if (lane >= o && ku == key) v = merge(vu, v);
  }
  if (lane == kWave - 1) {
    s_wtail[w] = v;
    s_wlast[w] = key;
  }
  if (lane == 0) s_wfirst[w] = key;
  __syncthreads();
  {
    Acc before{};
    for (int q = w - 1; q >= 0; --q) {
      if (s_wlast[q] != key) break;
      before = merge(s_wtail[q], before);
      if (s_wfirst[q] != key) break;
    }
    v = merge(before, v);
  }
  s_pre[tid] = v;
  __syncthreads();

  typename Form<V>::Part first_part{};
  bool has_first = false;
  if (first_row >= 0) {
    // The first row this thread ends is the row thread tid-1 left open, so
    // its earlier part is that thread's segmented prefix.
    const int32_t R = i0 + first_row;
    const Acc sum = tid > 0 ? merge(s_pre[tid - 1], first) : first;
    if (R == i0 && mid_row) {
      blk_head[b] = sum;  // row began in an earlier workgroup: completed later
    } else if constexpr (kRaw) {
      first_part = Form<V>::part(sum);
      has_first = true;
    } else {
      const V yv = Form<V>::finish(sum, c, tk);
      y[R] = yv;
      ysum += double(yv);
    }
  }
  if (tid == kThreads - 1) blk_carry[b] = c1.x < n ? v : Acc{};
  if constexpr (kRaw) {
    // Every completed pair of the tile (local rows [0, na), less a first
    // row carried in from the previous tile) has its partial in LDS: the
    // first one a thread ends in s_pre[tid] (free once every thread has read
    // its neighbour's prefix), the others in the thread's consumed product
    // slots; s_end, free after the walk, maps each row to its slot.
    using Part = typename Form<V>::Part;
    Part *s_first = reinterpret_cast<Part *>(s_pre);
    __syncthreads();
    if (has_first) {
      s_first[tid] = first_part;
      s_end[first_row] = -(tid + 1);
    }
    for (int32_t k = 0; k < nstaged; ++k) s_end[first_row + 1 + k] = tj0 + k;
    __syncthreads();
    for (int32_t r = tid; r < na; r += kThreads) {
      if (r == 0 && mid_row) continue;
      const int32_t loc = s_end[r];
      part[i0 + r] = loc >= 0 ? Part(s_prod[loc]) : s_first[-loc - 1];
    }
  } else {
    const double bs = block_sum256(ysum, s_red);
    if (tid == 0) blk_ysum[b] = bs;
  }
}

// ------------------------------------------------------------------ SpMM
// Y = c * A^T X + t_j per column j, X and Y n x k row-major, k = nrhs in
// 2..64 independent PageRank vectors on one matrix.  The workgroup stages
// the same merge-path item range as the SpMV (columns, values, row ends),
// but each item is processed by a group of G = nextpow2(k) lanes, lane l
// owning right-hand side l: a non-zero gathers the k consecutive values of
// row col of X (one 128 B line at k = 32), so the gather moves only useful
// bytes.  Each group walks its items in order, gathering the next U
// non-zeros' rows while it adds up the current U.  Carries between groups and workgroups, the per-column FP64
// sum(y) and the per-column teleport scalar work as in the SpMV.
template <typename V, int G>
__global__ __launch_bounds__(kThreads) void k_spmm(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const V *__restrict__ val,
    const V *__restrict__ x, V *__restrict__ y, int32_t n, int32_t k,
    const int2 *__restrict__ coord, double c, const double *__restrict__ tele,
    double *__restrict__ blk_ysum, typename Form<V>::Acc *__restrict__ blk_carry,
    typename Form<V>::Acc *__restrict__ blk_head) {
  using Acc = typename Form<V>::Acc;
  constexpr int NG = kThreads / G;  // lane groups per workgroup
  constexpr int P = kItems / NG;    // merge items per group
  constexpr int U = 8;              // gathers in flight per lane
  __shared__ int32_t s_end[kItems];
  __shared__ int32_t s_col[kItems];
  __shared__ V s_val[kItems];
  __shared__ Acc s_carry[kThreads];
  __shared__ int32_t s_key[NG];
  __shared__ double s_ysum[kThreads];

  const int b = blockIdx.x, tid = threadIdx.x;
  const int g = tid / G, l = tid % G;
  const bool active = l < k;
  const int2 c0 = coord[b], c1 = coord[b + 1];
  const int32_t i0 = c0.x, j0 = c0.y;
  const int32_t na = c1.x - c0.x, nz = c1.y - c0.y;
  for (int q = tid; q < nz; q += kThreads) {
    s_col[q] = __builtin_nontemporal_load(col + j0 + q);
    s_val[q] = __builtin_nontemporal_load(val + j0 + q);
  }
  for (int q = tid; q < na; q += kThreads) s_end[q] = rp[i0 + 1 + q] - j0;
  const bool mid_row = i0 < n && rp[i0] < j0;
  const double tk = active ? tele[l] : 0.0;
  __syncthreads();

  const int32_t tot = na + nz;
  int32_t d = g * P < tot ? g * P : tot;
  const int32_t dend = d + P < tot ? d + P : tot;
  int32_t lo = d - nz > 0 ? d - nz : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const int32_t m = (lo + hi) >> 1;
    if (s_end[m] <= d - m - 1)
      lo = m + 1;
    else
      hi = m;
  }
  int32_t ti = lo, tj = d - lo;

  Acc acc{}, first{};
  int32_t first_row = -1;
  double ysum = 0.0;
  // Gathers of U non-zeros from tj on (indices clamped into the tile).
  auto gather = [&](V *dst, int32_t from) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t q = from + u < nz ? from + u : nz - 1;
      dst[u] = (active && q >= 0) ? x[int64_t(s_col[q]) * k + l] : V(0);
    }
  };
  // A batch that does not end the group's items consumes exactly U
  // non-zeros, so the next batch starts U further: its gathers are issued
  // before the current batch is added up.
  V buf[U], nxt[U];
  gather(buf, tj);
  while (d < dend) {
    gather(nxt, tj + U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      while (d < dend && ti < na && s_end[ti] <= tj) {
        if (first_row < 0) {
          first_row = ti;
          first = acc;
        } else if (active) {
          const V yv = Form<V>::finish(acc, c, tk);
          y[int64_t(i0 + ti) * k + l] = yv;
          ysum += double(yv);
        }
        acc = Acc{};
        ++ti;
        ++d;
      }
      if (d < dend) {
        acc.add(buf[u] * s_val[tj]);
        ++tj;
        ++d;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) buf[u] = nxt[u];
  }
  s_carry[tid] = acc;
  if (l == 0) s_key[g] = i0 + ti;
  __syncthreads();

  if (first_row >= 0 && active) {
    const int32_t R = i0 + first_row;
    int gg = g - 1;
    while (gg >= 0 && s_key[gg] == R) --gg;
    Acc sum{};
    for (int q = gg + 1; q < g; ++q) sum = merge(sum, s_carry[q * G + l]);
    sum = merge(sum, first);
    if (R == i0 && mid_row) {
      blk_head[int64_t(b) * k + l] = sum;
    } else {
      const V yv = Form<V>::finish(sum, c, tk);
      y[int64_t(R) * k + l] = yv;
      ysum += double(yv);
    }
  }
  if (g == NG - 1 && active) {
    Acc sum{};
    if (c1.x < n) {
      int gg = NG - 1;
      while (gg >= 0 && s_key[gg] == c1.x) --gg;
      for (int q = gg + 1; q < NG; ++q) sum = merge(sum, s_carry[q * G + l]);
    }
    blk_carry[int64_t(b) * k + l] = sum;
  }
  s_ysum[tid] = ysum;
  __syncthreads();
  if (tid < k) {
    double t = 0.0;
    for (int q = 0; q < NG; ++q) t += s_ysum[q * G + tid];
    blk_ysum[int64_t(b) * k + tid] = t;
  }
}

// Per-column completion of rows spanning workgroups and per-column sum(y).
template <typename V>
__global__ __launch_bounds__(kThreads) void k_finish_mm(
    V *__restrict__ y, int32_t nb, int32_t k, int32_t G, const int2 *__restrict__ coord,
    const uint8_t *__restrict__ closes, const int32_t *__restrict__ carry_row,
    const typename Form<V>::Acc *__restrict__ blk_carry,
    const typename Form<V>::Acc *__restrict__ blk_head, const double *__restrict__ blk_ysum,
    double c, const double *__restrict__ tele_in, double *part, uint32_t *counter, double w,
    double *sum_out, double *tele_out) {
  using Acc = typename Form<V>::Acc;
  __shared__ double sh[kThreads];
  __shared__ bool is_last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int slots = kThreads / G, slot = tid / G, j = tid % G;
  const int64_t lo = int64_t(g) * kFinishPer;
  const int64_t hi = lo + kFinishPer < nb ? lo + kFinishPer : nb;
  double acc = 0.0;
  if (j < k) {
    const double tk = tele_in[j];
    for (int64_t b = lo + slot; b < hi; b += slots) {
      double v = blk_ysum[b * k + j];
      if (closes[b]) {
        const int32_t R = coord[b].x;
        int64_t q = b - 1;
        while (q >= 0 && carry_row[q] == R) --q;
        Acc sum{};
        for (int64_t t = q + 1; t < b; ++t) sum = merge(sum, blk_carry[t * k + j]);
        sum = merge(sum, blk_head[b * k + j]);
        const V yv = Form<V>::finish(sum, c, tk);
        y[int64_t(R) * k + j] = yv;
        v += double(yv);
      }
      acc += v;
    }
  }
  sh[tid] = acc;
  __syncthreads();
  if (tid < k) {
    double t = 0.0;
    for (int q = 0; q < slots; ++q) t += sh[q * G + tid];
    part[int64_t(g) * k + tid] = t;
    __threadfence();
  }
  __syncthreads();
  if (tid == 0) is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (is_last) {
    __threadfence();
    if (tid < k) {
      double t = 0.0;
      for (int q = 0; q < int(gridDim.x); ++q) t += load_acquire(part + int64_t(q) * k + tid);
      if (sum_out) sum_out[tid] = t;
      tele_out[tid] = w * t;
    }
    if (tid == 0) *counter = 0u;
  }
}

// Per-column sum of the n x k starting block.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_sum0_mm(const V *__restrict__ r, int64_t n, int32_t k,
                                                      int32_t G, int64_t chunk, double *part,
                                                      uint32_t *counter, double w, double *sum_out,
                                                      double *tele_out) {
  __shared__ double sh[kThreads];
  __shared__ bool is_last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int slots = kThreads / G, slot = tid / G, j = tid % G;
  const int64_t lo = int64_t(g) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  if (j < k)
    for (int64_t i = lo + slot; i < hi; i += slots) acc += double(r[i * k + j]);
  sh[tid] = acc;
  __syncthreads();
  if (tid < k) {
    double t = 0.0;
    for (int q = 0; q < slots; ++q) t += sh[q * G + tid];
    part[int64_t(g) * k + tid] = t;
    __threadfence();
  }
  __syncthreads();
  if (tid == 0) is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (is_last) {
    __threadfence();
    if (tid < k) {
      double t = 0.0;
      for (int q = 0; q < int(gridDim.x); ++q) t += load_acquire(part + int64_t(q) * k + tid);
      if (sum_out) sum_out[tid] = t;
      tele_out[tid] = w * t;
    }
    if (tid == 0) *counter = 0u;
  }
}

// Completes rows that span workgroups, then reduces sum(y) in a fixed
// order: per finish-workgroup partials, and the last workgroup to arrive
// adds those partials, stores sum(y) and the next teleport scalar.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_finish(
    V *__restrict__ y, int32_t nb, const int2 *__restrict__ coord,
    const uint8_t *__restrict__ closes, const int32_t *__restrict__ carry_row,
    const typename Form<V>::Acc *__restrict__ blk_carry,
    const typename Form<V>::Acc *__restrict__ blk_head, const double *__restrict__ blk_ysum,
    double c, const double *__restrict__ tele_in, double *part, uint32_t *counter, double w,
    double *sum_out, double *tele_out) {
  using Acc = typename Form<V>::Acc;
  __shared__ double sh[4];
  __shared__ bool is_last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const double tk = *tele_in;
  const int64_t lo = int64_t(g) * kFinishPer;
  const int64_t hi = lo + kFinishPer < nb ? lo + kFinishPer : nb;
  double acc = 0.0;
  for (int64_t b = lo + tid; b < hi; b += kThreads) {
    double v = blk_ysum[b];
    if (closes[b]) {
      const int32_t R = coord[b].x;
      int64_t q = b - 1;
      while (q >= 0 && carry_row[q] == R) --q;
      Acc sum{};
      for (int64_t k = q + 1; k < b; ++k) sum = merge(sum, blk_carry[k]);
      sum = merge(sum, blk_head[b]);
      const V yv = Form<V>::finish(sum, c, tk);
      y[R] = yv;
      v += double(yv);
    }
    acc += v;
  }
  const double tot = block_sum256(acc, sh);
  if (tid == 0) {
    part[g] = tot;
    __threadfence();
    is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (is_last) {
    __threadfence();
    double a = 0.0;
    for (int k = tid; k < int(gridDim.x); k += kThreads) a += load_acquire(part + k);
    const double s = block_sum256(a, sh);
    if (tid == 0) {
      if (sum_out) *sum_out = s;
      *tele_out = w * s;
      *counter = 0u;
    }
  }
}

// sum(r_0) with the same two-level fixed-order reduction.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_sum0(const V *__restrict__ r, int64_t n,
                                                   int64_t chunk, double *part, uint32_t *counter,
                                                   double w, double *sum_out, double *tele_out) {
  __shared__ double sh[4];
  __shared__ bool is_last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int64_t lo = int64_t(g) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (int64_t i = lo + tid; i < hi; i += kThreads) acc += double(r[i]);
  const double tot = block_sum256(acc, sh);
  if (tid == 0) {
    part[g] = tot;
    __threadfence();
    is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (is_last) {
    __threadfence();
    double a = 0.0;
    for (int k = tid; k < int(gridDim.x); k += kThreads) a += load_acquire(part + k);
    const double s = block_sum256(a, sh);
    if (tid == 0) {
      if (sum_out) *sum_out = s;
      *tele_out = w * s;
      *counter = 0u;
    }
  }
}

// ------------------------------------------------------------ initial r
__global__ __launch_bounds__(256) void k_init_sum(int64_t n, int32_t nrhs, uint32_t k0,
                                                  uint32_t k1, unsigned long long *ksum) {
  const int32_t j = blockIdx.y;
  unsigned long long acc = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const U4 w = philox10(U4{uint32_t(i), uint32_t(j), 0u, 2u}, k0, k1);
    acc += w.x >> 8;
  }
  // One atomic per workgroup (integer sums, so the order does not matter).
  __shared__ unsigned long long sh[4];
  acc = wave_sum(acc);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = sh[0] + sh[1] + sh[2] + sh[3];
    if (t) atomicAdd(ksum + j, t);
  }
}

template <typename V>
__global__ __launch_bounds__(256) void k_init_write(int64_t n, int32_t nrhs, uint32_t k0,
                                                    uint32_t k1,
                                                    const unsigned long long *__restrict__ ksum,
                                                    V *__restrict__ r) {
  const int32_t j = blockIdx.y;
  const unsigned long long K = ksum[j];
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const U4 w = philox10(U4{uint32_t(i), uint32_t(j), 0u, 2u}, k0, k1);
    const double q = K ? double(w.x >> 8) / double(K) : 1.0 / double(n);
    r[i * nrhs + j] = V(q);
  }
}

// ------------------------------------------------------ vertex relabelling
// Graph500-style random labels scatter the high-degree sources over all of
// r, so nearly every gather r[u] misses L2 and moves a 128 B line.  When the
// caller passes per-vertex weights (pp_filter's d_out: the number of kept
// edges leaving u, i.e. how often r[u] is gathered), K3 relabels vertices by
// decreasing floor(log2(weight + 1)) -- a stable bucket order, ties in label
// order -- and iterates on P A^T P^T.  Hot sources then share cache lines.
// Rows are permuted with the same map, so x and y stay in one numbering; r
// is permuted in before the first iteration and out after the last.

// Bucket of a vertex: clz(weight + 1) for a weight > 0 (0 .. 30), so
// heavier vertices sort first; weights <= 0 come after every positive one,
// those with entries in their row of A^T (bucket 31) before those without
// (bucket 32): in the degree-scaled form the latter are isolated, no entry
// gathers them and nothing adds into their row.
constexpr int kBuckets = 33;
__device__ __forceinline__ uint32_t vertex_bucket(int32_t w, int32_t rowlen) {
  if (w > 0) return uint32_t(__clz(int(uint32_t(w) + 1u)));
  return rowlen > 0 ? 31u : 32u;
}

// The new order is a stable counting sort of the vertices by bucket, in
// blocks of kRelTile vertices; each wave takes a contiguous quarter of its
// block, so wave-ballot ranks (in vertex order) keep the sort stable.
constexpr int kRelTile = 4096;
constexpr int kRelPer = kRelTile / kThreads;

// Bucket counts of each block, bucket-major: hist[c * nblk + b].
__global__ __launch_bounds__(kThreads) void k_bucket_count(const int32_t *__restrict__ w,
                                                           const int32_t *__restrict__ rp,
                                                           int32_t n, int32_t nblk,
                                                           uint32_t *__restrict__ hist) {
  constexpr int kWaves = kThreads / kWave;
  __shared__ uint32_t wh[kWaves][64];
  const int tid = threadIdx.x, wv = tid / kWave, lane = lane_id();
  (&wh[0][0])[tid] = 0u;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRelTile + wv * (kRelTile / kWaves);
  int32_t ww[kRelPer], len[kRelPer];
#pragma unroll
  for (int r = 0; r < kRelPer; ++r) {
    const int64_t v = base + r * kWave + lane;
    const int64_t vc = v < n ? v : 0;
    ww[r] = w[vc];
    len[r] = rp[vc + 1] - rp[vc];
  }
#pragma unroll
  for (int r = 0; r < kRelPer; ++r)
    wave_digit_rank(vertex_bucket(ww[r], len[r]), base + r * kWave + lane < n, 6, wh[wv]);
  __syncthreads();
  if (tid < kBuckets) {
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) t += wh[q][tid];
    hist[int64_t(tid) * nblk + blockIdx.x] = t;
  }
}

// off = the exclusive scan of hist: vertex v of block b goes to p = off[c *
// nblk + b] + (its rank among the block's vertices of bucket c).  Writes
// order[p] = v, lab[v] = (p, weight of v), wnew[p] = weight of v and the row
// lengths in the new order (into rp2, scanned afterwards).  Reads are in
// vertex order; each block's writes in the new order are one run per bucket.
__global__ __launch_bounds__(kThreads) void k_bucket_scatter(
    const int32_t *__restrict__ w, const int32_t *__restrict__ rp, int32_t n, int32_t nblk,
    const uint32_t *__restrict__ off, int32_t *__restrict__ order, int2 *__restrict__ lab,
    int32_t *__restrict__ wnew, uint32_t *__restrict__ len2) {
  constexpr int kWaves = kThreads / kWave;
  __shared__ uint32_t wh[kWaves][64];
  __shared__ uint32_t s_off[kBuckets];
  const int tid = threadIdx.x, wv = tid / kWave, lane = lane_id();
  (&wh[0][0])[tid] = 0u;
  if (tid < kBuckets) s_off[tid] = off[int64_t(tid) * nblk + blockIdx.x];
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRelTile + wv * (kRelTile / kWaves);
  int32_t ww[kRelPer], r0[kRelPer], r1[kRelPer];
  uint32_t rank[kRelPer];
#pragma unroll
  for (int r = 0; r < kRelPer; ++r) {
    const int64_t v = base + r * kWave + lane;
    const int64_t vc = v < n ? v : 0;
    ww[r] = w[vc];
    r0[r] = rp[vc];
    r1[r] = rp[vc + 1];
  }
#pragma unroll
  for (int r = 0; r < kRelPer; ++r)
    rank[r] = wave_digit_rank(vertex_bucket(ww[r], r1[r] - r0[r]), base + r * kWave + lane < n,
                              6, wh[wv]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRelPer; ++r) {
    const int64_t v = base + r * kWave + lane;
    if (v >= n) continue;
    const uint32_t c = vertex_bucket(ww[r], r1[r] - r0[r]);
    uint32_t p = s_off[c] + rank[r];
    for (int q = 0; q < wv; ++q) p += wh[q][c];
    order[p] = int32_t(v);
    lab[v] = make_int2(int32_t(p), ww[r]);
    wnew[p] = ww[r];
    len2[p] = uint32_t(r1[r] - r0[r]);
  }
}

// Cache in front of lab[] for the heaviest vertices: one 8-byte slot per
// hash bucket for the heaviest vertex hashed there, packing (tag, new
// label, weight).  hot_mix is a bijection of 32-bit words, so the bucket
// (its low lg bits) and the tag (the other 32 - lg bits) identify the
// vertex; the new label takes nbits and the weight the remaining bits, and
// weight 0 marks an empty slot (the cache holds weights >= 8 only).  A
// lookup reads the slot and falls back to lab[u] when the slot holds
// another vertex; results never depend on what the cache holds.  Packing
// doubles the vertices a 2 MiB table (one XCD's L2 half) holds.
struct Hot2 {
  const uint64_t *tab;
  uint32_t mask;
  int32_t lg, nbits;
};

__device__ __forceinline__ int2 hot2_get(Hot2 h, const int2 *__restrict__ lab, int32_t u) {
  const uint32_t m = hot_mix(uint32_t(u));
  const uint64_t e = h.tab[m & h.mask];
  const int tb = 32 - h.lg;
  const uint64_t rest = e >> tb;
  const uint32_t wgt = uint32_t(rest >> h.nbits);
  if (wgt != 0u && uint32_t(e & ((1ull << tb) - 1ull)) == (m >> h.lg))
    return make_int2(int32_t(rest & ((1ull << h.nbits) - 1ull)), int32_t(wgt));
  return lab[u];
}

// kN lookups at once, every read issued before any is used: first all slot
// reads, then all fallback reads (a hit reads lab[0] instead, so the read is
// unconditional and the hit lanes of a wave share one line).  A read under
// a per-lane condition would be waited for before the next one is issued.
template <int kN>
__device__ __forceinline__ void hot2_get_n(Hot2 h, const int2 *__restrict__ lab,
                                           const int32_t (&u)[kN], int2 (&out)[kN]) {
  const int tb = 32 - h.lg;
  uint64_t e[kN];
  uint32_t m[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    m[i] = hot_mix(uint32_t(u[i]));
    e[i] = h.tab[m[i] & h.mask];
  }
  bool hit[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const uint32_t wgt = uint32_t((e[i] >> tb) >> h.nbits);
    hit[i] = wgt != 0u && uint32_t(e[i] & ((1ull << tb) - 1ull)) == (m[i] >> h.lg);
  }
  int2 fb[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) fb[i] = lab[hit[i] ? 0 : u[i]];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    const uint64_t rest = e[i] >> tb;
    out[i] = hit[i] ? make_int2(int32_t(rest & ((1ull << h.nbits) - 1ull)),
                                int32_t(uint32_t(rest >> h.nbits)))
                    : fb[i];
  }
}

// Winners (weight << 32 | u, 0 = empty) -> packed slots; a winner whose
// weight does not fit the slot's weight bits leaves the slot empty.
__global__ __launch_bounds__(256) void k_hot2_fill(const uint64_t *__restrict__ win,
                                                   const int2 *__restrict__ lab,
                                                   uint64_t *__restrict__ tab, int32_t lg,
                                                   int32_t nbits) {
  const uint32_t slots = 1u << lg;
  const int tb = 32 - lg;
  const int wbits = 64 - tb - nbits;
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < slots; k += gridDim.x * 256) {
    const uint64_t e = win[k];
    uint64_t slot = 0;
    if (e) {
      const uint32_t u = uint32_t(e);
      const int2 l = lab[u];
      const uint64_t w = uint64_t(uint32_t(l.y));
      if (l.y > 0 && (wbits >= 32 || w < (1ull << wbits)))
        slot = uint64_t(hot_mix(u) >> lg) | (uint64_t(uint32_t(l.x)) << tb) |
               (w << (tb + nbits));
    }
    tab[k] = slot;
  }
}

// rp2[n] = the entry count; npos[0] = the vertices of weight > 0, which
// take the new labels [0, npos[0]) (the start of bucket 31 in the new
// order); npos[1] = the start of bucket 32 (weight <= 0, empty row).
__global__ void k_set_total(int32_t *rp2, int32_t n, const int64_t *total,
                            const uint32_t *__restrict__ start31,
                            const uint32_t *__restrict__ start32, uint32_t *npos) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rp2[n] = int32_t(*total);
    npos[0] = *start31;
    npos[1] = *start32;
  }
}

// Entries of the relabelled matrix, one thread per entry q of the new
// layout (balanced by the same merge-path partition the SpMV uses): its row
// p is found in the workgroup's staged row ends, its source position is the
// same offset inside old row order[p], its column is newlabel[col].
template <typename V>
__global__ __launch_bounds__(kThreads) void k_relabel_copy(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const V *__restrict__ val,
    const int32_t *__restrict__ order, const int2 *__restrict__ lab, Hot2 hot,
    const int32_t *__restrict__ rp2, int32_t n, const int2 *__restrict__ coord,
    int32_t *__restrict__ col2, V *__restrict__ val2) {
  __shared__ int32_t s_end[kItemsMax];
  __shared__ int32_t s_old[kItemsMax + 1];
  __shared__ int32_t s_new[kItemsMax + 1];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int2 c0 = coord[b], c1 = coord[b + 1];
  const int32_t i0 = c0.x, j0 = c0.y, na = c1.x - c0.x, nz = c1.y - c0.y;
  for (int k = tid; k <= na; k += kThreads) {
    const int32_t row = i0 + k;
    if (row < n) {
      s_new[k] = rp2[row];
      s_old[k] = rp[order[row]];
    }
    if (k < na) s_end[k] = rp2[row + 1];
  }
  __syncthreads();
  for (int32_t q = j0 + tid; q < j0 + nz; q += kThreads) {
    int32_t lo = 0, hi = na;
    while (lo < hi) {
      const int32_t m = (lo + hi) >> 1;
      if (s_end[m] <= q)
        lo = m + 1;
      else
        hi = m;
    }
    const int32_t src = s_old[lo] + (q - s_new[lo]);
    col2[q] = hot2_get(hot, lab, col[src]).x;
    val2[q] = val[src];
  }
}

// Rows of width k: dst row p <- src row order[p] (in), dst row order[p] <-
// src row p (out); order null keeps the labels.  The iterations' side of
// the copy is stored in column tiles of T right-hand sides (T >= k: plain
// row-major): tile t holds columns [tT, tT + Tt), Tt = min(T, k - tT), as an
// n x Tt row-major block starting at element n * tT.
__device__ __forceinline__ int64_t tiled_index(int64_t p, int32_t j, int64_t n, int32_t k,
                                               int32_t T) {
  const int32_t t = j / T, jj = j - t * T;
  const int32_t Tt = k - t * T < T ? k - t * T : T;
  return n * t * T + p * Tt + jj;
}

template <typename V>
__global__ __launch_bounds__(256) void k_permute_in(const V *__restrict__ src,
                                                    const int32_t *__restrict__ order, int32_t n,
                                                    int32_t k, int32_t T, V *__restrict__ dst) {
  const int64_t total = int64_t(n) * k;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int64_t p = e / k;
    const int32_t j = int32_t(e - p * k);
    dst[tiled_index(p, j, n, k, T)] = src[int64_t(order ? order[p] : int32_t(p)) * k + j];
  }
}

// Degree-scaled form, one right-hand side: dst[p] = src[order[p]] / d[p]
// (0 where d[p] <= 0: such a vertex has no entries in its column).
template <typename V>
__global__ __launch_bounds__(256) void k_permute_in_scaled(const V *__restrict__ src,
                                                           const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ d,
                                                           int32_t n, V *__restrict__ dst) {
  for (int32_t p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
    const int32_t dp = d[p];
    dst[p] = dp > 0 ? V(double(src[order[p]]) / double(dp)) : V(0);
  }
}

template <typename V>
__global__ __launch_bounds__(256) void k_permute_out(const V *__restrict__ src,
                                                     const int32_t *__restrict__ order, int32_t n,
                                                     int32_t k, int32_t T, V *__restrict__ dst) {
  const int64_t total = int64_t(n) * k;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int64_t p = e / k;
    const int32_t j = int32_t(e - p * k);
    dst[int64_t(order ? order[p] : int32_t(p)) * k + j] = src[tiled_index(p, j, n, k, T)];
  }
}

// --------------------------------------------- column-segmented iteration
// CSR segmenting (Zhang, Kiriansky et al., "Making caches work for graph
// analytics", IEEE BigData 2017).  The columns of the iterate matrix are cut
// into slabs of 2^sbits vertices.  Entries are stored slab by slab, each
// slab in row order (entries of a row keep their order), so one pass over a
// slab gathers only from a range of r small enough to stay in L2.  Every
// (slab, row) run of entries is a "pair"; the pairs form a CSR of their own
// that the merge-path SpMV walks in raw mode, writing one partial sum per
// pair.  A combine pass then adds each row's partials in slab order and
// applies c * sum + t.  Sums stay in a fixed order, so results are
// reproducible; they differ from the unsegmented order only by rounding.
constexpr int kSegTile = kThreads * 4;    // merge items per build tile
constexpr int kSegPer = kSegTile / kThreads;
constexpr int kMaxSlabs = 256;
constexpr int kCombItems = kThreads * 8;  // rows + pairs per combine workgroup

__device__ __forceinline__ int32_t row_of(const int32_t *s_end, int32_t na, int32_t e) {
  int32_t lo = 0, hi = na;
  while (lo < hi) {
    const int32_t m = (lo + hi) >> 1;
    if (s_end[m] <= e)
      lo = m + 1;
    else
      hi = m;
  }
  return lo;
}

constexpr int kMaskWords = kMaxSlabs / 32;

// Slab of column c: c >> sbits, the columns from the last slab on all in
// the last one (a relabelled matrix puts the vertices of weight <= 0, which
// normally have no entries, past the last slab).
__device__ __forceinline__ uint32_t slab_of(int32_t c, int32_t sbits, int32_t ns) {
  const uint32_t d = uint32_t(c) >> sbits;
  return d < uint32_t(ns) ? d : uint32_t(ns - 1);
}

// One build tile (kSegTile merge items of the matrix) ordered stably by
// slab: ranks come from wave ballots in entry order, so inside a slab the
// entries keep their order and rows ascend.  Every (slab, row) run of the
// tile starts a pair, except the run of the tile's first row in a slab
// where that row already had entries in an earlier tile (cont).
//
// Count pass (kScatter false), per slab d of tile b: entries -> ecnt[b *
// ns + d], runs -> pcnt[...]; slab masks of the tile's first row ->
// fmask[b], of the row left open at its end -> lmask[b].  With kRelabel the
// tile is one of the relabelled matrix (row pointers rp): the count pass
// also produces its entries, new row p taking old row order[p] of (rp0,
// col0, val0) with every column mapped through newlabel, into (col, val).
// Scatter pass: ecnt / pcnt hold the offsets in slab-major, then tile,
// order (still stored tile by tile) and fmask the cont masks.  The tile is staged in LDS in slab order
// so that one slab's run is stored contiguously; a pair start also stores
// its entry position and row (prp, pair_row).
//
// E is the stored entry type: V (the matrix values) or, in the degree-scaled
// form, uint8_t: the integer count k of the entry, with the entry's value
// k / w[u] carried by the ranks (the iterations gather r_u / w[u]).  The
// relabelling count pass derives k from the value and the weight of its
// column, k = rint(val * w), and accepts the entry only if k is in [1, 255]
// and V(k / w) reproduces the value bit for bit (the IEEE FP64 quotient,
// rounded to FP32 in the FP32 form); any other entry sets *bad, and the
// caller falls back to storing values.  The count pass also keeps the
// largest new column (bad[1]); with packed set, the scatter pass stores
// each count entry as one word, its column inside the slab (< 2^24) in the
// low 24 bits and the count in the high 8, into seg_col alone.
struct RelabelSrc {
  const int32_t *rp0, *col0, *order;
  const int2 *lab;   // (new label, weight) of every old label
  const void *val0;
  Hot2 hot;          // cache of lab for the heaviest vertices
  uint32_t *bad;     // [0] set when an entry is not count / weight (scaled form);
                     // [1] largest new column of the count form's entries
};

template <typename V, typename E, bool kScatter, bool kRelabel>
__global__ __launch_bounds__(kThreads) void k_seg_tile(
    const int32_t *__restrict__ rp, int32_t *__restrict__ col, E *__restrict__ val, int32_t n,
    RelabelSrc rs, const int2 *__restrict__ coord, int32_t sbits, int32_t ns, int32_t dbits,
    int32_t ntiles, uint32_t *__restrict__ ecnt, uint32_t *__restrict__ pcnt,
    uint32_t *__restrict__ fmask, uint32_t *__restrict__ lmask, int32_t *__restrict__ seg_col,
    E *__restrict__ seg_val, int32_t *__restrict__ prp, int32_t *__restrict__ pair_row,
    int32_t packed) {
  constexpr bool kCount = !std::is_same<E, V>::value;
  static_assert(!(kScatter && kRelabel), "relabelling happens in the count pass");
  constexpr int kWaves = kThreads / kWave;
  constexpr int kChunks = kSegTile / kWave;   // 64 consecutive slots each
  __shared__ uint32_t wh[kWaves][kMaxSlabs];
  __shared__ uint32_t s_toff[kMaxSlabs], s_goff[kMaxSlabs], s_poff[kMaxSlabs];
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_cont[kMaskWords];
  __shared__ uint64_t s_bal[kChunks];          // pair starts of each chunk
  __shared__ uint32_t s_pre[kChunks + 1];      // pair starts before each chunk
  __shared__ int32_t s_end[kSegTile];   // row ends; then the staged local rows
  __shared__ int32_t s_col[kSegTile];
  __shared__ E s_val[kScatter ? kSegTile : 1];
  __shared__ int32_t s_src[kRelabel ? kSegTile + 1 : 1];   // old row start - new row start
  for (int i = threadIdx.x; i < kWaves * kMaxSlabs; i += kThreads) (&wh[0][0])[i] = 0u;
  const int b = blockIdx.x, tid = threadIdx.x, w = tid / kWave, lane = lane_id();
  const int2 c0 = coord[b], c1 = coord[b + 1];
  const int32_t i0 = c0.x, j0 = c0.y, na = c1.x - c0.x, nz = c1.y - c0.y;
  for (int k = tid; k < na; k += kThreads) s_end[k] = rp[i0 + 1 + k] - j0;
  if constexpr (kRelabel) {
    for (int k = tid; k <= na; k += kThreads)
      if (i0 + k < n) s_src[k] = rs.rp0[rs.order[i0 + k]] - rp[i0 + k];
  }
  if (kScatter && tid < kMaskWords) s_cont[tid] = fmask[int64_t(b) * kMaskWords + tid];
  __syncthreads();
  int32_t cc[kSegPer], rr[kSegPer];
  E vv[kSegPer];
  V v0[kRelabel ? kSegPer : 1];
  uint32_t rank[kSegPer];
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const int32_t e = w * (kSegTile / kWaves) + r * kWave + lane;
    const bool valid = e < nz;
    rr[r] = valid ? row_of(s_end, na, e) : 0;
    if constexpr (kRelabel) {
      // Unconditional reads (entry 0 for lanes past the end), so that they
      // are all in flight together.
      const int32_t src = valid ? j0 + e + s_src[rr[r]] : 0;
      const int32_t c0v = rs.col0[src];
      const V v0v = static_cast<const V *>(rs.val0)[src];
      cc[r] = valid ? c0v : 0;
      v0[r] = valid ? v0v : V(0);
    } else {
      cc[r] = valid ? col[j0 + e] : 0;
      if constexpr (kScatter) vv[r] = valid ? val[j0 + e] : E(0);
    }
  }
  if constexpr (kRelabel) {
    bool bad = false;
    int2 lk[kSegPer];
    hot2_get_n<kSegPer>(rs.hot, rs.lab, cc, lk);   // lanes past the end look up column 0
#pragma unroll
    for (int r = 0; r < kSegPer; ++r) {
      vv[r] = E(0);
      if (w * (kSegTile / kWaves) + r * kWave + lane < nz) {
        const int2 l = lk[r];
        cc[r] = l.x;
        if constexpr (kCount) {
          const double wd = double(l.y);
          const double k = rint(double(v0[r]) * wd);
          const bool ok = l.y > 0 && k >= 1.0 && k <= 255.0 && V(k / wd) == v0[r];
          bad = bad || !ok;
          vv[r] = ok ? E(k) : E(0);
        } else {
          vv[r] = v0[r];
        }
      }
    }
    if constexpr (kCount) {
      const uint64_t any_bad = __ballot(bad);
      if (any_bad && lane == 0) atomicOr(rs.bad, 1u);
      int32_t cmax = 0;
#pragma unroll
      for (int r = 0; r < kSegPer; ++r)
        if (w * (kSegTile / kWaves) + r * kWave + lane < nz) cmax = cc[r] > cmax ? cc[r] : cmax;
      cmax = wave_max(cmax);
      // One address for the whole pass: update it only when it is below
      // this wave's maximum (it settles early, so few waves write it).
      int32_t *mp = reinterpret_cast<int32_t *>(rs.bad) + 1;
      if (lane == 0 && cmax > __hip_atomic_load(mp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(mp, cmax);
    }
#pragma unroll
    for (int r = 0; r < kSegPer; ++r) {
      const int32_t e = w * (kSegTile / kWaves) + r * kWave + lane;
      if (e < nz) {
        col[j0 + e] = cc[r];
        val[j0 + e] = vv[r];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const bool valid = w * (kSegTile / kWaves) + r * kWave + lane < nz;
    rank[r] = wave_digit_rank(slab_of(cc[r], sbits, ns), valid, dbits, wh[w]);
  }
  __syncthreads();
  const int d = tid;   // one slab per thread (ns <= 256 = kThreads)
  uint32_t total = 0;
  if (d < ns) {
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t t = wh[q][d];
      wh[q][d] = total;
      total += t;
    }
  }
  uint32_t all;
  const uint32_t first = block_exscan256(total, s_scan, &all);
  if (d < ns) {
    s_toff[d] = first;
    if constexpr (kScatter) {
      s_goff[d] = ecnt[int64_t(b) * ns + d];
      s_poff[d] = pcnt[int64_t(b) * ns + d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const int32_t e = w * (kSegTile / kWaves) + r * kWave + lane;
    if (e < nz) {
      const uint32_t dg = slab_of(cc[r], sbits, ns);
      const uint32_t slot = s_toff[dg] + wh[w][dg] + rank[r];
      s_col[slot] = cc[r];
      s_end[slot] = rr[r];
      if constexpr (kScatter) s_val[slot] = vv[r];
    }
  }
  __syncthreads();
  // Pair starts: slot k * kThreads + tid, so each wave flags 64 consecutive
  // slots (chunk k * kWaves + w) with one ballot.
  uint64_t bal[kSegPer];
#pragma unroll
  for (int k = 0; k < kSegPer; ++k) {
    const int32_t slot = k * kThreads + tid;
    bool f = false;
    if (slot < nz) {
      const uint32_t dg = slab_of(s_col[slot], sbits, ns);
      const int32_t lr = s_end[slot];
      const bool head = slot == 0 || slab_of(s_col[slot - 1], sbits, ns) != dg;
      f = head || s_end[slot - 1] != lr;
      if (kScatter && head && lr == 0 && ((s_cont[dg >> 5] >> (dg & 31)) & 1u)) f = false;
    }
    bal[k] = __ballot(f);
    if (lane == 0) s_bal[k * kWaves + w] = bal[k];
  }
  __syncthreads();
  if (tid <= kChunks) {
    uint32_t a = 0;
    for (int q = 0; q < tid; ++q) a += uint32_t(__popcll(s_bal[q]));
    s_pre[tid] = a;
  }
  __syncthreads();
  // Pair starts before slot x of the tile.
  auto starts_before = [&](uint32_t x) -> uint32_t {
    const uint32_t q = x / kWave, o = x % kWave;
    return s_pre[q] + (o ? uint32_t(__popcll(s_bal[q] & ((1ull << o) - 1ull))) : 0u);
  };
  if constexpr (!kScatter) {
    bool fb = false, lb = false;
    if (d < ns) {
      const uint32_t a0 = s_toff[d];
      ecnt[int64_t(b) * ns + d] = total;
      pcnt[int64_t(b) * ns + d] = starts_before(a0 + total) - starts_before(a0);
      // Slots of a slab run are in row order: its head holds the smallest
      // local row, its tail the largest.
      fb = total > 0 && s_end[a0] == 0;
      lb = total > 0 && s_end[a0 + total - 1] == na;
    }
    const uint64_t fmb = __ballot(fb), lmb = __ballot(lb);
    if (lane == 0) {
      fmask[int64_t(b) * kMaskWords + 2 * w] = uint32_t(fmb);
      fmask[int64_t(b) * kMaskWords + 2 * w + 1] = uint32_t(fmb >> 32);
      lmask[int64_t(b) * kMaskWords + 2 * w] = uint32_t(lmb);
      lmask[int64_t(b) * kMaskWords + 2 * w + 1] = uint32_t(lmb >> 32);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
      const int32_t slot = k * kThreads + tid;
      if (slot < nz) {
        const int32_t cv = s_col[slot];
        const uint32_t dg = slab_of(cv, sbits, ns);
        const int64_t pos = int64_t(s_goff[dg]) + (slot - int32_t(s_toff[dg]));
        if (kCount && packed) {
          // Packed count form: the column inside its slab (< 2^24) and the count.
          seg_col[pos] = int32_t(uint32_t(cv - int32_t(dg << sbits)) | (uint32_t(s_val[slot]) << 24));
        } else {
          seg_col[pos] = cv;
          seg_val[pos] = s_val[slot];
        }
        if ((bal[k] >> lane) & 1ull) {
          const uint32_t here = s_pre[k * kWaves + w] + uint32_t(__popcll(bal[k] & lanes_below()));
          const uint32_t pid = s_poff[dg] + here - starts_before(s_toff[dg]);
          prp[pid] = int32_t(pos);
          pair_row[pid] = i0 + s_end[slot];
        }
      }
    }
  }
}

// Offsets of a tiles x slabs count matrix stored tile by tile (row b =
// tile b, ns counts): out[b * ns + d] = counts of all slabs d' < d plus
// those of slab d in tiles before b, i.e. an exclusive scan in slab-major
// order, computed with whole rows only.  Tiles are taken kColTiles at a time:
// block sums per slab, a scan of those (slab-major), then each block's
// running prefix.
constexpr int kColTiles = 256;

__global__ __launch_bounds__(kThreads) void k_col_sums(const uint32_t *__restrict__ cnt,
                                                       int32_t ntiles, int32_t ns, int32_t nblk,
                                                       uint32_t *__restrict__ bsum) {
  const int d = threadIdx.x, blk = blockIdx.x;
  if (d >= ns) return;
  const int32_t b0 = blk * kColTiles;
  const int32_t b1 = b0 + kColTiles < ntiles ? b0 + kColTiles : ntiles;
  uint32_t a = 0;
#pragma unroll 8
  for (int32_t b = b0; b < b1; ++b) a += cnt[int64_t(b) * ns + d];
  bsum[int64_t(d) * nblk + blk] = a;
}

__global__ __launch_bounds__(kThreads) void k_col_offsets(const uint32_t *__restrict__ cnt,
                                                          int32_t ntiles, int32_t ns,
                                                          int32_t nblk,
                                                          const uint32_t *__restrict__ boff,
                                                          uint32_t *__restrict__ out) {
  const int d = threadIdx.x, blk = blockIdx.x;
  if (d >= ns) return;
  const int32_t b0 = blk * kColTiles;
  const int32_t b1 = b0 + kColTiles < ntiles ? b0 + kColTiles : ntiles;
  uint32_t run = boff[int64_t(d) * nblk + blk];
  for (int32_t b = b0; b < b1; ++b) {
    const uint32_t v = cnt[int64_t(b) * ns + d];
    out[int64_t(b) * ns + d] = run;
    run += v;
  }
}

// A tile that starts inside a row R continues R's runs from the earlier
// tiles that hold R: their end-of-tile slab masks are OR-ed (walking back
// while the tiles stay inside R), kept where the tile's first row has
// entries too, and stored as the tile's cont mask; each such slab's run is
// taken off the tile's pair count.
__global__ __launch_bounds__(256) void k_seg_cont(const int32_t *__restrict__ rp, int32_t n,
                                                  const int2 *__restrict__ coord, int32_t ntiles,
                                                  int32_t ns, const uint32_t *__restrict__ lmask,
                                                  uint32_t *__restrict__ fmask,
                                                  uint32_t *__restrict__ pcnt) {
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b < ntiles; b += gridDim.x * 256) {
    const int2 c0 = coord[b];
    const int32_t R = c0.x;
    uint32_t m[kMaskWords];
#pragma unroll
    for (int k = 0; k < kMaskWords; ++k) m[k] = 0u;
    if (b > 0 && R < n && rp[R] < c0.y) {
      int32_t q = b - 1;
      for (;;) {
#pragma unroll
        for (int k = 0; k < kMaskWords; ++k) m[k] |= lmask[int64_t(q) * kMaskWords + k];
        if (q > 0 && coord[q].x == R && rp[R] < coord[q].y)
          --q;
        else
          break;
      }
#pragma unroll
      for (int k = 0; k < kMaskWords; ++k) {
        m[k] &= fmask[int64_t(b) * kMaskWords + k];
        uint32_t bits = m[k];
        while (bits) {
          const int d = k * 32 + __builtin_ctz(bits);
          pcnt[int64_t(b) * ns + d] -= 1u;
          bits &= bits - 1u;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaskWords; ++k) fmask[int64_t(b) * kMaskWords + k] = m[k];
  }
}

// Completes pairs that span SpMV workgroups (raw accumulators, no sum).
template <typename V>
__global__ __launch_bounds__(256) void k_fix_raw(typename Form<V>::Part *__restrict__ part,
                                                 int32_t nb, const int2 *__restrict__ coord,
                                                 const uint8_t *__restrict__ closes,
                                                 const int32_t *__restrict__ carry_row,
                                                 const typename Form<V>::Acc *__restrict__ blk_carry,
                                                 const typename Form<V>::Acc *__restrict__ blk_head) {
  using Acc = typename Form<V>::Acc;
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256) {
    if (!closes[b]) continue;
    const int32_t R = coord[b].x;
    int32_t q = b - 1;
    while (q >= 0 && carry_row[q] == R) --q;
    Acc sum{};
    for (int32_t k = q + 1; k < b; ++k) sum = merge(sum, blk_carry[k]);
    part[R] = Form<V>::part(merge(sum, blk_head[b]));
  }
}

// Combine blocks: rows [cstart[b], cstart[b+1]) with cstart[b] the first
// row v whose cost v + rpp[v] (rows plus pairs before it) reaches
// b * kCombItems, so a block never splits a row and holds at most
// kCombItems + kMaxSlabs rows plus pairs, hub rows and empty ones alike.
// cstart[b] = (first row, its first pair rpp[row]).
__global__ __launch_bounds__(256) void k_comb_bounds(const int32_t *__restrict__ rpp, int32_t n,
                                                     int32_t nblk, int2 *__restrict__ cstart) {
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b <= nblk; b += gridDim.x * 256) {
    const int64_t target = int64_t(b) * kCombItems;
    int32_t lo = 0, hi = n;   // first v in [0, n] with v + rpp[v] >= target
    while (lo < hi) {
      const int32_t m = (lo + hi) >> 1;
      if (int64_t(m) + rpp[m] < target)
        lo = m + 1;
      else
        hi = m;
    }
    const int32_t R = b == nblk ? n : lo;
    cstart[b] = make_int2(R, rpp[R]);
  }
}

// First pair of slab d whose row is >= R.  The pairs are stored slab by
// slab and, inside a slab, build tile by tile (poff[t * ns + d] = first
// pair of tile t in slab d), rows ascending.  Row R's first merge item lies
// in build tile t = (R + rp[R]) / kSegTile; pairs of rows >= R start in
// tiles >= t and pairs of earlier rows in tiles <= t, so the answer is
// found by a binary search of tile t's run alone.
__device__ __forceinline__ int64_t slab_bound(const int32_t *__restrict__ pair_row,
                                              const uint32_t *__restrict__ poff,
                                              const int64_t *__restrict__ slab_start,
                                              const int32_t *__restrict__ rp, int32_t n,
                                              int32_t ntiles, int32_t ns, int32_t d, int32_t R) {
  if (R >= n) return slab_start[d + 1];
  const int64_t t = (int64_t(R) + rp[R]) / kSegTile;
  int64_t lo = poff[t * ns + d];
  int64_t hi = t + 1 < ntiles ? int64_t(poff[(t + 1) * ns + d]) : slab_start[d + 1];
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (pair_row[m] < R)
      lo = m + 1;
    else
      hi = m;
  }
  return lo;
}

// lo[b * ns + d] = first pair of slab d whose row is >= the first row of
// block b, b <= nblk: row min(n, b * row_step) for row blocks of a fixed
// height, cstart[b].x for combine blocks (row_step 0; block nblk starts at
// row n).
__global__ __launch_bounds__(256) void k_pair_bounds(const int32_t *__restrict__ pair_row,
                                                     const uint32_t *__restrict__ poff,
                                                     const int64_t *__restrict__ slab_start,
                                                     const int32_t *__restrict__ rp, int32_t n,
                                                     int32_t ntiles, int32_t ns, int32_t nblk,
                                                     int32_t row_step,
                                                     const int2 *__restrict__ cstart,
                                                     int32_t *__restrict__ lo) {
  const int64_t total = (int64_t(nblk) + 1) * ns;
  for (int64_t k = blockIdx.x * int64_t(256) + threadIdx.x; k < total;
       k += int64_t(gridDim.x) * 256) {
    const int32_t b = int32_t(k / ns), d = int32_t(k - int64_t(b) * ns);
    const int64_t R = row_step > 0 ? int64_t(b) * row_step : int64_t(cstart[b].x);
    lo[k] = int32_t(slab_bound(pair_row, poff, slab_start, rp, n, ntiles, ns, d,
                               R < n ? int32_t(R) : n));
  }
}

// Slab d of item i of a block whose slab runs start at s_base[0 .. ns]:
// s_base[d] <= i < s_base[d + 1], searched in [lo, hi).
__device__ __forceinline__ int32_t run_of(const int32_t *s_base, int32_t i, int32_t lo,
                                          int32_t hi) {
  while (hi - lo > 1) {
    const int32_t m = (lo + hi) >> 1;
    if (s_base[m] <= i)
      lo = m;
    else
      hi = m;
  }
  return lo;
}

// Pairs per row, for rows in blocks of kCountRows: the block's pairs in
// slab d are [lo[b][d], lo[b + 1][d]), each adds one to its row's counter
// in LDS (integer adds, so the order does not matter), and the block then
// stores its rows' counts in order (pcount, scanned into rpp afterwards).
constexpr int kCountRows = 4096;
constexpr int kBatch = 8;
__global__ __launch_bounds__(kThreads) void k_pair_count(const int32_t *__restrict__ pair_row,
                                                         const int32_t *__restrict__ lo_tab,
                                                         int32_t ns, int32_t n,
                                                         uint32_t *__restrict__ pcount) {
  __shared__ uint32_t s_cnt[kCountRows];
  __shared__ int32_t s_lo[kMaxSlabs];
  __shared__ int32_t s_base[kMaxSlabs + 1];
  __shared__ uint32_t s_scan[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int32_t R0 = b * kCountRows;
  const int32_t nr = n - R0 < kCountRows ? n - R0 : kCountRows;
  uint32_t cnt = 0;
  if (tid < ns) {
    const int32_t lo = lo_tab[int64_t(b) * ns + tid];
    s_lo[tid] = lo;
    cnt = uint32_t(lo_tab[int64_t(b + 1) * ns + tid] - lo);
  }
  uint32_t all;
  const uint32_t base = block_exscan256(cnt, s_scan, &all);
  if (tid < ns) s_base[tid] = int32_t(base);
  if (tid == 0) s_base[ns] = int32_t(all);
  for (int32_t r = tid; r < kCountRows; r += kThreads) s_cnt[r] = 0u;
  __syncthreads();
  // kBatch items per thread at a time, every read issued before any is
  // used (items past the end read pair 0 and are dropped).
  for (int32_t i0 = 0; i0 < int32_t(all); i0 += kThreads * kBatch) {
    int32_t rr[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int32_t i = i0 + k * kThreads + tid;
      const int32_t d = run_of(s_base, i < int32_t(all) ? i : 0, 0, ns);
      rr[k] = pair_row[i < int32_t(all) ? s_lo[d] + (i - s_base[d]) : 0];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int32_t i = i0 + k * kThreads + tid;
      const int32_t r = rr[k] - R0;
      if (i < int32_t(all) && r >= 0 && r < nr) atomicAdd(&s_cnt[r], 1u);
    }
  }
  __syncthreads();
  for (int32_t r = tid; r < nr; r += kThreads) pcount[R0 + r] = s_cnt[r];
}

// Row-major order of the pairs (pidx) for the combine: each row's pairs,
// in slab order, at rpp[row] ...  One workgroup per combine block (rows
// [R0, R1), at most kCap rows plus pairs); its pairs in slab d are
// [lo[b][d], lo[b + 1][d]) (rows ascending, each row at most once), taken
// 32 slabs at a time.  Every pair sets its slab's bit in its row's word;
// then its rank inside the row is the row's pairs in earlier windows plus
// the set bits below its own.  OR commutes, so the result does not depend
// on the order of the updates.  bad is set (and nothing stored) if a
// block's runs do not add up to its pair count.
__global__ __launch_bounds__(kThreads) void k_pair_index(
    const int32_t *__restrict__ pair_row, const int32_t *__restrict__ lo_tab, int32_t ns,
    const int2 *__restrict__ cstart, const int32_t *__restrict__ rpp, int32_t *__restrict__ pidx,
    uint32_t *__restrict__ bad) {
  constexpr int kCap = kCombItems + kMaxSlabs;
  __shared__ uint32_t s_bits[kCap];
  __shared__ uint16_t s_cum[kCap], s_off[kCap], s_row[kCap];
  __shared__ int32_t s_lo[kMaxSlabs];
  __shared__ int32_t s_base[kMaxSlabs + 1];
  __shared__ uint32_t s_scan[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int2 c0 = cstart[b], c1 = cstart[b + 1];
  const int32_t R0 = c0.x, nr = c1.x - c0.x, j0 = c0.y, np = c1.y - c0.y;
  uint32_t cnt = 0;
  if (tid < ns) {
    const int32_t lo = lo_tab[int64_t(b) * ns + tid];
    s_lo[tid] = lo;
    cnt = uint32_t(lo_tab[int64_t(b + 1) * ns + tid] - lo);
  }
  uint32_t all;
  const uint32_t base = block_exscan256(cnt, s_scan, &all);
  if (tid < ns) s_base[tid] = int32_t(base);
  if (tid == 0) s_base[ns] = int32_t(all);
  if (all != uint32_t(np) || nr + np > kCap) {
    if (tid == 0) atomicOr(bad, 1u);
    return;   // uniform: every thread sees the same all, np and nr
  }
  for (int32_t r = tid; r < nr; r += kThreads) {
    s_bits[r] = 0u;
    s_cum[r] = 0;
    s_off[r] = uint16_t(rpp[R0 + r] - j0);
  }
  __syncthreads();
  for (int32_t w0 = 0; w0 < ns; w0 += 32) {
    const int32_t w1 = w0 + 32 < ns ? w0 + 32 : ns;
    const int32_t i0 = s_base[w0], i1 = s_base[w1];
    if (i0 == i1) continue;   // uniform
    for (int32_t i = i0 + tid; i < i1; i += kThreads) {
      const int32_t d = run_of(s_base, i, w0, w1);
      const int32_t r = pair_row[s_lo[d] + (i - s_base[d])] - R0;
      const bool ok = r >= 0 && r < nr;
      if (ok) atomicOr(&s_bits[r], 1u << (d - w0));
      else atomicOr(bad, 1u);
      s_row[i] = uint16_t(ok ? r : 0xFFFF);
    }
    __syncthreads();
    for (int32_t i = i0 + tid; i < i1; i += kThreads) {
      const int32_t r = s_row[i];
      if (r == 0xFFFF) continue;
      const int32_t d = run_of(s_base, i, w0, w1);
      const uint32_t bit = 1u << (d - w0);
      const int32_t dst = int32_t(s_off[r]) + s_cum[r] + __popc(s_bits[r] & (bit - 1u));
      if (dst < np)
        pidx[j0 + dst] = s_lo[d] + (i - s_base[d]);
      else
        atomicOr(bad, 1u);
    }
    __syncthreads();
    for (int32_t r = tid; r < nr; r += kThreads) {
      s_cum[r] = uint16_t(s_cum[r] + __popc(s_bits[r]));
      s_bits[r] = 0u;
    }
    __syncthreads();
  }
}

// y[v] = c * (partials of row v, slab by slab) + t.  The block's row
// offsets and pairs, row-major (part[pidx[rpp[v] ..]], each row's in slab
// order), are gathered into LDS with every load in flight, then one thread
// per row adds its run.  Each workgroup stores its part of sum(y) in
// blk_ysum; k_sum_blocks adds them (tens of thousands of workgroups would
// queue on a shared arrival counter).
//
// With wdiv (degree-scaled form, every iteration but the last) the block
// stores y[v] / wdiv[v], the vector the next iteration gathers, instead of
// y[v], and nothing where wdiv[v] <= 0 (such a column holds no entries, its
// value is never gathered); sum(y) is formed from y either way.
// With perm (the last iteration of a relabelled run) y[v] goes to
// y[perm[v]]: the result in the caller's labels, with no pass of its own.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_seg_combine(
    const typename Form<V>::Part *__restrict__ part, const int32_t *__restrict__ rpp,
    const int32_t *__restrict__ pidx, const int2 *__restrict__ cstart, double c,
    const double *__restrict__ tele_in, V *__restrict__ y, double *__restrict__ blk_ysum,
    const int32_t *__restrict__ wdiv, const int32_t *__restrict__ perm) {
  using Acc = typename Form<V>::Acc;
  using Part = typename Form<V>::Part;
  constexpr int kCap = kCombItems + kMaxSlabs;
  constexpr int kPer = kCap / kThreads;
  __shared__ Part s_part[kCap];
  __shared__ uint16_t s_off[kCap + 1];   // rpp[R0 + i] - rpp[R0]
  __shared__ double sh[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int2 c0 = cstart[b], c1 = cstart[b + 1];
  const int32_t R0 = c0.x, nr = c1.x - c0.x, j0 = c0.y, np = c1.y - c0.y;
  {
    int32_t pi[kPer], ro[kPer + 1];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t q = k * kThreads + tid;
      // Indices clamped into range, so every load is issued unconditionally
      // (a load under a per-lane condition is waited for before the next).
      pi[k] = pidx[np > 0 ? j0 + (q < np ? q : np - 1) : 0];
      ro[k] = rpp[R0 + (q <= nr ? q : nr)];
    }
    {
      const int32_t q = kPer * kThreads + tid;
      ro[kPer] = rpp[R0 + (q <= nr ? q : nr)];
    }
#pragma unroll
    for (int k = 0; k <= kPer; ++k) {
      const int32_t q = k * kThreads + tid;
      if (q <= nr) s_off[q] = uint16_t(ro[k] - j0);
    }
    Part pa[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) pa[k] = part[pi[k]];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t q = k * kThreads + tid;
      if (q < np) s_part[q] = pa[k];
    }
  }
  __syncthreads();
  const double tk = *tele_in;
  double ysum = 0.0;
  for (int32_t i = tid; i < nr; i += kThreads) {
    const int32_t e = s_off[i + 1];
    Acc acc{};
    for (int32_t j = s_off[i]; j < e; ++j) acc = merge(acc, Form<V>::acc(s_part[j]));
    const V yv = Form<V>::finish(acc, c, tk);
    if (wdiv) {
      const int32_t d = wdiv[R0 + i];
      if (d > 0) y[R0 + i] = V(double(yv) / double(d));
    } else if (perm) {
      y[perm[R0 + i]] = yv;
    } else {
      y[R0 + i] = yv;
    }
    ysum += double(yv);
  }
  const double tot = block_sum256(ysum, sh);
  if (tid == 0) blk_ysum[b] = tot;
}

// sum(y) = the nblk workgroup partials added in a fixed order by one
// workgroup of 1024 threads, plus niso rows without entries left out of
// the combine (each y = the teleport term tele_in, rounded to FP32 when
// f32); stores it and the next teleport scalar.  Each thread keeps 8
// running sums over interleaved partials (8 reads in flight), added in a
// fixed order at the end.
__global__ __launch_bounds__(1024) void k_sum_blocks(const double *__restrict__ blk_ysum,
                                                     int32_t nblk, int64_t niso,
                                                     const double *__restrict__ tele_in,
                                                     int32_t f32, double w, double *sum_out,
                                                     double *tele_out) {
  __shared__ double sh[1024 / kWave];
  double acc[8] = {};
  for (int k0 = 0; k0 < nblk; k0 += 8 * 1024) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + i * 1024 + int(threadIdx.x);
      const double v = blk_ysum[k < nblk ? k : 0];   // unconditional read (nblk >= 1)
      acc[i] += k < nblk ? v : 0.0;
    }
  }
  double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  a = wave_sum(a);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < 1024 / kWave; ++q) s += sh[q];
    if (niso > 0) {
      const double t = *tele_in;
      s += double(niso) * (f32 ? double(float(t)) : t);
    }
    if (sum_out) *sum_out = s;
    *tele_out = w * s;
  }
}

// The last iteration's rows [p0, n) in the new order, which hold no entries:
// y = the teleport term, stored at dst[order[p]] (the caller's labels).
template <typename V>
__global__ __launch_bounds__(256) void k_iso_out(const int32_t *__restrict__ order, int32_t p0,
                                                 int32_t n, const double *__restrict__ tele_in,
                                                 V *__restrict__ dst) {
  const V t = V(*tele_in);
  for (int32_t p = p0 + blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256)
    dst[order[p]] = t;
}

// ------------------------------------------------ run to a convergence test
// Sec. IV.D notes that applications iterate until the normed sum of the
// differences between iterations is small; Sec. IV.C-D and V name the
// adjustments for dangling vertices (rows of A without entries).  An
// iteration's launches give y = c * x A + t and S_y = sum(y) (fixed order).
// One pass over x and y then finishes the step:
//   mode SELF adds c * x_j to y_j for every dangling j (the entry A(j,j) = 1
//   of an empty row), so the new sum is S_y + c * D_x, D_x the mass of x on
//   dangling vertices (from the previous pass);
//   block sums of |y_j / S_y - x_j / S_x| (as products with the sums'
//   reciprocals) and of y over dangling vertices.
// A one-workgroup finish adds them in a fixed order: delta (infinite unless
// both sums are positive), the stop flag delta <= tol, sum(r) of the new
// iterate, and the next teleport (1-c)/N * S_y, plus c/N * D_y in mode
// UNIFORM (a dangling vertex's damped mass spread evenly).  r_0's S and D
// come from a pass of their own.
enum : int32_t { kDangNone = 0, kDangUniform = 1, kDangSelf = 2 };
constexpr int kConvBlocks = 8192;

struct ConvState {
  double sx, sy, dx, delta, stop;
};

__global__ __launch_bounds__(256) void k_dflag(const int32_t *__restrict__ d_out,
                                               const int32_t *__restrict__ order, int32_t n,
                                               uint8_t *__restrict__ dflag) {
  for (int32_t p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256)
    dflag[p] = d_out[order ? order[p] : p] == 0 ? 1 : 0;
}

// sum(r_0) and its mass on dangling vertices (dflag may be null).
template <typename V>
__global__ __launch_bounds__(kThreads) void k_conv_init(const V *__restrict__ x, int64_t n,
                                                        const uint8_t *__restrict__ dflag,
                                                        double *__restrict__ part) {
  __shared__ double sh[4];
  double a = 0.0, d = 0.0;
  for (int64_t j = blockIdx.x * int64_t(kThreads) + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * kThreads) {
    const double v = double(x[j]);
    a += v;
    if (dflag && dflag[j]) d += v;
  }
  const double ba = block_sum256(a, sh);
  const double bd = block_sum256(d, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ba;
    part[kConvBlocks + blockIdx.x] = bd;
  }
}

template <typename V>
__global__ __launch_bounds__(kThreads) void k_conv_step(const V *__restrict__ x, V *__restrict__ y,
                                                        int64_t n, const uint8_t *__restrict__ dflag,
                                                        double self_c, const ConvState *__restrict__ st,
                                                        double *__restrict__ part) {
  __shared__ double sh[4];
  const double sx = st->sx, sy = st->sy + self_c * st->dx;
  const bool ok = sx > 0.0 && sy > 0.0;
  const double ix = ok ? 1.0 / sx : 0.0, iy = ok ? 1.0 / sy : 0.0;
  double a = 0.0, d = 0.0;
  for (int64_t j = blockIdx.x * int64_t(kThreads) + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * kThreads) {
    double v = double(y[j]);
    const bool dang = dflag && dflag[j];
    if (dang && self_c != 0.0) {
      const V nv = V(v + self_c * double(x[j]));
      y[j] = nv;
      v = double(nv);
    }
    if (ok) a += fabs(v * iy - double(x[j]) * ix);
    if (dang) d += v;
  }
  const double ba = block_sum256(a, sh);
  const double bd = block_sum256(d, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ba;
    part[kConvBlocks + blockIdx.x] = bd;
  }
}

// first: the pass was k_conv_init over r_0 (part = sums, not differences).
__global__ __launch_bounds__(kThreads) void k_conv_fin(const double *__restrict__ part,
                                                       int32_t nblk, double w, double cn,
                                                       int32_t uniform, double self_c, double tol,
                                                       int32_t first, ConvState *st,
                                                       double *tele_out, double *sum_out,
                                                       double *delta_out) {
  __shared__ double sh[4];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kThreads) {
    a += part[k];
    b += part[kConvBlocks + k];
  }
  const double sa = block_sum256(a, sh);
  const double dn = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    double s;
    if (first) {
      s = sa;
    } else {
      s = st->sy + self_c * st->dx;
      const double delta = (st->sx > 0.0 && s > 0.0) ? sa : INFINITY;
      st->delta = delta;
      st->stop = delta <= tol ? 1.0 : 0.0;
      if (delta_out) *delta_out = delta;
    }
    st->sx = s;
    st->dx = dn;
    *tele_out = uniform ? w * s + cn * dn : w * s;
    if (sum_out) *sum_out = s;
  }
}

// Optional event pairs around each SpMV launch (benchmark instrumentation).
struct Timing {
  bool on = false;
  int used = 0;
  std::vector<hipEvent_t> start, stop;
};
Timing g_timing;
constexpr int kMaxTimed = 256;

pp_status timed_begin(hipStream_t s) {
  if (!g_timing.on || g_timing.used >= kMaxTimed) return PP_OK;
  PP_HIP(hipEventRecord(g_timing.start[g_timing.used], s));
  return PP_OK;
}
pp_status timed_end(hipStream_t s) {
  if (!g_timing.on || g_timing.used >= kMaxTimed) return PP_OK;
  PP_HIP(hipEventRecord(g_timing.stop[g_timing.used], s));
  ++g_timing.used;
  return PP_OK;
}

template <typename V>
struct Layout {
  V *y;
  int2 *coord;
  uint8_t *closes;
  int32_t *carry_row;
  typename Form<V>::Acc *blk_carry, *blk_head;
  double *blk_ysum, *part, *tele;
  uint32_t *counter;
  unsigned long long *ksum;
  // vertex relabelling
  uint64_t *keys_in;
  uint32_t *bucket_off;
  int32_t *order, *wnew, *rp2, *col2;
  int2 *lab;
  uint64_t *hot;
  uint32_t *bad, *npos;
  V *val2, *x2;
  int64_t *total;
  // column segmenting
  int32_t *seg_col, *prp, *pair_row, *rpp, *pidx;
  int2 *cstart, *seg_coord;
  int64_t *info;
  int32_t *seg_es;   // slab starts in the segmented entries
  int2 *tile_slab;   // SpMV workgroups' first slab and the next slab's start
  V *seg_val;
  typename Form<V>::Part *seg_part;
  // run to a convergence test
  uint8_t *dflag;
  double *conv_part;
  ConvState *conv;
  uint32_t *seg_cnt, *seg_pcnt, *seg_bsum, *seg_fmask, *seg_lmask, *seg_scan;
};

// One layout function serves both measuring (ws == nullptr) and carving.
template <typename V>
Layout<V> carve(void *ws, int64_t n, int64_t nnz_cap, int32_t nrhs, size_t *bytes = nullptr) {
  using Acc = typename Form<V>::Acc;
  Carve c(ws);
  Layout<V> L{};
  // SpMV tiles: over (rows, entries), or over (pairs, entries) when the
  // columns are segmented (at most one pair per entry).
  const int64_t rows_cap = n > nnz_cap ? n : nnz_cap;
  const int64_t nb = (rows_cap + nnz_cap + kItemsMin - 1) / kItemsMin + 1;
  const int64_t G = (nb + kFinishPer - 1) / kFinishPer + 1;
  const int64_t G0 = (n + kSumChunk - 1) / kSumChunk + 1;
  L.ksum = c.take<unsigned long long>(64);
  L.counter = c.take<uint32_t>(4);
  L.tele = c.take<double>(2 * 64);
  L.total = c.take<int64_t>(1);
  L.y = c.take<V>(size_t(n) * nrhs);
  L.coord = c.take<int2>(size_t(nb + 1));
  L.closes = c.take<uint8_t>(size_t(nb));
  L.carry_row = c.take<int32_t>(size_t(nb));
  L.blk_carry = c.take<Acc>(size_t(nb) * nrhs);
  L.blk_head = c.take<Acc>(size_t(nb) * nrhs);
  L.blk_ysum = c.take<double>(size_t(nb) * nrhs);
  L.part = c.take<double>(size_t(G > G0 ? G : G0) * nrhs);
  L.keys_in = c.take<uint64_t>(size_t(n));
  L.bucket_off = c.take<uint32_t>(size_t(kBuckets) * size_t((n + kRelTile - 1) / kRelTile));
  L.order = c.take<int32_t>(size_t(n));
  L.lab = c.take<int2>(size_t(n));
  L.wnew = c.take<int32_t>(size_t(n));
  L.hot = c.take<uint64_t>(size_t(2) << hot_log2(n));
  L.bad = c.take<uint32_t>(2);
  L.npos = c.take<uint32_t>(2);
  L.rp2 = c.take<int32_t>(size_t(n + 1));
  {
    // One region for the relabelled entries; when the columns are
    // segmented it is free after the build and holds the pairs' row-major
    // index (and, during the build, the second buffer of a sort of pairs).
    const size_t z = size_t(nnz_cap > 0 ? nnz_cap : 1);
    const size_t colb = (z * 4 + 255) / 256 * 256;
    uint8_t *rl = c.take<uint8_t>(colb + z * sizeof(V));
    L.col2 = reinterpret_cast<int32_t *>(rl);
    L.val2 = rl ? reinterpret_cast<V *>(rl + colb) : nullptr;
  }
  L.x2 = c.take<V>(size_t(n) * nrhs);
  if (nrhs == 1) {
    L.dflag = c.take<uint8_t>(size_t(n));
    L.conv_part = c.take<double>(2 * kConvBlocks);
    L.conv = c.take<ConvState>(1);
  }
  if (nrhs == 1) {
    const int64_t z = nnz_cap > 0 ? nnz_cap : 1;
    const int64_t ntiles = (n + nnz_cap + kSegTile - 1) / kSegTile + 1;
    L.seg_col = c.take<int32_t>(size_t(z));
    L.seg_val = c.take<V>(size_t(z));
    L.prp = c.take<int32_t>(size_t(z + 1));
    L.pair_row = c.take<int32_t>(size_t(z));
    // One partial per pair (at most one pair per entry), written by the
    // iterations.
    L.seg_part = c.take<typename Form<V>::Part>(size_t(z));
    const int64_t cnt_n = kMaxSlabs * ntiles;
    L.seg_cnt = c.take<uint32_t>(size_t(cnt_n));
    L.seg_pcnt = c.take<uint32_t>(size_t(kMaxSlabs * ntiles));
    L.seg_bsum = c.take<uint32_t>(size_t(kMaxSlabs) * size_t((ntiles + kColTiles - 1) / kColTiles + 1));
    L.seg_fmask = c.take<uint32_t>(size_t(kMaskWords * ntiles));
    L.seg_lmask = c.take<uint32_t>(size_t(kMaskWords * ntiles));
    L.seg_coord = c.take<int2>(size_t(ntiles + 1));
    int64_t scan_n = z + 1 > cnt_n ? z + 1 : cnt_n;
    if (n + 1 > scan_n) scan_n = n + 1;
    L.seg_scan = c.take<uint32_t>(size_t(scan_ws_elems(scan_n)));
    L.rpp = c.take<int32_t>(size_t(n + 1));
    L.info = c.take<int64_t>(4 + kMaxSlabs);
    L.seg_es = c.take<int32_t>(kMaxSlabs + 2);
    L.tile_slab = c.take<int2>(size_t(nb + 1));
    L.cstart = c.take<int2>(size_t((n + z + kCombItems - 1) / kCombItems + 2));
    L.pidx = L.col2;
  }
  if (bytes) *bytes = c.bytes();
  return L;
}

template <typename V>
size_t ws_bytes_t(int64_t n, int64_t nnz_cap, int32_t nrhs) {
  size_t b = 0;
  carve<V>(nullptr, n, nnz_cap, nrhs, &b);
  return b;
}

template <typename V, int G>
void launch_spmm_g(int32_t nb, hipStream_t s, const int32_t *rp, const int32_t *col, const V *val,
                   const V *x, V *y, int32_t n, int32_t k, const int2 *coord, double c,
                   const double *tele, double *blk_ysum, typename Form<V>::Acc *blk_carry,
                   typename Form<V>::Acc *blk_head) {
  hipLaunchKernelGGL((k_spmm<V, G>), dim3(nb), dim3(kThreads), 0, s, rp, col, val, x, y, n, k,
                     coord, c, tele, blk_ysum, blk_carry, blk_head);
}

template <typename V>
void launch_spmm(int G, int32_t nb, hipStream_t s, const int32_t *rp, const int32_t *col,
                 const V *val, const V *x, V *y, int32_t n, int32_t k, const int2 *coord, double c,
                 const double *tele, double *blk_ysum, typename Form<V>::Acc *blk_carry,
                 typename Form<V>::Acc *blk_head) {
  switch (G) {
    case 2: launch_spmm_g<V, 2>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
    case 4: launch_spmm_g<V, 4>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
    case 8: launch_spmm_g<V, 8>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
    case 16: launch_spmm_g<V, 16>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
    case 32: launch_spmm_g<V, 32>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
    default: launch_spmm_g<V, 64>(nb, s, rp, col, val, x, y, n, k, coord, c, tele, blk_ysum, blk_carry, blk_head); break;
  }
}

template <typename V, bool kRaw, typename E = V>
void launch_spmv(int ipt, int32_t nb, hipStream_t s, const int32_t *rp, const int32_t *col,
                 const E *val, const V *x, V *y, int32_t n, const int2 *coord, double c,
                 const double *tele, double *blk_ysum, typename Form<V>::Acc *blk_carry,
                 typename Form<V>::Acc *blk_head, typename Form<V>::Part *part,
                 SlabMap sm = SlabMap{}) {
  if (ipt == 4)
    hipLaunchKernelGGL((k_spmv<V, 4, kRaw, E>), dim3(nb), dim3(kThreads), 0, s, rp, col, val, x,
                       y, n, coord, c, tele, blk_ysum, blk_carry, blk_head, part, sm);
  else if (ipt == 16)
    hipLaunchKernelGGL((k_spmv<V, 16, kRaw, E>), dim3(nb), dim3(kThreads), 0, s, rp, col, val, x,
                       y, n, coord, c, tele, blk_ysum, blk_carry, blk_head, part, sm);
  else
    hipLaunchKernelGGL((k_spmv<V, 8, kRaw, E>), dim3(nb), dim3(kThreads), 0, s, rp, col, val, x,
                       y, n, coord, c, tele, blk_ysum, blk_carry, blk_head, part, sm);
}

// Per SpMV workgroup b: the slab of its first entry and the next slab's
// first entry (es holds the slab starts, es[ns] = nnz).
__global__ __launch_bounds__(256) void k_tile_slab(const int2 *__restrict__ coord, int32_t nb,
                                                   const int32_t *__restrict__ es, int32_t ns,
                                                   int2 *__restrict__ ts) {
  for (int32_t b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256) {
    const int32_t j = coord[b].y;
    int32_t lo = 0, hi = ns - 1;   // last d with es[d] <= j
    while (lo < hi) {
      const int32_t m = (lo + hi + 1) >> 1;
      if (es[m] <= j)
        lo = m;
      else
        hi = m - 1;
    }
    ts[b] = make_int2(lo, es[lo + 1]);
  }
}

// es[d] = first segmented entry of slab d (tile 0's offset), es[ns] = nnz.
__global__ void k_slab_starts(const uint32_t *__restrict__ eoff, int32_t ns, int64_t nnz,
                              int32_t *__restrict__ es) {
  for (int d = threadIdx.x; d <= ns; d += blockDim.x) es[d] = d < ns ? int32_t(eoff[d]) : int32_t(nnz);
}

// info[0] = P, info[1 + d] = first pair of slab d (d <= ns; slab ns = the
// end, P); prp[P] = nnz.  poff holds the per-(tile, slab) offsets, so its
// entry for (tile 0, slab d) is the start of slab d.
__global__ void k_seg_info(const uint32_t *__restrict__ poff, int32_t ns, int64_t nnz,
                           const int64_t *__restrict__ total, int32_t *__restrict__ prp,
                           int64_t *__restrict__ info) {
  const int64_t P = *total;
  for (int d = threadIdx.x; d <= ns; d += blockDim.x) info[1 + d] = d < ns ? int64_t(poff[d]) : P;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    info[0] = P;
    if (P >= 0 && P <= nnz) prp[P] = int32_t(nnz);
  }
}

// What build_segments produced.  P == 0: segmenting does not apply.
struct SegInfo {
  int32_t sbits = 0, ns = 0;
  int64_t P = 0;
  bool relabelled = false;   // the count pass wrote the relabelled entries
  bool scaled = false;       // ... as counts (degree-scaled form), stored so by the scatter
  bool packed = false;       // ... packed with their column inside the slab (seg_col only)
  int32_t nlive = 0;         // the combine covers rows [0, nlive)
  int32_t ncomb = 0;         // combine blocks
};

// In-place slab-major offsets of a tile-by-tile count matrix (k_col_sums,
// a scan of the block sums, k_col_offsets); *total gets the sum when given.
pp_status col_offsets(uint32_t *cnt, int32_t ntiles, int32_t ns, uint32_t *bsum, uint32_t *scan_ws,
                      int64_t *total, hipStream_t s) {
  const int32_t nblk = (ntiles + kColTiles - 1) / kColTiles;
  hipLaunchKernelGGL(k_col_sums, dim3(nblk), dim3(kThreads), 0, s, cnt, ntiles, ns, nblk, bsum);
  PP_LAUNCHED("k_col_sums");
  pp_status st = exscan_u32(bsum, bsum, int64_t(ns) * nblk, scan_ws, total, s);
  if (st != PP_OK) return st;
  hipLaunchKernelGGL(k_col_offsets, dim3(nblk), dim3(kThreads), 0, s, cnt, ntiles, ns, nblk, bsum,
                     cnt);
  PP_LAUNCHED("k_col_offsets");
  return PP_OK;
}

// Segmented layout of the matrix (rp, col, val): see the kernels above.
// The slabs cover columns [0, ncols) (columns beyond fall into the last
// slab).  Rows [nlive, n) must have no entries: in the count form the
// combine leaves them out (out->nlive; otherwise it covers all n).  With rl the matrix is the relabelled one, whose entries (col, val) the
// count pass writes from rl's source matrix (out->relabelled tells whether
// it ran).  With scaled (and rl) the count pass first tries the
// degree-scaled form, writing the entries' counts (as bytes, into val's
// space) instead of their values; if any entry is not count / weight it
// runs again storing values.  The host reads that verdict (one stream
// synchronisation) and the scatter pass stores whichever form was written
// (out->scaled).  Segmenting does not apply with fewer than two slabs or
// when pairs + entries reach 2^31; if the count form was written then, the
// relabelled entries are left to k_relabel_copy (out->relabelled false).
// Reads the pair counts back to the host, so it synchronizes the stream
// once more.
template <typename V>
pp_status build_segments(const Layout<V> &L, const int32_t *rp, int32_t *col, V *val, int64_t n,
                         int64_t ncols, int64_t nlive, int64_t nnz, int slab_log2,
                         const RelabelSrc *rl, bool scaled, SegInfo *out, hipStream_t s) {
  *out = SegInfo{};
  int sbits = slab_log2;
  if (ncols < 1) ncols = 1;
  while (((ncols - 1) >> sbits) + 1 > kMaxSlabs) ++sbits;
  const int32_t ns = int32_t(((ncols - 1) >> sbits) + 1);
  if (ns < 2 || nnz <= 0) return PP_OK;
  const int32_t dbits = 32 - __builtin_clz(uint32_t(ns - 1));
  const int32_t n32 = int32_t(n);
  const int32_t ntiles = int32_t((n + nnz + kSegTile - 1) / kSegTile);
  uint8_t *cnt = reinterpret_cast<uint8_t *>(val);
  hipLaunchKernelGGL(k_partition, dim3(grid_for(int64_t(ntiles) + 1, 256, 4096)), dim3(256), 0, s,
                     rp, n32, int32_t(nnz), ntiles, kSegTile, L.seg_coord);
  bool counts = false;
  int32_t maxcol = 0;
  if (rl && scaled) {
    pp_status st = fill_i32(reinterpret_cast<int32_t *>(rl->bad), 2, 0, s);
    if (st != PP_OK) return st;
    hipLaunchKernelGGL((k_seg_tile<V, uint8_t, false, true>), dim3(ntiles), dim3(kThreads), 0, s,
                       rp, col, cnt, n32, *rl, L.seg_coord, sbits, ns, dbits, ntiles, L.seg_cnt,
                       L.seg_pcnt, L.seg_fmask, L.seg_lmask, nullptr, nullptr, nullptr, nullptr, 0);
    PP_LAUNCHED("k_seg_tile (count, scaled)");
    uint32_t flags[2] = {1u, 0u};
    PP_HIP(hipMemcpyAsync(flags, rl->bad, sizeof(flags), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    counts = flags[0] == 0;
    maxcol = int32_t(flags[1]);
  }
  if (rl && !counts) {
    hipLaunchKernelGGL((k_seg_tile<V, V, false, true>), dim3(ntiles), dim3(kThreads), 0, s, rp,
                       col, val, n32, *rl, L.seg_coord, sbits, ns, dbits, ntiles, L.seg_cnt,
                       L.seg_pcnt, L.seg_fmask, L.seg_lmask, nullptr, nullptr, nullptr, nullptr, 0);
  } else if (!rl) {
    hipLaunchKernelGGL((k_seg_tile<V, V, false, false>), dim3(ntiles), dim3(kThreads), 0, s, rp,
                       col, val, n32, RelabelSrc{}, L.seg_coord, sbits, ns, dbits, ntiles,
                       L.seg_cnt, L.seg_pcnt, L.seg_fmask, L.seg_lmask, nullptr, nullptr, nullptr,
                       nullptr, 0);
  }
  out->relabelled = rl != nullptr;
  hipLaunchKernelGGL(k_seg_cont, dim3(grid_for(ntiles, 256, 4096)), dim3(256), 0, s, rp, n32,
                     L.seg_coord, ntiles, ns, L.seg_lmask, L.seg_fmask, L.seg_pcnt);
  PP_LAUNCHED("k_seg_tile (count)/k_seg_cont");
  pp_status st = col_offsets(L.seg_cnt, ntiles, ns, L.seg_bsum, L.seg_scan, nullptr, s);
  if (st != PP_OK) return st;
  st = col_offsets(L.seg_pcnt, ntiles, ns, L.seg_bsum, L.seg_scan, L.total, s);
  if (st != PP_OK) return st;
  // Slab starts in the segmented entries (tile 0's offsets), for the raw
  // SpMV of the packed count form.
  hipLaunchKernelGGL(k_slab_starts, dim3(1), dim3(256), 0, s, L.seg_cnt, ns, nnz, L.seg_es);
  // Counts are packed with their column inside the slab when every such
  // column fits 24 bits (the last slab takes all columns beyond it).
  const int32_t packed =
      counts && sbits <= 24 && int64_t(maxcol) - (int64_t(ns - 1) << sbits) < (int64_t(1) << 24);
  if (counts)
    hipLaunchKernelGGL((k_seg_tile<V, uint8_t, true, false>), dim3(ntiles), dim3(kThreads), 0, s,
                       rp, col, cnt, n32, RelabelSrc{}, L.seg_coord, sbits, ns, dbits, ntiles,
                       L.seg_cnt, L.seg_pcnt, L.seg_fmask, nullptr, L.seg_col,
                       reinterpret_cast<uint8_t *>(L.seg_val), L.prp, L.pair_row, packed);
  else
    hipLaunchKernelGGL((k_seg_tile<V, V, true, false>), dim3(ntiles), dim3(kThreads), 0, s, rp,
                       col, val, n32, RelabelSrc{}, L.seg_coord, sbits, ns, dbits, ntiles,
                       L.seg_cnt, L.seg_pcnt, L.seg_fmask, nullptr, L.seg_col, L.seg_val, L.prp,
                       L.pair_row, 0);
  hipLaunchKernelGGL(k_seg_info, dim3(1), dim3(256), 0, s, L.seg_pcnt, ns, nnz, L.total, L.prp,
                     L.info);
  PP_LAUNCHED("k_seg_tile (scatter)/k_seg_info");
  int64_t info[2 + kMaxSlabs] = {};
  PP_HIP(hipMemcpyAsync(info, L.info, sizeof(int64_t) * size_t(2 + ns), hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  const int64_t P = info[0];
  if (P <= 0 || P > nnz || P + nnz > int64_t(INT32_MAX)) {
    if (counts) out->relabelled = false;   // the one-pass path needs values
    return PP_OK;
  }
  SegInfo si;
  si.relabelled = out->relabelled;
  si.scaled = counts;
  si.packed = packed != 0;
  si.sbits = sbits;
  si.ns = ns;
  si.P = P;
  // In the count form rows [nlive, n) hold no entries and their gathered
  // values are never read (weight <= 0): the combine leaves them out.
  const int32_t nrow = counts ? int32_t(nlive) : n32;
  si.nlive = nrow;

  // Row-major index of the pairs for the combine: per-row pair counts,
  // their scan (rpp), the combine blocks, then one workgroup per block
  // places the block's pairs (k_pair_index).  The bounds tables take the
  // entry offsets' buffer, dead after the scatter pass (kMaxSlabs * ntiles
  // entries, more than (blocks + 1) * ns for either kind of block).
  int32_t *lo_tab = reinterpret_cast<int32_t *>(L.seg_cnt);
  const int32_t ncnt = int32_t((n + kCountRows - 1) / kCountRows);
  if ((st = fill_i32(L.rpp + n, 1, 0, s)) != PP_OK) return st;   // the scan's last element
  hipLaunchKernelGGL(k_pair_bounds, dim3(grid_for((int64_t(ncnt) + 1) * ns, 256, 16384)),
                     dim3(256), 0, s, L.pair_row, L.seg_pcnt, L.info + 1, rp, n32, ntiles, ns,
                     ncnt, kCountRows, nullptr, lo_tab);
  hipLaunchKernelGGL(k_pair_count, dim3(ncnt), dim3(kThreads), 0, s, L.pair_row, lo_tab, ns, n32,
                     reinterpret_cast<uint32_t *>(L.rpp));
  PP_LAUNCHED("k_pair_bounds/k_pair_count");
  st = exscan_u32(reinterpret_cast<uint32_t *>(L.rpp), reinterpret_cast<uint32_t *>(L.rpp), n + 1,
                  L.seg_scan, nullptr, s);
  if (st != PP_OK) return st;
  const int32_t ncomb = int32_t((nrow + P + kCombItems - 1) / kCombItems);
  si.ncomb = ncomb;
  hipLaunchKernelGGL(k_comb_bounds, dim3(grid_for(int64_t(ncomb) + 1, 256, 4096)), dim3(256), 0, s,
                     L.rpp, nrow, ncomb, L.cstart);
  if ((st = fill_i32(reinterpret_cast<int32_t *>(L.bad), 1, 0, s)) != PP_OK) return st;
  hipLaunchKernelGGL(k_pair_bounds, dim3(grid_for((int64_t(ncomb) + 1) * ns, 256, 16384)),
                     dim3(256), 0, s, L.pair_row, L.seg_pcnt, L.info + 1, rp, n32, ntiles, ns,
                     ncomb, 0, L.cstart, lo_tab);
  hipLaunchKernelGGL(k_pair_index, dim3(ncomb), dim3(kThreads), 0, s, L.pair_row, lo_tab, ns,
                     L.cstart, L.rpp, L.pidx, L.bad);
  PP_LAUNCHED("k_comb_bounds/k_pair_bounds/k_pair_index");
  uint32_t bad = 0;
  PP_HIP(hipMemcpyAsync(&bad, L.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  if (bad) return fail(PP_EINTERNAL, "k_pair_index: a combine block's pairs do not match its count");
  *out = si;
  return PP_OK;
}

// Options of a run to a convergence test (see k_conv_sums); null: the
// benchmark's fixed iteration count.
struct ConvOpts {
  int32_t mode;
  double tol;
  const int32_t *d_out;
  double *deltas;
  int32_t *iters_done;   // host
};

template <typename V>
pp_status run_pagerank(const pp_csr &AT0, int32_t nrhs, int32_t iters, double c,
                       const int32_t *weights, V *r, double *sums, void *ws, size_t ws_bytes,
                       hipStream_t s, const ConvOpts *cv = nullptr) {
  const int64_t n = AT0.n, nnz = AT0.nnz;
  if (ws_bytes < ws_bytes_t<V>(n, nnz, nrhs))
    return fail(PP_EWORKSPACE, "pagerank workspace too small");
  Layout<V> L = carve<V>(ws, n, nnz, nrhs);
  const int ipt = (g_cfg.ipt == 4 || g_cfg.ipt == 16) ? g_cfg.ipt : 8;
  const int32_t D = nrhs == 1 ? kThreads * ipt : kItems;
  const int32_t nb = int32_t((n + nnz + D - 1) / D);
  const int32_t G = (nb + kFinishPer - 1) / kFinishPer;
  const double w = (1.0 - c) / double(n);
  const int32_t n32 = int32_t(n), k = nrhs;
  int lanes = 2;
  while (lanes < k) lanes <<= 1;
  if (k > 1 && g_cfg.rhs_lanes >= lanes && g_cfg.rhs_lanes <= 64 &&
      (g_cfg.rhs_lanes & (g_cfg.rhs_lanes - 1)) == 0)
    lanes = g_cfg.rhs_lanes;
  const int gN = grid_for(n, 256, 8192);
  const int gNK = grid_for(n * k, 256, 8192);
  // SpMM column tiles: T < k runs the right-hand sides T at a time, each
  // tile an n x Tt block of its own (see k_permute_in), so one pass gathers
  // rows of Tt values from a block small enough to stay in the Infinity
  // Cache; T = k is the single pass over row-major blocks.
  const int32_t T = (k > 1 && g_cfg.rhs_tile > 0 && g_cfg.rhs_tile < k) ? g_cfg.rhs_tile : k;
  const bool tiled = T < k;
  const int32_t ntile = (k + T - 1) / T;
  auto tile_cols = [&](int32_t t) { return k - t * T < T ? k - t * T : T; };
  auto tile_lanes = [&](int32_t Tt) {
    if (!tiled) return lanes;
    int gl = 2;
    while (gl < Tt) gl <<= 1;
    if (g_cfg.rhs_lanes >= gl && g_cfg.rhs_lanes <= 64) gl = g_cfg.rhs_lanes;
    return gl;
  };
  pp_status st;
  if ((st = fill_i32(reinterpret_cast<int32_t *>(L.counter), 4, 0, s)) != PP_OK) return st;

  // The matrix the iterations run on, and the vectors they start from.
  const int32_t *rp = AT0.row_ptr, *col = AT0.col;
  const V *val = static_cast<const V *>(AT0.val);
  V *x0 = r;
  Hot2 hot{nullptr, 0};
  if (weights) {
    const int32_t nrb = int32_t((n + kRelTile - 1) / kRelTile);
    hipLaunchKernelGGL(k_bucket_count, dim3(nrb), dim3(kThreads), 0, s, weights, AT0.row_ptr, n32,
                       nrb, L.bucket_off);
    st = exscan_u32(L.bucket_off, L.bucket_off, int64_t(kBuckets) * nrb,
                    reinterpret_cast<uint32_t *>(L.keys_in), nullptr, s);
    if (st != PP_OK) return st;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nrb), dim3(kThreads), 0, s, weights, AT0.row_ptr,
                       n32, nrb, L.bucket_off, L.order, L.lab, L.wnew,
                       reinterpret_cast<uint32_t *>(L.rp2));
    PP_LAUNCHED("k_bucket_count/k_bucket_scatter");
    st = exscan_u32(reinterpret_cast<uint32_t *>(L.rp2), reinterpret_cast<uint32_t *>(L.rp2), n,
                    reinterpret_cast<uint32_t *>(L.keys_in), L.total, s);
    if (st != PP_OK) return st;
    hipLaunchKernelGGL(k_set_total, dim3(1), dim3(64), 0, s, L.rp2, n32, L.total,
                       L.bucket_off + int64_t(31) * nrb, L.bucket_off + int64_t(32) * nrb,
                       L.npos);
    // Every entry's column goes through lab at random; the heaviest
    // sources' entries are cached in an L2-sized table in front of it (the
    // winners are picked into keys_in, free once rp2 is scanned).
    const int lg = hot_log2(n) + 1;
    const int nbits = n > 1 ? 32 - __builtin_clz(uint32_t(n - 1)) : 1;
    if ((st = hot_select(weights, n32, L.keys_in, lg, s)) != PP_OK) return st;
    hipLaunchKernelGGL(k_hot2_fill, dim3(grid_for(int64_t(1) << lg, 256, 1024)), dim3(256), 0, s,
                       L.keys_in, L.lab, L.hot, lg, nbits);
    PP_LAUNCHED("k_hot2_fill");
    hot = Hot2{L.hot, (1u << lg) - 1u, lg, nbits};
    rp = L.rp2;
    col = L.col2;
    val = L.val2;
    x0 = L.x2;
  }

  hipLaunchKernelGGL(k_partition, dim3(grid_for(int64_t(nb) + 1, 256, 4096)), dim3(256), 0, s,
                     rp, n32, int32_t(nnz), nb, D, L.coord);
  hipLaunchKernelGGL(k_block_flags, dim3(grid_for(nb, 256, 4096)), dim3(256), 0, s, rp, n32, nb,
                     L.coord, L.carry_row, L.closes);
  PP_LAUNCHED("k_partition/k_block_flags");

  // Column segmenting (single vector only).  Automatic choice: segment
  // once r no longer fits one XCD's 4 MiB L2, in slabs of 2 MiB of r.
  // When it applies to a relabelled matrix, its first pass writes the
  // relabelled entries; otherwise k_relabel_copy does.
  int slab_log2 = g_cfg.slab_log2;
  if (slab_log2 < 0)
    slab_log2 = n * int64_t(sizeof(V)) > (int64_t(4) << 20) ? (sizeof(V) == 4 ? 19 : 18) : 0;
  const bool segment = k == 1 && slab_log2 > 0 && iters > 0;
  SegInfo si;
  int32_t nbp = 0, ncomb = 0;
  int64_t Pr = 0;     // pairs (and their entries) left to the raw SpMV
  int64_t npos = n;   // after relabelling: vertices of weight > 0 ...
  int64_t nlive = n;  // ... and those with weight > 0 or entries in their row
  if (segment) {
    // The degree-scaled form needs the relabelled, segmented path and is
    // left out of runs to a convergence test (their pass reads x as ranks).
    const RelabelSrc rl{AT0.row_ptr, AT0.col, L.order, L.lab, AT0.val, hot, L.bad};
    // The slabs need only cover the columns that can hold entries: after
    // relabelling, the vertices of weight > 0 come first; the vertices of
    // weight <= 0 with an empty row come last (one more stream
    // synchronisation to read both counts).
    if (weights) {
      uint32_t cnt[2] = {0u, 0u};
      PP_HIP(hipMemcpyAsync(cnt, L.npos, sizeof(cnt), hipMemcpyDeviceToHost, s));
      PP_HIP(hipStreamSynchronize(s));
      npos = int64_t(cnt[0]);
      nlive = int64_t(cnt[1]);
    }
    st = build_segments<V>(L, rp, const_cast<int32_t *>(col), const_cast<V *>(val), n, npos,
                           nlive, nnz, slab_log2, weights ? &rl : nullptr,
                           g_cfg.scaled != 0 && !cv, &si, s);
    if (st != PP_OK) return st;
  }
  if (weights && !si.relabelled) {
    hipLaunchKernelGGL(k_relabel_copy<V>, dim3(nb), dim3(kThreads), 0, s, AT0.row_ptr, AT0.col,
                       static_cast<const V *>(AT0.val), L.order, L.lab, hot, L.rp2, n32,
                       L.coord, L.col2, L.val2);
    PP_LAUNCHED("k_relabel_copy");
  }
  const bool scaled = si.P > 0 && si.scaled;
  g_last_layout = (weights ? 1 : 0) | (si.P > 0 ? 2 : 0) | (scaled ? 4 : 0) |
                  (scaled && si.packed ? 8 : 0);
  if (weights) {
    // r into the new labels; in the degree-scaled form divided by the
    // weights (the gathered vector is r_u / w[u]), for the vertices of
    // weight > 0 only: no entry gathers the others.
    if (scaled)
      hipLaunchKernelGGL(k_permute_in_scaled<V>, dim3(grid_for(npos, 256, 8192)), dim3(256), 0, s,
                         r, L.order, L.wnew, int32_t(npos), L.x2);
    else
      hipLaunchKernelGGL(k_permute_in<V>, dim3(gNK), dim3(256), 0, s, r, L.order, n32, k, T,
                         L.x2);
    PP_LAUNCHED("k_permute_in");
  } else if (tiled) {
    hipLaunchKernelGGL(k_permute_in<V>, dim3(gNK), dim3(256), 0, s, r, nullptr, n32, k, T, L.x2);
    PP_LAUNCHED("k_permute_in (tiles)");
    x0 = L.x2;
  }
  if (segment) {
    if (si.P > 0) {
      Pr = si.P;
      nbp = int32_t((Pr + nnz + D - 1) / D);
      ncomb = si.ncomb;
      hipLaunchKernelGGL(k_partition, dim3(grid_for(int64_t(nbp) + 1, 256, 4096)), dim3(256), 0,
                         s, L.prp, int32_t(Pr), int32_t(nnz), nbp, D, L.coord);
      hipLaunchKernelGGL(k_block_flags, dim3(grid_for(nbp, 256, 4096)), dim3(256), 0, s, L.prp,
                         int32_t(Pr), nbp, L.coord, L.carry_row, L.closes);
      if (si.packed)
        hipLaunchKernelGGL(k_tile_slab, dim3(grid_for(nbp, 256, 4096)), dim3(256), 0, s, L.coord,
                           nbp, L.seg_es, si.ns, L.tile_slab);
      PP_LAUNCHED("k_partition/k_block_flags (pairs)");

    }
  }

  const int G0 = int((n + kSumChunk - 1) / kSumChunk);
  if (k == 1)   // sum(r_0) from the ranks themselves (x0 holds r_0 / w in the scaled form)
    hipLaunchKernelGGL(k_sum0<V>, dim3(G0), dim3(kThreads), 0, s, scaled ? r : x0, n, kSumChunk,
                       L.part, L.counter, w, sums, L.tele);
  else
    for (int32_t t = 0; t < ntile; ++t)
      hipLaunchKernelGGL(k_sum0_mm<V>, dim3(G0), dim3(kThreads), 0, s, x0 + n * t * T, n,
                         tile_cols(t), tile_lanes(tile_cols(t)), kSumChunk, L.part, L.counter, w,
                         sums ? sums + t * T : nullptr, L.tele + t * T);
  PP_LAUNCHED("k_sum0");
  const int cblk = grid_for(n, kThreads * 4, kConvBlocks);
  const uint8_t *dflag = nullptr;
  if (cv) {
    if (cv->mode != kDangNone) {
      hipLaunchKernelGGL(k_dflag, dim3(gN), dim3(256), 0, s, cv->d_out,
                         weights ? L.order : nullptr, n32, L.dflag);
      dflag = L.dflag;
    }
    hipLaunchKernelGGL(k_conv_init<V>, dim3(cblk), dim3(kThreads), 0, s, x0, n, dflag,
                       L.conv_part);
    hipLaunchKernelGGL(k_conv_fin, dim3(1), dim3(kThreads), 0, s, L.conv_part, cblk, w,
                       c / double(n), int32_t(cv->mode == kDangUniform), 0.0, cv->tol, 1, L.conv,
                       L.tele, sums, nullptr);
    PP_LAUNCHED("k_dflag/k_conv_init/k_conv_fin (r_0)");
  }

  g_timing.used = 0;
  int32_t done = 0;
  bool out_done = false;   // the last combine wrote r already
  for (int32_t it = 0; it < iters; ++it) {
    const V *x = (it & 1) ? L.y : x0;
    V *yv = (it & 1) ? x0 : L.y;
    const double *t_in = L.tele + 64 * (it & 1);
    double *t_out = L.tele + 64 * ((it + 1) & 1);
    // With a convergence test the iteration's sum(y) goes to the test's state.
    double *s_out = cv ? &L.conv->sy : sums ? sums + int64_t(it + 1) * k : nullptr;
    done = it + 1;
    if ((st = timed_begin(s)) != PP_OK) return st;
    if (si.P > 0) {
      if (scaled && si.packed)
        launch_spmv<V, true, PackedCol>(ipt, nbp, s, L.prp, L.seg_col, nullptr, x, nullptr,
                                        int32_t(Pr), L.coord, c, t_in, nullptr, L.blk_carry,
                                        L.blk_head, L.seg_part,
                                        SlabMap{L.seg_es, L.tile_slab, si.sbits, si.ns});
      else if (scaled)
        launch_spmv<V, true, uint8_t>(ipt, nbp, s, L.prp, L.seg_col,
                                      reinterpret_cast<const uint8_t *>(L.seg_val), x, nullptr,
                                      int32_t(Pr), L.coord, c, t_in, nullptr, L.blk_carry,
                                      L.blk_head, L.seg_part);
      else
        launch_spmv<V, true>(ipt, nbp, s, L.prp, L.seg_col, L.seg_val, x, nullptr, int32_t(Pr),
                             L.coord, c, t_in, nullptr, L.blk_carry, L.blk_head, L.seg_part);
      hipLaunchKernelGGL(k_fix_raw<V>, dim3(grid_for(nbp, 256, 4096)), dim3(256), 0, s,
                         L.seg_part, nbp, L.coord, L.closes, L.carry_row, L.blk_carry,
                         L.blk_head);
      // The scaled form stores y / w for the next iteration, y itself after
      // the last; a relabelled run stores the last y straight into r in the
      // caller's labels (not with a convergence test, which may stop early).
      const bool last_out = weights && !cv && it + 1 == iters;
      hipLaunchKernelGGL(k_seg_combine<V>, dim3(ncomb), dim3(kThreads), 0, s, L.seg_part, L.rpp,
                         L.pidx, L.cstart, c, t_in, last_out ? r : yv, L.blk_ysum,
                         scaled && it + 1 < iters ? L.wnew : nullptr,
                         last_out ? L.order : nullptr);
      out_done = last_out;
      // Rows [nlive, n) (count form only, whose last iteration is always
      // last_out) hold y = the teleport term: added to the sum as a count,
      // stored by the last iteration alone.
      const int64_t niso = n - si.nlive;
      if (last_out && niso > 0)
        hipLaunchKernelGGL(k_iso_out<V>, dim3(grid_for(niso, 256, 8192)), dim3(256), 0, s, L.order,
                           si.nlive, n32, t_in, r);
      hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(1024), 0, s, L.blk_ysum, ncomb, niso, t_in,
                         int32_t(sizeof(V) == 4), w, s_out, t_out);
      if ((st = timed_end(s)) != PP_OK) return st;
      PP_LAUNCHED("k_spmv raw/k_fix_raw/k_seg_combine");
    } else if (k == 1) {
      launch_spmv<V, false>(ipt, nb, s, rp, col, val, x, yv, n32, L.coord, c, t_in, L.blk_ysum,
                            L.blk_carry, L.blk_head, nullptr);
      if ((st = timed_end(s)) != PP_OK) return st;
      hipLaunchKernelGGL(k_finish<V>, dim3(G), dim3(kThreads), 0, s, yv, nb, L.coord, L.closes,
                         L.carry_row, L.blk_carry, L.blk_head, L.blk_ysum, c, t_in, L.part,
                         L.counter, w, s_out, t_out);
      PP_LAUNCHED("k_spmv/k_finish");
    } else {
      // One SpMM and its finish per column tile; the event pair spans them all.
      for (int32_t t = 0; t < ntile; ++t) {
        const int32_t Tt = tile_cols(t), gl = tile_lanes(Tt);
        const int64_t off = n * t * T;
        launch_spmm<V>(gl, nb, s, rp, col, val, x + off, yv + off, n32, Tt, L.coord, c,
                       t_in + t * T, L.blk_ysum, L.blk_carry, L.blk_head);
        hipLaunchKernelGGL(k_finish_mm<V>, dim3(G), dim3(kThreads), 0, s, yv + off, nb, Tt, gl,
                           L.coord, L.closes, L.carry_row, L.blk_carry, L.blk_head, L.blk_ysum,
                           c, t_in + t * T, L.part, L.counter, w, s_out ? s_out + t * T : nullptr,
                           t_out + t * T);
      }
      if ((st = timed_end(s)) != PP_OK) return st;
      PP_LAUNCHED("k_spmm/k_finish_mm");
    }
    if (cv) {
      // The step's dangling term, difference, sum and teleport; the host
      // reads the stop flag (one stream synchronisation per iteration).
      const double self_c = cv->mode == kDangSelf ? c : 0.0;
      hipLaunchKernelGGL(k_conv_step<V>, dim3(cblk), dim3(kThreads), 0, s, x, yv, n, dflag,
                         self_c, L.conv, L.conv_part);
      hipLaunchKernelGGL(k_conv_fin, dim3(1), dim3(kThreads), 0, s, L.conv_part, cblk, w,
                         c / double(n), int32_t(cv->mode == kDangUniform), self_c, cv->tol, 0,
                         L.conv, t_out, sums ? sums + it + 1 : nullptr,
                         cv->deltas ? cv->deltas + it : nullptr);
      PP_LAUNCHED("k_conv_step/k_conv_fin");
      double stop = 0.0;
      PP_HIP(hipMemcpyAsync(&stop, &L.conv->stop, sizeof(double), hipMemcpyDeviceToHost, s));
      PP_HIP(hipStreamSynchronize(s));
      if (stop != 0.0) break;
    }
  }
  if (cv) *cv->iters_done = done;
  const V *last = (done & 1) ? L.y : x0;
  if (out_done) return PP_OK;
  if (weights || tiled) {
    hipLaunchKernelGGL(k_permute_out<V>, dim3(gNK), dim3(256), 0, s, last,
                       weights ? L.order : nullptr, n32, k, T, r);
    PP_LAUNCHED("k_permute_out");
    return PP_OK;
  }
  if (done & 1) return copy_bytes(r, L.y, size_t(n) * k * sizeof(V), s);
  return PP_OK;
}

}  // namespace

pp_status set_kernel_timing(bool enable) {
  if (enable && g_timing.start.empty()) {
    g_timing.start.resize(kMaxTimed);
    g_timing.stop.resize(kMaxTimed);
    for (int i = 0; i < kMaxTimed; ++i) {
      PP_HIP(hipEventCreate(&g_timing.start[i]));
      PP_HIP(hipEventCreate(&g_timing.stop[i]));
    }
  }
  g_timing.on = enable;
  g_timing.used = 0;
  return PP_OK;
}

int32_t kernel_times(float *ms, int32_t cap) {
  const int n = g_timing.used < cap ? g_timing.used : cap;
  if (n <= 0) return 0;
  if (hipEventSynchronize(g_timing.stop[g_timing.used - 1]) != hipSuccess) return -1;
  for (int i = 0; i < n; ++i)
    if (hipEventElapsedTime(ms + i, g_timing.start[i], g_timing.stop[i]) != hipSuccess) return -1;
  return n;
}

int32_t k3_last_layout() { return g_last_layout; }

pp_status set_k3_config(int32_t ipt, int32_t rhs_lanes, int32_t slab_log2, int32_t scaled,
                        int32_t rhs_tile) {
  if (ipt != 4 && ipt != 8 && ipt != 16) return fail(PP_EINVAL, "items per thread %d", ipt);
  if (rhs_lanes != 0 && (rhs_lanes < 2 || rhs_lanes > 64 || (rhs_lanes & (rhs_lanes - 1))))
    return fail(PP_EINVAL, "rhs lanes %d", rhs_lanes);
  if (slab_log2 < -1 || slab_log2 > 30) return fail(PP_EINVAL, "slab log2 %d", slab_log2);
  if (scaled != 0 && scaled != 1) return fail(PP_EINVAL, "scaled form %d", scaled);
  if (rhs_tile != 0 && (rhs_tile < 2 || rhs_tile > 32 || (rhs_tile & (rhs_tile - 1))))
    return fail(PP_EINVAL, "rhs tile %d", rhs_tile);
  g_cfg.ipt = ipt;
  g_cfg.rhs_lanes = rhs_lanes;
  g_cfg.slab_log2 = slab_log2;
  g_cfg.scaled = scaled;
  g_cfg.rhs_tile = rhs_tile;
  return PP_OK;
}

void get_k3_config(int32_t *ipt, int32_t *rhs_lanes, int32_t *slab_log2, int32_t *scaled,
                   int32_t *rhs_tile) {
  *ipt = g_cfg.ipt;
  *rhs_lanes = g_cfg.rhs_lanes;
  *slab_log2 = g_cfg.slab_log2;
  *scaled = g_cfg.scaled;
  *rhs_tile = g_cfg.rhs_tile;
}

size_t pagerank_ws_bytes(int64_t n, int64_t nnz_cap, pp_dtype dt, int32_t nrhs) {
  return dt == PP_F64 ? ws_bytes_t<double>(n, nnz_cap, nrhs) : ws_bytes_t<float>(n, nnz_cap, nrhs);
}

pp_status launch_init_r(int64_t n, int32_t nrhs, uint64_t seed, pp_dtype dt, void *r, void *ws,
                        size_t ws_bytes, hipStream_t s) {
  if (ws_bytes < 64 * sizeof(unsigned long long) + 256)
    return fail(PP_EWORKSPACE, "init_r workspace too small");
  Carve cv(ws);
  unsigned long long *ksum = cv.take<unsigned long long>(64);
  pp_status st = fill_u64(reinterpret_cast<uint64_t *>(ksum), nrhs, 0ull, s);
  if (st != PP_OK) return st;
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  const dim3 grid(grid_for(n, 256, 2048), unsigned(nrhs));
  hipLaunchKernelGGL(k_init_sum, grid, dim3(256), 0, s, n, nrhs, k0, k1, ksum);
  if (dt == PP_F64)
    hipLaunchKernelGGL(k_init_write<double>, grid, dim3(256), 0, s, n, nrhs, k0, k1, ksum,
                       static_cast<double *>(r));
  else
    hipLaunchKernelGGL(k_init_write<float>, grid, dim3(256), 0, s, n, nrhs, k0, k1, ksum,
                       static_cast<float *>(r));
  PP_LAUNCHED("k_init_sum/k_init_write");
  return PP_OK;
}

pp_status launch_pagerank(const pp_csr &AT, pp_dtype dt, int32_t nrhs, int32_t iters, double c,
                          const int32_t *weights, void *r, double *sums, void *ws, size_t ws_bytes,
                          hipStream_t s) {
  if (dt == PP_F64)
    return run_pagerank<double>(AT, nrhs, iters, c, weights, static_cast<double *>(r), sums, ws,
                                ws_bytes, s);
  return run_pagerank<float>(AT, nrhs, iters, c, weights, static_cast<float *>(r), sums, ws,
                             ws_bytes, s);
}

pp_status launch_pagerank_converge(const pp_csr &AT, pp_dtype dt, int32_t max_iters, double c,
                                   double tol, int32_t mode, const int32_t *d_out,
                                   const int32_t *weights, void *r, double *sums, double *deltas,
                                   int32_t *iters_done, void *ws, size_t ws_bytes, hipStream_t s) {
  const ConvOpts cv{mode, tol, d_out, deltas, iters_done};
  if (dt == PP_F64)
    return run_pagerank<double>(AT, 1, max_iters, c, weights, static_cast<double *>(r), sums, ws,
                                ws_bytes, s, &cv);
  return run_pagerank<float>(AT, 1, max_iters, c, weights, static_cast<float *>(r), sums, ws,
                             ws_bytes, s, &cv);
}

}  // namespace pp
