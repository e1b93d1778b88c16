// pp_files.hip -- the benchmark's edge files (Sec. IV.A-C): one edge per
// line, the two labels as decimal strings separated by a tab, a newline
// after each edge; the number of files is free.  Text is formatted and
// parsed on the GPU; files are written and read through pinned host buffers.
//
// Format: blocks of 2048 edges.  Pass 1 sums each block's line lengths, a
// 64-bit scan gives block offsets, pass 2 formats the block's lines into LDS
// and stores them contiguously.  Split points for the files are line
// boundaries (file k takes lines [m*k/F, m*(k+1)/F)).
//
// Parse: blocks of 16 KiB of text, 64 bytes per thread.  Pass 1 counts
// newlines per block, a 64-bit scan gives each block's first line number,
// pass 2 stages each block's chunk (and the 32 bytes before it) in LDS,
// lists the chunk's newlines in order (bit masks per thread, a block scan),
// and parses one line per thread: a line starts after the previous newline
// (for the chunk's first line, found by walking back at most 22 bytes: a
// valid line has at most 22, labels below 2^30 having at most 10 digits).
// A last line without a newline ends at the end of the text.
#include "pp_common.hpp"

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace pp {

namespace {

constexpr int kFmtThreads = 256;
constexpr int kFmtPer = 8;
constexpr int kFmtEdges = kFmtThreads * kFmtPer;
constexpr int kMaxLine = 22;
constexpr int kParseThreads = 256;
constexpr int kParseBytes = 64;
constexpr int64_t kParseChunk = int64_t(kParseThreads) * kParseBytes;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ int ndigits(uint32_t x) {
  int d = 1;
  uint32_t p = 10u;
  while (d < 10 && x >= p) {
    ++d;
    p *= 10u;
  }
  return d;
}

// Writes x in decimal ending just before `end`; returns the first byte.
__device__ __forceinline__ char *put_dec(char *end, uint32_t x) {
  do {
    *--end = char('0' + x % 10u);
    x /= 10u;
  } while (x);
  return end;
}

// Line length of edge e (0 for e >= m); flags labels outside [0, n).
__device__ __forceinline__ int line_len(const int64_t *u, const int64_t *v, int64_t e, int64_t m,
                                        int64_t n, uint32_t *flag) {
  if (e >= m) return 0;
  const int64_t a = u[e], b = v[e];
  if (a < 0 || a >= n || b < 0 || b >= n) {
    atomicOr(flag, 1u);
    return 0;
  }
  return ndigits(uint32_t(a)) + ndigits(uint32_t(b)) + 2;
}

__global__ __launch_bounds__(kFmtThreads) void k_fmt_len(const int64_t *__restrict__ u,
                                                         const int64_t *__restrict__ v, int64_t m,
                                                         int64_t n, uint32_t *__restrict__ blen,
                                                         uint32_t *flag) {
  __shared__ uint32_t sh[4];
  const int64_t e0 = int64_t(blockIdx.x) * kFmtEdges + threadIdx.x * kFmtPer;
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kFmtPer; ++k) t += uint32_t(line_len(u, v, e0 + k, m, n, flag));
  const uint32_t s = block_sum256(t, sh);
  if (threadIdx.x == 0) blen[blockIdx.x] = s;
}

// Exclusive scan of n uint32 counts into n + 1 int64 offsets (the last is
// the total), one workgroup: contiguous chunks per thread.
__global__ __launch_bounds__(kScanThreads) void k_scan64(const uint32_t *__restrict__ in,
                                                         int64_t n, int64_t *__restrict__ out) {
  __shared__ int64_t sh[kScanThreads / kWave];
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const int64_t i0 = t * chunk < n ? t * chunk : n;
  const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
  int64_t sum = 0;
  for (int64_t i = i0; i < i1; ++i) sum += in[i];
  int64_t x = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sh[w] = x;
  __syncthreads();
  int64_t before = 0;
  for (int q = 0; q < w; ++q) before += sh[q];
  int64_t run = before + x - sum;
  for (int64_t i = i0; i < i1; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == kScanThreads - 1) out[n] = before + x;
}

__global__ __launch_bounds__(kFmtThreads) void k_fmt_write(const int64_t *__restrict__ u,
                                                           const int64_t *__restrict__ v,
                                                           int64_t m, int64_t n,
                                                           const int64_t *__restrict__ boff,
                                                           char *__restrict__ text,
                                                           uint32_t *flag) {
  __shared__ char s_text[kFmtEdges * kMaxLine];
  __shared__ uint32_t sh[4];
  const int64_t e0 = int64_t(blockIdx.x) * kFmtEdges + threadIdx.x * kFmtPer;
  int len[kFmtPer];
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kFmtPer; ++k) {
    len[k] = line_len(u, v, e0 + k, m, n, flag);
    t += uint32_t(len[k]);
  }
  uint32_t total;
  uint32_t off = block_exscan256(t, sh, &total);
#pragma unroll
  for (int k = 0; k < kFmtPer; ++k) {
    if (len[k] > 0) {
      char *end = s_text + off + len[k];
      end[-1] = '\n';
      char *p = put_dec(end - 1, uint32_t(v[e0 + k]));
      p[-1] = '\t';
      put_dec(p - 1, uint32_t(u[e0 + k]));
    }
    off += uint32_t(len[k]);
  }
  __syncthreads();
  char *dst = text + boff[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < total; i += kFmtThreads) dst[i] = s_text[i];
}

// split[p] = byte offset of line floor(m * p / nsplit), p = 0..nsplit.
__global__ __launch_bounds__(256) void k_fmt_split(const int64_t *__restrict__ u,
                                                   const int64_t *__restrict__ v, int64_t m,
                                                   int64_t n, const int64_t *__restrict__ boff,
                                                   int32_t nsplit, int64_t *__restrict__ split,
                                                   uint32_t *flag) {
  for (int32_t p = blockIdx.x * 256 + threadIdx.x; p <= nsplit; p += gridDim.x * 256) {
    const int64_t L = m * p / nsplit;
    const int64_t b = L / kFmtEdges;
    int64_t off = boff[b];
    for (int64_t e = b * kFmtEdges; e < L; ++e) off += line_len(u, v, e, m, n, flag);
    split[p] = off;
  }
}

__global__ __launch_bounds__(kParseThreads) void k_parse_count(const char *__restrict__ text,
                                                               int64_t nbytes,
                                                               uint32_t *__restrict__ cnt) {
  __shared__ uint32_t sh[4];
  const int64_t b0 = int64_t(blockIdx.x) * kParseChunk + int64_t(threadIdx.x) * kParseBytes;
  uint32_t c = 0;
  if (b0 + kParseBytes <= nbytes) {
    const uint4 *p = reinterpret_cast<const uint4 *>(text + b0);
#pragma unroll
    for (int q = 0; q < kParseBytes / 16; ++q) {
      const uint4 w = p[q];
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) c += ((ws[k] >> (8 * j)) & 0xFFu) == uint32_t('\n');
    }
  } else {
    for (int64_t i = b0; i < nbytes; ++i) c += text[i] == '\n';
  }
  const uint32_t s = block_sum256(c, sh);
  if (threadIdx.x == 0) cnt[blockIdx.x] = s;
}

// A block's text, staged in LDS: thread t's 64 bytes in window t, windows
// 68 bytes apart (17 words: lanes reading the same byte of their windows hit
// 64 different banks), and the 32 bytes before the chunk (the longest valid
// line is 22 bytes) in a halo.
constexpr int kHalo = 32;
constexpr int kWinStride = kParseBytes + 4;

struct Staged {
  const char *win, *halo;
  int64_t c0;
  __device__ __forceinline__ char operator[](int64_t g) const {
    const int64_t d = g - c0;
    return d >= 0 ? win[(d >> 6) * kWinStride + (d & 63)] : halo[d + kHalo];
  }
};

constexpr int kMaxLinesPerChunk = int(kParseChunk / 4);   // a valid line has >= 4 bytes

// Parses the line [start, end) (end: its newline or the end of the text)
// as line number li.
__device__ __forceinline__ void parse_line(const Staged &t, int64_t start, int64_t end,
                                           int64_t li, int64_t n, int64_t *__restrict__ u,
                                           int64_t *__restrict__ v, uint32_t *flag) {
  if (end - start > kMaxLine - 1 || end <= start) {
    atomicOr(flag, 1u);
    return;
  }
  int64_t a = -1, b = -1, x = 0;
  int digits = 0;
  for (int64_t q = start; q < end; ++q) {
    const char ch = t[q];
    if (ch >= '0' && ch <= '9') {
      x = x * 10 + (ch - '0');
      ++digits;
      if (x >= n) {
        atomicOr(flag, 1u);
        return;
      }
    } else if (ch == '\t' && a < 0 && digits > 0) {
      a = x;
      x = 0;
      digits = 0;
    } else {
      atomicOr(flag, 1u);
      return;
    }
  }
  if (a < 0 || digits == 0) {
    atomicOr(flag, 1u);
    return;
  }
  b = x;
  u[li] = a;
  v[li] = b;
}

__global__ __launch_bounds__(kParseThreads) void k_parse_lines(const char *__restrict__ text,
                                                               int64_t nbytes,
                                                               const int64_t *__restrict__ base,
                                                               int64_t nl_total, int64_t n,
                                                               int64_t *__restrict__ u,
                                                               int64_t *__restrict__ v,
                                                               uint32_t *flag) {
  __shared__ __align__(16) char s_win[kParseThreads * kWinStride];
  __shared__ __align__(16) char s_halo[kHalo];
  __shared__ uint16_t s_nl[kMaxLinesPerChunk + 1];   // line ends, offsets in the chunk
  __shared__ uint32_t sh[4];
  __shared__ int32_t s_lines;
  const int tid = threadIdx.x;
  const int64_t c0 = int64_t(blockIdx.x) * kParseChunk;
  const int64_t g1 = c0 + kParseChunk < nbytes ? c0 + kParseChunk : nbytes;
  // Stage [c0, g1) in 16-byte pieces (c0 is a multiple of 16; a piece that
  // crosses the end of the text is copied byte by byte), and the halo.
  for (int k = tid; k < kParseChunk / 16; k += kParseThreads) {
    const int64_t g = c0 + int64_t(k) * 16;
    if (g >= g1) continue;
    uint32_t *dst = reinterpret_cast<uint32_t *>(s_win + (k >> 2) * kWinStride + (k & 3) * 16);
    if (g + 16 <= nbytes) {
      const uint4 w = *reinterpret_cast<const uint4 *>(text + g);
      dst[0] = w.x;
      dst[1] = w.y;
      dst[2] = w.z;
      dst[3] = w.w;
    } else {
      char *db = reinterpret_cast<char *>(dst);
      for (int64_t i = g; i < g1; ++i) db[i - g] = text[i];
    }
  }
  if (c0 > 0 && tid < kHalo / 16)
    *reinterpret_cast<uint4 *>(s_halo + tid * 16) =
        *reinterpret_cast<const uint4 *>(text + c0 - kHalo + tid * 16);
  __syncthreads();
  const Staged st{s_win, s_halo, c0};
  // Newlines of this thread's 64 bytes, as a bit mask.
  const int64_t b0 = c0 + int64_t(tid) * kParseBytes;
  const int nb = b0 < g1 ? int(g1 - b0 < kParseBytes ? g1 - b0 : kParseBytes) : 0;
  const uint32_t *mine = reinterpret_cast<const uint32_t *>(s_win + tid * kWinStride);
  uint64_t mask = 0;
#pragma unroll
  for (int i = 0; i < kParseBytes / 4; ++i) {
    const uint32_t w = mine[i];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (((w >> (8 * j)) & 0xFFu) == uint32_t('\n')) mask |= 1ull << (4 * i + j);
  }
  if (nb < kParseBytes) mask &= nb > 0 ? (~0ull >> (kParseBytes - nb)) : 0ull;
  uint32_t all;
  uint32_t idx = block_exscan256(uint32_t(__popcll(mask)), sh, &all);
  const bool tail = nb > 0 && b0 + nb == nbytes && !((mask >> (nb - 1)) & 1ull);
  if (all > uint32_t(kMaxLinesPerChunk)) {   // shorter lines than any valid one
    if (tid == 0) atomicOr(flag, 1u);
    return;
  }
  while (mask) {
    s_nl[idx++] = uint16_t(tid * kParseBytes + __builtin_ctzll(mask));
    mask &= mask - 1;
  }
  if (tid == 0) s_lines = int32_t(all);
  __syncthreads();
  // The last line may end at the end of the text.
  if (tail) {
    s_nl[all] = uint16_t(nbytes - c0);
    s_lines = int32_t(all) + 1;
  }
  __syncthreads();
  const int32_t lines = s_lines;
  for (int32_t i = tid; i < lines; i += kParseThreads) {
    const int64_t end = c0 + s_nl[i];
    int64_t start;
    if (i > 0) {
      start = c0 + s_nl[i - 1] + 1;
    } else {   // the previous newline is at most kMaxLine bytes back, or none
      const int64_t lo = end - kMaxLine > 0 ? end - kMaxLine : 0;
      start = -1;
      for (int64_t q = end - 1; q >= lo; --q)
        if (st[q] == '\n') {
          start = q + 1;
          break;
        }
      if (start < 0) {
        if (lo > 0) {
          atomicOr(flag, 1u);
          continue;
        }
        start = 0;
      }
    }
    parse_line(st, start, end, i < int32_t(all) ? base[blockIdx.x] + i : nl_total, n, u, v,
               flag);
  }
}

struct FmtLayout {
  uint32_t *flag, *blen;
  int64_t *boff, *split;
};

FmtLayout fmt_carve(void *ws, int64_t m, int32_t nsplit, size_t *bytes = nullptr) {
  Carve c(ws);
  FmtLayout L{};
  const int64_t nb = (m + kFmtEdges - 1) / kFmtEdges;
  L.flag = c.take<uint32_t>(4);
  L.blen = c.take<uint32_t>(size_t(nb > 0 ? nb : 1));
  L.boff = c.take<int64_t>(size_t(nb + 1));
  L.split = c.take<int64_t>(size_t(nsplit + 1));
  if (bytes) *bytes = c.bytes();
  return L;
}

struct ParseLayout {
  uint32_t *flag, *cnt;
  int64_t *base;
};

ParseLayout parse_carve(void *ws, int64_t nbytes, size_t *bytes = nullptr) {
  Carve c(ws);
  ParseLayout L{};
  const int64_t nb = (nbytes + kParseChunk - 1) / kParseChunk;
  L.flag = c.take<uint32_t>(4);
  L.cnt = c.take<uint32_t>(size_t(nb > 0 ? nb : 1));
  L.base = c.take<int64_t>(size_t(nb + 1));
  if (bytes) *bytes = c.bytes();
  return L;
}

std::string file_name(const char *prefix, int32_t k) {
  char suf[16];
  std::snprintf(suf, sizeof suf, ".%05d", int(k));
  return std::string(prefix) + suf;
}

constexpr size_t kStage = size_t(16) << 20;   // bytes per pinned staging buffer
constexpr int kMaxWorkers = 8;

// One I/O worker: its own stream (default priority), two pinned staging
// buffers and events.  The stream is drained before the buffers are freed,
// so no copy is left reading or writing them.
struct Worker {
  hipStream_t s = nullptr;
  char *buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  // Host-to-device copies out of buf[b] may still run until ev[b] is done;
  // next alternates the buffers across chunks, files and calls.
  bool pending[2] = {false, false};
  uint32_t next = 0;
  std::string err;
  Worker() = default;
  Worker(const Worker &) = delete;
  Worker &operator=(const Worker &) = delete;
  ~Worker() {
    if (s) (void)hipStreamSynchronize(s);
    for (int i = 0; i < 2; ++i) {
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (buf[i]) (void)hipHostFree(buf[i]);
    }
    if (s) (void)hipStreamDestroy(s);
  }
  bool init() {
    if (hipStreamCreate(&s) != hipSuccess) return set("stream creation failed");
    for (int i = 0; i < 2; ++i) {
      if (hipHostMalloc(reinterpret_cast<void **>(&buf[i]), kStage, hipHostMallocDefault) !=
          hipSuccess)
        return set("pinned allocation failed");
      if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess)
        return set("event creation failed");
    }
    return true;
  }
  bool set(const std::string &m) {
    if (err.empty()) err = m;
    return false;
  }
};

// Writes bytes [b0, b1) of text to `name`, copy of chunk i + 1 overlapping
// the write of chunk i.
bool write_one(Worker &W, const std::string &name, const char *text, int64_t b0, int64_t b1,
               bool sync) {
  const int fd = ::open(name.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return W.set("open " + name + ": " + std::strerror(errno));
  const int64_t nchunk = (b1 - b0 + int64_t(kStage) - 1) / int64_t(kStage);
  auto issue = [&](int64_t i) {
    const int64_t o = b0 + i * int64_t(kStage);
    const int64_t len = b1 - o < int64_t(kStage) ? b1 - o : int64_t(kStage);
    return hipMemcpyAsync(W.buf[i & 1], text + o, size_t(len), hipMemcpyDeviceToHost, W.s) ==
               hipSuccess &&
           hipEventRecord(W.ev[i & 1], W.s) == hipSuccess;
  };
  bool ok = nchunk == 0 || issue(0);
  for (int64_t i = 0; ok && i < nchunk; ++i) {
    if (i + 1 < nchunk && !issue(i + 1)) {
      ok = false;
      break;
    }
    if (hipEventSynchronize(W.ev[i & 1]) != hipSuccess) {
      ok = false;
      break;
    }
    const int64_t o = b0 + i * int64_t(kStage);
    int64_t left = b1 - o < int64_t(kStage) ? b1 - o : int64_t(kStage);
    const char *p = W.buf[i & 1];
    while (left > 0) {
      const ssize_t w = ::write(fd, p, size_t(left));
      if (w < 0 && errno == EINTR) continue;
      if (w <= 0) {
        W.set("write " + name + ": " + std::strerror(errno));
        ::close(fd);
        return false;
      }
      p += w;
      left -= w;
    }
  }
  if (!ok) {
    ::close(fd);
    return W.set("device to host copy failed for " + name);
  }
  if (sync && ::fsync(fd) != 0) {
    W.set("fsync " + name + ": " + std::strerror(errno));
    ::close(fd);
    return false;
  }
  if (::close(fd) != 0) return W.set("close " + name + ": " + std::strerror(errno));
  return true;
}

// Reads `name` (size bytes) into text + dst, the read of one chunk
// overlapping the copy of the one before.  A buffer is refilled only after
// its previous copy, from this file or an earlier one, has finished.
bool read_one(Worker &W, const std::string &name, char *text, int64_t dst, int64_t size) {
  const int fd = ::open(name.c_str(), O_RDONLY);
  if (fd < 0) return W.set("open " + name + ": " + std::strerror(errno));
  int64_t done = 0;
  while (done < size) {
    const int64_t len = size - done < int64_t(kStage) ? size - done : int64_t(kStage);
    const uint32_t b = W.next++ & 1u;
    if (W.pending[b]) {
      if (hipEventSynchronize(W.ev[b]) != hipSuccess) {
        ::close(fd);
        return W.set("host to device copy failed for " + name);
      }
      W.pending[b] = false;
    }
    char *p = W.buf[b];
    int64_t got = 0;
    while (got < len) {
      const ssize_t r = ::read(fd, p + got, size_t(len - got));
      if (r < 0 && errno == EINTR) continue;
      if (r <= 0) {
        W.set("read " + name + ": " + (r == 0 ? std::string("file shrank") : std::strerror(errno)));
        ::close(fd);
        return false;
      }
      got += r;
    }
    if (hipMemcpyAsync(text + dst + done, p, size_t(len), hipMemcpyHostToDevice, W.s) !=
            hipSuccess ||
        hipEventRecord(W.ev[b], W.s) != hipSuccess) {
      ::close(fd);
      return W.set("host to device copy failed for " + name);
    }
    W.pending[b] = true;
    done += len;
  }
  ::close(fd);
  return true;
}

// The workers (streams, pinned buffers) are kept for later calls, for the
// device that was current when they were made; file calls are serialized.
// The pool is never destroyed (no HIP calls from static destructors after
// the runtime may have shut down); the process's exit releases it.
std::mutex g_io_mutex;
std::vector<std::unique_ptr<Worker>> &g_pool = *new std::vector<std::unique_ptr<Worker>>();
int g_pool_device = -1;

// Runs job(worker, file) for every file on up to kMaxWorkers threads (file
// k on worker k % W); returns the first error message, or "".
template <typename Job>
std::string run_workers(int32_t nfiles, Job job) {
  std::lock_guard<std::mutex> lock(g_io_mutex);
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return "no current device";
  if (device != g_pool_device) {
    g_pool.clear();
    g_pool_device = device;
  }
  const int nw = nfiles < kMaxWorkers ? int(nfiles) : kMaxWorkers;
  while (int(g_pool.size()) < nw) {
    std::unique_ptr<Worker> w(new Worker());
    if (!w->init()) return w->err;
    g_pool.push_back(std::move(w));
  }
  for (auto &w : g_pool) w->err.clear();
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w)
    th.emplace_back([&, w]() {
      Worker &me = *g_pool[size_t(w)];
      for (int32_t k = w; k < nfiles; k += nw)
        if (!job(me, k)) break;
      if (hipStreamSynchronize(me.s) != hipSuccess)
        me.set("stream synchronisation failed");
      else
        me.pending[0] = me.pending[1] = false;
    });
  for (auto &t : th) t.join();
  for (int w = 0; w < nw; ++w)
    if (!g_pool[size_t(w)]->err.empty()) return g_pool[size_t(w)]->err;
  return "";
}

}  // namespace

size_t tsv_format_ws_bytes(int64_t m, int32_t nsplit) {
  size_t b = 0;
  fmt_carve(nullptr, m, nsplit, &b);
  return b;
}

size_t tsv_parse_ws_bytes(int64_t nbytes) {
  size_t b = 0;
  parse_carve(nullptr, nbytes, &b);
  return b;
}

pp_status launch_tsv_format(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                            char *text, int64_t cap, int32_t nsplit, int64_t *split_host,
                            void *ws, size_t ws_bytes, hipStream_t s) {
  if (ws_bytes < tsv_format_ws_bytes(m, nsplit))
    return fail(PP_EWORKSPACE, "pp_tsv_format: workspace too small");
  FmtLayout L = fmt_carve(ws, m, nsplit);
  const int64_t n = int64_t(1) << scale;
  const int64_t nb = (m + kFmtEdges - 1) / kFmtEdges;
  pp_status st = fill_i32(reinterpret_cast<int32_t *>(L.flag), 1, 0, s);
  if (st != PP_OK) return st;
  if (nb > 0) {
    hipLaunchKernelGGL(k_fmt_len, dim3(unsigned(nb)), dim3(kFmtThreads), 0, s, u, v, m, n,
                       L.blen, L.flag);
    hipLaunchKernelGGL(k_scan64, dim3(1), dim3(kScanThreads), 0, s, L.blen, nb, L.boff);
    PP_LAUNCHED("k_fmt_len/k_scan64");
  } else {
    if ((st = fill_i32(reinterpret_cast<int32_t *>(L.boff), 2, 0, s)) != PP_OK) return st;
  }
  int64_t total = 0;
  uint32_t flag = 0;
  PP_HIP(hipMemcpyAsync(&total, L.boff + nb, sizeof(total), hipMemcpyDeviceToHost, s));
  PP_HIP(hipMemcpyAsync(&flag, L.flag, sizeof(flag), hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  if (flag) return fail(PP_EINVAL, "pp_tsv_format: label outside [0, 2^%d)", scale);
  if (total > cap) return fail(PP_EINVAL, "pp_tsv_format: text needs %lld bytes, cap %lld",
                               (long long)total, (long long)cap);
  if (nb > 0) {
    hipLaunchKernelGGL(k_fmt_write, dim3(unsigned(nb)), dim3(kFmtThreads), 0, s, u, v, m, n,
                       L.boff, text, L.flag);
    PP_LAUNCHED("k_fmt_write");
  }
  hipLaunchKernelGGL(k_fmt_split, dim3(grid_for(int64_t(nsplit) + 1, 256, 64)), dim3(256), 0, s,
                     u, v, m, n, L.boff, nsplit, L.split, L.flag);
  PP_LAUNCHED("k_fmt_split");
  PP_HIP(hipMemcpyAsync(split_host, L.split, sizeof(int64_t) * size_t(nsplit + 1),
                        hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  return PP_OK;
}

pp_status launch_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap,
                           int64_t *u, int64_t *v, int64_t *m_out, void *ws, size_t ws_bytes,
                           hipStream_t s) {
  *m_out = 0;
  if (ws_bytes < tsv_parse_ws_bytes(nbytes))
    return fail(PP_EWORKSPACE, "pp_tsv_parse: workspace too small");
  if (nbytes == 0) return PP_OK;
  ParseLayout L = parse_carve(ws, nbytes);
  const int64_t nb = (nbytes + kParseChunk - 1) / kParseChunk;
  if (nb >= (int64_t(1) << 31)) return fail(PP_ERANGE, "pp_tsv_parse: text too long");
  pp_status st = fill_i32(reinterpret_cast<int32_t *>(L.flag), 1, 0, s);
  if (st != PP_OK) return st;
  hipLaunchKernelGGL(k_parse_count, dim3(unsigned(nb)), dim3(kParseThreads), 0, s, text, nbytes,
                     L.cnt);
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(kScanThreads), 0, s, L.cnt, nb, L.base);
  PP_LAUNCHED("k_parse_count/k_scan64");
  int64_t nl = 0;
  char last = 0;
  PP_HIP(hipMemcpyAsync(&nl, L.base + nb, sizeof(nl), hipMemcpyDeviceToHost, s));
  PP_HIP(hipMemcpyAsync(&last, text + nbytes - 1, 1, hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  const int64_t m = nl + (last != '\n' ? 1 : 0);
  if (m > cap) return fail(PP_EINVAL, "pp_tsv_parse: %lld lines, capacity %lld", (long long)m,
                           (long long)cap);
  if (m > 0 && (!u || !v)) return fail(PP_EINVAL, "pp_tsv_parse: null output");
  hipLaunchKernelGGL(k_parse_lines, dim3(unsigned(nb)), dim3(kParseThreads), 0, s, text, nbytes,
                     L.base, nl, int64_t(1) << scale, u, v, L.flag);
  PP_LAUNCHED("k_parse_lines");
  uint32_t flag = 0;
  PP_HIP(hipMemcpyAsync(&flag, L.flag, sizeof(flag), hipMemcpyDeviceToHost, s));
  PP_HIP(hipStreamSynchronize(s));
  if (flag) return fail(PP_EINVAL, "pp_tsv_parse: malformed line or label outside [0, 2^%d)", scale);
  *m_out = m;
  return PP_OK;
}

pp_status write_text_files(const char *prefix, int32_t nfiles, const char *text,
                           const int64_t *split, int32_t sync, hipStream_t s) {
  for (int32_t k = 0; k < nfiles; ++k)
    if (split[k + 1] < split[k]) return fail(PP_EINVAL, "pp_write_text_files: split not ascending");
  // The text must be complete before other streams copy it out.
  PP_HIP(hipStreamSynchronize(s));
  const std::string err = run_workers(nfiles, [&](Worker &W, int32_t k) {
    return write_one(W, file_name(prefix, k), text, split[k], split[k + 1], sync != 0);
  });
  if (!err.empty()) return fail(PP_EINVAL, "pp_write_text_files: %s", err.c_str());
  return PP_OK;
}

pp_status read_text_files(const char *prefix, int32_t nfiles, char *text, int64_t cap,
                          int64_t *nbytes, hipStream_t s) {
  *nbytes = 0;
  std::vector<int64_t> size(static_cast<size_t>(nfiles), 0), at(static_cast<size_t>(nfiles), 0);
  int64_t total = 0;
  for (int32_t k = 0; k < nfiles; ++k) {
    const std::string name = file_name(prefix, k);
    struct stat sb;
    if (::stat(name.c_str(), &sb) != 0)
      return fail(PP_EINVAL, "pp_read_text_files: stat %s: %s", name.c_str(), std::strerror(errno));
    size[size_t(k)] = int64_t(sb.st_size);
    at[size_t(k)] = total;
    total += int64_t(sb.st_size);
  }
  if (total > cap) return fail(PP_EINVAL, "pp_read_text_files: %lld bytes, capacity %lld",
                               (long long)total, (long long)cap);
  // Earlier work on the caller's stream may still use the buffer.
  PP_HIP(hipStreamSynchronize(s));
  const std::string err = run_workers(nfiles, [&](Worker &W, int32_t k) {
    return read_one(W, file_name(prefix, k), text, at[size_t(k)], size[size_t(k)]);
  });
  if (!err.empty()) return fail(PP_EINVAL, "pp_read_text_files: %s", err.c_str());
  *nbytes = total;
  return PP_OK;
}

}  // namespace pp
