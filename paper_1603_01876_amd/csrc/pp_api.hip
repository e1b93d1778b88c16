// pp_api.hip -- the extern "C" entry points of libpp.so (declared in
// include/pp.h): host-side argument checks, then the launchers of k0..k3.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "pp_common.hpp"

namespace pp {

namespace {
thread_local char g_last_error[512] = "";
}

pp_status fail(pp_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

pp_status check_hip(hipError_t e, const char *where) {
  return fail(PP_EHIP, "%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
}

namespace {

constexpr int64_t kI32Max = (int64_t(1) << 31) - 1;

bool kron_ok(const pp_kron_params *p) {
  if (!p) return false;
  if (p->scale < 1 || p->scale > 30) return false;
  if (p->edge_factor < 1 || p->edge_factor > 1024) return false;
  if (!(p->a >= 0 && p->b >= 0 && p->c >= 0 && p->d >= 0)) return false;
  const double s = p->a + p->b + p->c + p->d;
  return s > 0.999999999 && s < 1.000000001;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// Host checks shared by both batch entry points: every descriptor, so the
// kernel takes each graph as it is.  Sets the largest n of the batch.
pp_status check_graphs(const char *who, int32_t ngraphs, const pp_graph *graphs, pp_dtype dt,
                       int32_t iters, double c, int64_t *max_n_out) {
  if (ngraphs < 1 || ngraphs > (1 << 24)) return fail(PP_EINVAL, "%s: ngraphs %d", who, ngraphs);
  if (!graphs) return fail(PP_EINVAL, "%s: null graphs", who);
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "%s: dtype %d", who, int(dt));
  if (iters < 0) return fail(PP_EINVAL, "%s: iters %d", who, iters);
  if (!(c >= 0.0 && c <= 1.0)) return fail(PP_EINVAL, "%s: c = %g", who, c);
  const int64_t limit = graphs_max_n(dt);
  int64_t max_n = 0;
  for (int32_t g = 0; g < ngraphs; ++g) {
    const pp_graph &G = graphs[g];
    if (G.n < 1 || G.nnz < 0)
      return fail(PP_EINVAL, "%s: graph %d has n %lld, nnz %lld", who, g, (long long)G.n,
                  (long long)G.nnz);
    if (G.n > limit)
      return fail(PP_ERANGE, "%s: graph %d has n %lld > %lld", who, g, (long long)G.n,
                  (long long)limit);
    if (G.n + G.nnz > INT32_MAX)
      return fail(PP_ERANGE, "%s: graph %d: n + nnz beyond int32", who, g);
    if (!G.row_ptr || !G.r || (G.nnz > 0 && (!G.col || !G.val)))
      return fail(PP_EINVAL, "%s: graph %d lacks an array", who, g);
    if (G.n > max_n) max_n = G.n;
  }
  *max_n_out = max_n;
  return PP_OK;
}

}  // namespace
}  // namespace pp

using namespace pp;

extern "C" {

const char *pp_strerror(pp_status st) {
  switch (st) {
    case PP_OK: return "success";
    case PP_EINVAL: return "invalid argument";
    case PP_ERANGE: return "size out of range";
    case PP_EWORKSPACE: return "workspace missing or too small";
    case PP_EHIP: return "HIP runtime error";
    case PP_EINTERNAL: return "internal consistency check failed";
  }
  return "unknown status";
}

const char *pp_last_error(void) { return g_last_error; }

size_t pp_workspace_bytes(pp_kernel k, int64_t n, int64_t m, pp_dtype dt, int32_t nrhs) {
  // The edge-file codec sizes by edges or bytes only (n and dt unused).
  if (k == PP_TSV_FORMAT) {
    if (m < 0 || m > kI32Max || nrhs < 1 || nrhs > (1 << 20)) return size_t(-1);
    return tsv_format_ws_bytes(m, nrhs);
  }
  if (k == PP_TSV_PARSE) return m < 0 ? size_t(-1) : tsv_parse_ws_bytes(m);
  if (n < 1 || n > (int64_t(1) << 30) || m < 0 || m > kI32Max) return size_t(-1);
  if (dt != PP_F64 && dt != PP_F32) return size_t(-1);
  switch (k) {
    case PP_K0: return 0;
    case PP_K1: return radix_ws_bytes(m, 31) + 512;
    case PP_K2: return filter_ws_bytes(n, m);
    case PP_K3:
      if (nrhs < 1 || nrhs > 64 || n + m > kI32Max) return size_t(-1);
      return pagerank_ws_bytes(n, m, dt, nrhs);
    case PP_K3_GRAPHS:
      if (m < 1 || m > (int64_t(1) << 24)) return size_t(-1);
      return graphs_ws_bytes(int32_t(m));
    case PP_K2_ROWFORM:
      return transpose_ws_bytes(n, m);
    default:
      break;
  }
  return size_t(-1);
}

pp_status pp_generate(const pp_kron_params *p, int64_t *u, int64_t *v, void *stream) {
  if (!kron_ok(p)) return fail(PP_EINVAL, "pp_generate: bad generator parameters");
  if (!u || !v) return fail(PP_EINVAL, "pp_generate: null output");
  return launch_generate(*p, u, v, as_stream(stream));
}

pp_status pp_sort(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, int64_t *u_out,
                  int64_t *v_out, void *ws, size_t ws_bytes, void *stream) {
  if (scale < 1 || scale > 30) return fail(PP_ERANGE, "pp_sort: scale %d", scale);
  if (m < 0) return fail(PP_EINVAL, "pp_sort: m < 0");
  if (m > kI32Max) return fail(PP_ERANGE, "pp_sort: m = %lld >= 2^31", (long long)m);
  if (m == 0) return PP_OK;
  if (!u || !v || !u_out || !v_out) return fail(PP_EINVAL, "pp_sort: null array");
  if (u_out == u || u_out == v || v_out == u || v_out == v)
    return fail(PP_EINVAL, "pp_sort: output aliases input");
  const size_t need = radix_ws_bytes(m, 31) + 512;
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_sort: workspace needs %zu bytes", need);
  hipStream_t s = as_stream(stream);
  // The check flag lives at the start of the workspace, the sort after it.
  Carve c(ws);
  uint32_t *flag = c.take<uint32_t>(1);
  void *rest = reinterpret_cast<void *>(c.base + c.used);
  const size_t rest_bytes = ws_bytes - c.used;
  pp_status st = fill_i32(reinterpret_cast<int32_t *>(flag), 1, 0, s);
  if (st != PP_OK) return st;
  return radix_sort(RadixIn{nullptr, u, v}, RadixOut{nullptr, u_out, v_out}, m, scale, rest,
                    rest_bytes, int64_t(1) << scale, false, flag, s, true);
}

pp_status pp_sort_uv(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                     int64_t *u_out, int64_t *v_out, void *ws, size_t ws_bytes, void *stream) {
  if (scale < 1 || scale > 30) return fail(PP_ERANGE, "pp_sort_uv: scale %d", scale);
  if (m < 0) return fail(PP_EINVAL, "pp_sort_uv: m < 0");
  if (m > kI32Max) return fail(PP_ERANGE, "pp_sort_uv: m = %lld >= 2^31", (long long)m);
  if (m == 0) return PP_OK;
  if (!u || !v || !u_out || !v_out) return fail(PP_EINVAL, "pp_sort_uv: null array");
  if (u_out == u || u_out == v || v_out == u || v_out == v || u_out == v_out)
    return fail(PP_EINVAL, "pp_sort_uv: output aliases input");
  const size_t need = radix_ws_bytes(m, 31) + 512;
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_sort_uv: workspace needs %zu bytes", need);
  hipStream_t s = as_stream(stream);
  Carve c(ws);
  uint32_t *flag = c.take<uint32_t>(1);
  void *rest = reinterpret_cast<void *>(c.base + c.used);
  const size_t rest_bytes = ws_bytes - c.used;
  pp_status st = fill_i32(reinterpret_cast<int32_t *>(flag), 1, 0, s);
  if (st != PP_OK) return st;
  // LSD order: stably by v (both labels range-checked), into the outputs
  // (v in v_out, u in u_out); then stably by u, in place.  The second sort
  // takes at least two passes (9 key bits; the extra ones are zero), so no
  // pass reads the arrays it writes.
  st = radix_sort(RadixIn{nullptr, v, u}, RadixOut{nullptr, v_out, u_out}, m, scale, rest,
                  rest_bytes, int64_t(1) << scale, false, flag, s, true);
  if (st != PP_OK) return st;
  return radix_sort(RadixIn{nullptr, u_out, v_out}, RadixOut{nullptr, u_out, v_out}, m,
                    scale < 9 ? 9 : scale, rest, rest_bytes, 0, false, flag, s, false);
}

pp_status pp_tsv_format(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, char *text,
                        int64_t cap, int32_t nsplit, int64_t *split, void *ws, size_t ws_bytes,
                        void *stream) {
  if (scale < 1 || scale > 30) return fail(PP_ERANGE, "pp_tsv_format: scale %d", scale);
  if (m < 0 || m > kI32Max) return fail(PP_ERANGE, "pp_tsv_format: m = %lld", (long long)m);
  if (nsplit < 1 || nsplit > (1 << 20)) return fail(PP_EINVAL, "pp_tsv_format: nsplit %d", nsplit);
  if (!split || cap < 0 || (m > 0 && (!u || !v || !text)))
    return fail(PP_EINVAL, "pp_tsv_format: null argument");
  const size_t need = tsv_format_ws_bytes(m, nsplit);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_tsv_format: workspace needs %zu bytes", need);
  return launch_tsv_format(scale, m, u, v, text, cap, nsplit, split, ws, ws_bytes, as_stream(stream));
}

pp_status pp_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap, int64_t *u,
                       int64_t *v, int64_t *m, void *ws, size_t ws_bytes, void *stream) {
  if (!m) return fail(PP_EINVAL, "pp_tsv_parse: null m");
  *m = 0;
  if (scale < 1 || scale > 30) return fail(PP_ERANGE, "pp_tsv_parse: scale %d", scale);
  if (nbytes < 0 || cap < 0) return fail(PP_EINVAL, "pp_tsv_parse: negative size");
  if (nbytes > 0 && !text) return fail(PP_EINVAL, "pp_tsv_parse: null text");
  if (reinterpret_cast<uintptr_t>(text) % 16 != 0)
    return fail(PP_EINVAL, "pp_tsv_parse: text must be 16-byte aligned");
  const size_t need = tsv_parse_ws_bytes(nbytes);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_tsv_parse: workspace needs %zu bytes", need);
  return launch_tsv_parse(scale, text, nbytes, cap, u, v, m, ws, ws_bytes, as_stream(stream));
}

pp_status pp_write_text_files(const char *prefix, int32_t nfiles, const char *text,
                              const int64_t *split, int32_t sync, void *stream) {
  if (!prefix || !split) return fail(PP_EINVAL, "pp_write_text_files: null argument");
  if (nfiles < 1 || nfiles > 99999) return fail(PP_EINVAL, "pp_write_text_files: nfiles %d", nfiles);
  if (split[nfiles] > split[0] && !text) return fail(PP_EINVAL, "pp_write_text_files: null text");
  return write_text_files(prefix, nfiles, text, split, sync, as_stream(stream));
}

pp_status pp_read_text_files(const char *prefix, int32_t nfiles, char *text, int64_t cap,
                             int64_t *nbytes, void *stream) {
  if (!prefix || !nbytes) return fail(PP_EINVAL, "pp_read_text_files: null argument");
  if (nfiles < 1 || nfiles > 99999) return fail(PP_EINVAL, "pp_read_text_files: nfiles %d", nfiles);
  if (cap > 0 && !text) return fail(PP_EINVAL, "pp_read_text_files: null text");
  return read_text_files(prefix, nfiles, text, cap, nbytes, as_stream(stream));
}

pp_status pp_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, pp_dtype dt,
                    pp_csr *AT, int32_t *d_in, int32_t *d_out, void *ws, size_t ws_bytes,
                    void *stream) {
  if (scale < 1 || scale > 30) return fail(PP_ERANGE, "pp_filter: scale %d", scale);
  if (m < 0) return fail(PP_EINVAL, "pp_filter: m < 0");
  if (m > kI32Max) return fail(PP_ERANGE, "pp_filter: m = %lld >= 2^31", (long long)m);
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "pp_filter: dtype %d", int(dt));
  if (!AT || !AT->row_ptr || (m > 0 && (!AT->col || !AT->val || !u || !v)))
    return fail(PP_EINVAL, "pp_filter: null array");
  const int64_t n = int64_t(1) << scale;
  if (AT->n != n) return fail(PP_EINVAL, "pp_filter: AT->n = %lld, expected 2^%d", (long long)AT->n, scale);
  if (AT->cap < m) return fail(PP_EINVAL, "pp_filter: AT->cap %lld < m %lld", (long long)AT->cap, (long long)m);
  const size_t need = filter_ws_bytes(n, m);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_filter: workspace needs %zu bytes", need);
  return launch_filter(scale, m, u, v, dt, AT, d_in, d_out, ws, ws_bytes, as_stream(stream));
}

pp_status pp_transpose(const pp_csr *AT, pp_dtype dt, pp_csr *A, void *ws, size_t ws_bytes,
                       void *stream) {
  if (!AT || !A || !AT->row_ptr || !A->row_ptr) return fail(PP_EINVAL, "pp_transpose: null argument");
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "pp_transpose: dtype %d", int(dt));
  if (AT->n < 1 || AT->n > (int64_t(1) << 30))
    return fail(PP_ERANGE, "pp_transpose: n = %lld", (long long)AT->n);
  if (AT->nnz < 0 || AT->nnz > kI32Max)
    return fail(PP_ERANGE, "pp_transpose: nnz = %lld", (long long)AT->nnz);
  if (AT->nnz > 0 && (!AT->col || !AT->val || !A->col || !A->val))
    return fail(PP_EINVAL, "pp_transpose: null array");
  if (A->n != AT->n) return fail(PP_EINVAL, "pp_transpose: A->n %lld != AT->n %lld",
                                 (long long)A->n, (long long)AT->n);
  if (A->cap < AT->nnz) return fail(PP_EINVAL, "pp_transpose: A->cap %lld < nnz %lld",
                                    (long long)A->cap, (long long)AT->nnz);
  const size_t need = transpose_ws_bytes(AT->n, AT->nnz);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_transpose: workspace needs %zu bytes", need);
  return launch_transpose(*AT, dt, A, ws, ws_bytes, as_stream(stream));
}

pp_status pp_init_r(int64_t n, int32_t nrhs, uint64_t seed, pp_dtype dt, void *r, void *ws,
                    size_t ws_bytes, void *stream) {
  if (n < 1 || n > (int64_t(1) << 30)) return fail(PP_ERANGE, "pp_init_r: n = %lld", (long long)n);
  if (nrhs < 1 || nrhs > 64) return fail(PP_EINVAL, "pp_init_r: nrhs %d", nrhs);
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "pp_init_r: dtype %d", int(dt));
  if (!r) return fail(PP_EINVAL, "pp_init_r: null r");
  if (!ws) return fail(PP_EWORKSPACE, "pp_init_r: null workspace");
  return launch_init_r(n, nrhs, seed, dt, r, ws, ws_bytes, as_stream(stream));
}

pp_status pp_pagerank(const pp_csr *AT, pp_dtype dt, int32_t nrhs, int32_t iters, double c,
                      const int32_t *order_weights, void *r, double *sums, void *ws,
                      size_t ws_bytes, void *stream) {
  if (!AT || !AT->row_ptr || !r) return fail(PP_EINVAL, "pp_pagerank: null argument");
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "pp_pagerank: dtype %d", int(dt));
  if (AT->n < 1 || AT->n > (int64_t(1) << 30)) return fail(PP_ERANGE, "pp_pagerank: n = %lld", (long long)AT->n);
  if (AT->nnz < 0 || AT->nnz > AT->cap) return fail(PP_EINVAL, "pp_pagerank: nnz %lld, cap %lld", (long long)AT->nnz, (long long)AT->cap);
  if (AT->n + AT->nnz > kI32Max) return fail(PP_ERANGE, "pp_pagerank: n + nnz >= 2^31");
  if (AT->nnz > 0 && (!AT->col || !AT->val)) return fail(PP_EINVAL, "pp_pagerank: null col/val");
  if (nrhs < 1 || nrhs > 64) return fail(PP_EINVAL, "pp_pagerank: nrhs %d", nrhs);
  if (iters < 0) return fail(PP_EINVAL, "pp_pagerank: iters %d", iters);
  if (!(c >= 0.0 && c <= 1.0)) return fail(PP_EINVAL, "pp_pagerank: c = %g", c);
  const size_t need = pagerank_ws_bytes(AT->n, AT->nnz, dt, nrhs);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_pagerank: workspace needs %zu bytes", need);
  return launch_pagerank(*AT, dt, nrhs, iters, c, order_weights, r, sums, ws, ws_bytes,
                         as_stream(stream));
}

pp_status pp_pagerank_converge(const pp_csr *AT, pp_dtype dt, int32_t max_iters, double c,
                               double tol, pp_dangling mode, const int32_t *d_out,
                               const int32_t *order_weights, void *r, double *sums,
                               double *deltas, int32_t *iters_done, void *ws, size_t ws_bytes,
                               void *stream) {
  if (!AT || !AT->row_ptr || !r || !iters_done)
    return fail(PP_EINVAL, "pp_pagerank_converge: null argument");
  *iters_done = 0;
  if (dt != PP_F64 && dt != PP_F32) return fail(PP_EINVAL, "pp_pagerank_converge: dtype %d", int(dt));
  if (AT->n < 1 || AT->n > (int64_t(1) << 30)) return fail(PP_ERANGE, "pp_pagerank_converge: n = %lld", (long long)AT->n);
  if (AT->nnz < 0 || AT->nnz > AT->cap) return fail(PP_EINVAL, "pp_pagerank_converge: nnz %lld, cap %lld", (long long)AT->nnz, (long long)AT->cap);
  if (AT->n + AT->nnz > kI32Max) return fail(PP_ERANGE, "pp_pagerank_converge: n + nnz >= 2^31");
  if (AT->nnz > 0 && (!AT->col || !AT->val)) return fail(PP_EINVAL, "pp_pagerank_converge: null col/val");
  if (max_iters < 0) return fail(PP_EINVAL, "pp_pagerank_converge: max_iters %d", max_iters);
  if (!(c >= 0.0 && c <= 1.0)) return fail(PP_EINVAL, "pp_pagerank_converge: c = %g", c);
  if (mode != PP_DANGLING_NONE && mode != PP_DANGLING_UNIFORM && mode != PP_DANGLING_SELF)
    return fail(PP_EINVAL, "pp_pagerank_converge: dangling mode %d", int(mode));
  if (mode != PP_DANGLING_NONE && !d_out)
    return fail(PP_EINVAL, "pp_pagerank_converge: dangling mode %d needs d_out", int(mode));
  const size_t need = pagerank_ws_bytes(AT->n, AT->nnz, dt, 1);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_pagerank_converge: workspace needs %zu bytes", need);
  return launch_pagerank_converge(*AT, dt, max_iters, c, tol, int32_t(mode), d_out, order_weights,
                                  r, sums, deltas, iters_done, ws, ws_bytes, as_stream(stream));
}

int64_t pp_graphs_max_n(pp_dtype dt) {
  if (dt != PP_F64 && dt != PP_F32) return 0;
  return graphs_max_n(dt);
}

pp_status pp_pagerank_graphs(int32_t ngraphs, const pp_graph *graphs, pp_dtype dt, int32_t iters,
                             double c, int32_t use_graph, void *ws, size_t ws_bytes,
                             void *stream) {
  int64_t max_n = 0;
  const pp_status st = check_graphs("pp_pagerank_graphs", ngraphs, graphs, dt, iters, c, &max_n);
  if (st != PP_OK) return st;
  if (use_graph && !stream) return fail(PP_EINVAL, "pp_pagerank_graphs: graph capture needs a stream");
  const size_t need = graphs_ws_bytes(ngraphs);
  if (!ws || ws_bytes < need) return fail(PP_EWORKSPACE, "pp_pagerank_graphs: workspace needs %zu bytes", need);
  return launch_graphs(ngraphs, graphs, max_n, dt, iters, c, use_graph, ws, ws_bytes,
                       as_stream(stream));
}

pp_status pp_pagerank_graphs_noalloc(int32_t ngraphs, const pp_graph *graphs, pp_dtype dt,
                                     int32_t iters, double c, void *stream) {
  if (ngraphs > graphs_static_max())
    return fail(PP_ERANGE, "pp_pagerank_graphs_noalloc: %d graphs, at most %d", ngraphs,
                graphs_static_max());
  int64_t max_n = 0;
  const pp_status st =
      check_graphs("pp_pagerank_graphs_noalloc", ngraphs, graphs, dt, iters, c, &max_n);
  if (st != PP_OK) return st;
  return launch_graphs_static(ngraphs, graphs, max_n, dt, iters, c, as_stream(stream));
}

int32_t pp_graphs_noalloc_max(void) { return graphs_static_max(); }

pp_status pp_set_k3_config(const pp_k3_config *cfg) {
  if (!cfg) return set_k3_config(8, 0, -1, 1, 0);
  return set_k3_config(cfg->items_per_thread, cfg->rhs_lanes, cfg->slab_log2, cfg->scaled_form,
                       cfg->rhs_tile);
}

pp_status pp_get_k3_config(pp_k3_config *cfg) {
  if (!cfg) return fail(PP_EINVAL, "pp_get_k3_config: null");
  get_k3_config(&cfg->items_per_thread, &cfg->rhs_lanes, &cfg->slab_log2, &cfg->scaled_form,
                &cfg->rhs_tile);
  return PP_OK;
}

int32_t pp_k3_last_layout(void) { return k3_last_layout(); }

pp_status pp_set_kernel_timing(int enable) { return set_kernel_timing(enable != 0); }

int32_t pp_kernel_times(float *ms, int32_t cap) {
  if (!ms || cap <= 0) return 0;
  return kernel_times(ms, cap);
}

}  // extern "C"
