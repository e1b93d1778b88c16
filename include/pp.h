/*
 * pp.h -- C ABI of the MI355X (gfx950) PageRank pipeline library libpp.so.
 *
 * Implements the four kernels of the PageRank Pipeline Benchmark (Dreher et
 * al., arXiv 1603.01876, Sec. IV): K0 Kronecker edge generation (Sec. IV.A),
 * K1 sort by start vertex (Sec. IV.B), K2 filter into a normalised sparse
 * matrix (Sec. IV.C) and K3 PageRank iterations (Sec. IV.D and the
 * Appendix).
 *
 * Conventions for every entry point:
 *  - Array pointers are DEVICE memory owned by the caller, unless marked
 *    [host].  The library never allocates device memory; scratch comes from
 *    a caller-provided workspace of at least pp_workspace_bytes() bytes
 *    (any alignment; the library aligns inside it).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously; outputs are defined once the stream has been
 *    synchronised.  Exceptions are noted per call (pp_sort, pp_filter).
 *  - Arguments are checked on the host before anything is enqueued; a
 *    failed check returns PP_EINVAL / PP_ERANGE / PP_EWORKSPACE and leaves
 *    every output untouched.  PP_EHIP reports a HIP runtime failure;
 *    pp_last_error() then returns the HIP message.
 *  - Vertex labels are 0-based in [0, 2^S).  Edge lists are int64.  Sparse
 *    matrices use int32 row pointers and column indices, so edge counts
 *    must stay below 2^31 (PP_ERANGE otherwise).
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PP_OK = 0,
  PP_EINVAL = 1,     /* invalid argument or input that violates a precondition */
  PP_ERANGE = 2,     /* size beyond the int32 index range or scale > 30 */
  PP_EWORKSPACE = 3, /* workspace NULL or smaller than pp_workspace_bytes() */
  PP_EHIP = 4,       /* HIP runtime or launch failure */
  PP_EINTERNAL = 5   /* a device-side consistency check of the library failed (a library bug) */
} pp_status;

typedef enum {
  PP_F64 = 0, /* FP64 matrix values and ranks */
  PP_F32 = 1  /* FP32 values and ranks, compensated FP32 row sums;
                 sum(r), the teleport scalar and 1/d_out stay FP64 */
} pp_dtype;

typedef enum {
  PP_K0 = 0,
  PP_K1 = 1,
  PP_K2 = 2,
  PP_K3 = 3,
  PP_K3_GRAPHS = 4, /* pp_pagerank_graphs; the m argument is the number of graphs */
  PP_K2_ROWFORM = 5, /* pp_transpose; the m argument is the number of stored entries */
  PP_TSV_FORMAT = 6, /* pp_tsv_format; m = edges, nrhs = number of parts (files) */
  PP_TSV_PARSE = 7   /* pp_tsv_parse; m = bytes of text */
} pp_kernel;

/* Kronecker generator parameters [host] (Sec. IV.A): N = 2^scale vertices,
 * M = edge_factor * N edges, initiator quadrant probabilities a,b,c,d
 * (non-negative, summing to 1), seed of the counter-based random stream. */
typedef struct {
  int32_t scale;       /* 1..30 */
  int32_t edge_factor; /* 1..1024; the paper's k = 16 */
  double a, b, c, d;
  uint64_t seed;
} pp_kron_params;

/* A square sparse matrix in CSR form.  The struct itself is [host]; the
 * three arrays are device memory.  row_ptr has n+1 entries, col and val
 * have room for `cap` entries; val holds FP64 or FP32 values per the dtype
 * argument of the call that uses it.  nnz is the number of stored entries
 * (set by pp_filter, read by pp_pagerank). */
typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t cap;
  int32_t *row_ptr;
  int32_t *col;
  void *val;
} pp_csr;

/* One graph of a pp_pagerank_graphs batch (the descriptor table is host
 * memory; the arrays it points to are device memory):
 * CSR(A^T) with n rows and nnz entries (as written by pp_filter, values of
 * the batch's dtype), the output vector r (n entries), optional sums
 * (iters+1 FP64 entries, NULL = not returned) and the seed of the graph's
 * initial vector. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  void *r;
  double *sums;
  uint64_t seed;
} pp_graph;

/* Text for a status code (static storage). */
const char *pp_strerror(pp_status st);

/* Text of the most recent failure in this thread ("" if none). */
const char *pp_last_error(void);

/* Workspace bytes needed by kernel k for n vertices, m edges (K0..K2) or
 * at most m stored entries (K3), value type dt and nrhs right-hand sides
 * (K3; 1 otherwise).  Returns 0 when no workspace is needed and
 * (size_t)-1 for arguments out of range. */
size_t pp_workspace_bytes(pp_kernel k, int64_t n, int64_t m, pp_dtype dt, int32_t nrhs);

/* K0 (Sec. IV.A): writes the M = edge_factor * 2^scale edges (u[e], v[e]),
 * e = 0..M-1, of the Kronecker graph: per level, quadrant (u-bit, v-bit)
 * drawn with probabilities a,b,c,d from Philox4x32-10 keyed by the seed,
 * then both labels relabelled by a seed-keyed bijection on scale bits.
 * Self-loops and repeated edges are kept.  u, v: M int64 each.
 * Needs no workspace.  The result depends only on the parameters. */
pp_status pp_generate(const pp_kron_params *p, int64_t *u, int64_t *v, void *stream);

/* K1 (Sec. IV.B): stable sort of the m edges (u, v) by u, so that
 * u_out[i-1] <= u_out[i]; edges with equal u keep their input order.
 * Requires 0 <= u[i], v[i] < 2^scale (checked on the device: PP_EINVAL).
 * u_out/v_out must not overlap u/v.  Synchronises `stream` once, after the
 * first pass, to report the input check. */
pp_status pp_sort(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                  int64_t *u_out, int64_t *v_out, void *ws, size_t ws_bytes, void *stream);

/* K1 variant (Sec. V asks whether the end vertices should be sorted too):
 * the edges ordered by u, then by v.  Arguments, workspace and errors as
 * pp_sort; both labels are checked against [0, 2^scale) and u_out, v_out
 * must be distinct from the inputs and from each other.  Runs two stable
 * radix sorts (by v, then by u). */
pp_status pp_sort_uv(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, int64_t *u_out,
                     int64_t *v_out, void *ws, size_t ws_bytes, void *stream);

/* K2 (Sec. IV.C): from the K1 output (edges sorted by u), forms the count
 * matrix A(u,v) = number of edges u->v, the in-degrees d_in = column sums
 * of counts, removes every column whose in-degree equals the maximum and
 * every column whose in-degree is 1 (both tests on the same d_in), takes
 * d_out = row sums of the surviving counts and divides each surviving
 * entry by its row's d_out (IEEE FP64 division; PP_F32 stores the quotient
 * rounded to FP32).  Writes CSR(A^T): AT->row_ptr[v] .. AT->row_ptr[v+1]
 * lists the sources u (ascending) of the surviving entries in column v of
 * A, with their values; AT->n must be 2^scale and AT->cap >= m.
 * d_in / d_out (2^scale int32 each, NULL = not returned).
 * Input check on the device: labels in range and u non-decreasing, else
 * PP_EINVAL.  Synchronises `stream` twice (input check, then the entry
 * count, which it stores in AT->nnz). */
pp_status pp_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, pp_dtype dt,
                    pp_csr *AT, int32_t *d_in, int32_t *d_out, void *ws, size_t ws_bytes,
                    void *stream);

/* Row form of K2's matrix (Sec. IV.C, A indexed by (u, v)): writes CSR(A)
 * from the CSR(A^T) that pp_filter produced -- A->row_ptr[u] ..
 * A->row_ptr[u+1] lists the columns v (ascending) of row u with the same
 * values, copied bit for bit (value type dt).  A->n must equal AT->n and
 * A->cap >= AT->nnz; sets A->nnz.  Workspace:
 * pp_workspace_bytes(PP_K2_ROWFORM, n, AT->nnz, dt, 1). */
pp_status pp_transpose(const pp_csr *AT, pp_dtype dt, pp_csr *A, void *ws, size_t ws_bytes,
                       void *stream);

/* Edge files (Sec. IV.A-C): text with one edge per line, the two labels as
 * decimal strings separated by a tab, a newline after each edge; the number
 * of files is free.  K0 writes such files, K1 reads them and writes the
 * sorted edges the same way, K2 reads those.
 *
 * pp_tsv_format: the m edges (u, v: device int64, labels in [0, 2^scale))
 * as text into `text` (device, cap bytes; at most 22 bytes per edge).  The
 * lines are cut into nsplit parts of nearly equal edge counts (part k =
 * lines [m*k/nsplit, m*(k+1)/nsplit)); split (host, nsplit + 1 entries)
 * receives the byte offset of each part, split[nsplit] = total bytes.
 * PP_EINVAL for a label out of range or text longer than cap.  Synchronizes
 * the stream.  Workspace: pp_workspace_bytes(PP_TSV_FORMAT, 0, m, dt,
 * nsplit).
 *
 * pp_tsv_parse: the edges of `text` (device, nbytes, 16-byte aligned) into
 * u, v (device, cap entries); *m (host) = edges read.  Every line must be
 * digits, a tab, digits (the last newline may be missing), labels in
 * [0, 2^scale); anything else, or more than cap lines, is PP_EINVAL (u and v
 * then hold partial results).  Synchronizes the stream.  Workspace:
 * pp_workspace_bytes(PP_TSV_PARSE, 0, nbytes, dt, 1).
 *
 * pp_write_text_files: writes text[split[k], split[k+1]) (device) to file
 * "<prefix>.<k>" (k with five digits) for k < nfiles, through pinned host
 * staging buffers: up to 8 I/O workers, each with its own stream and two
 * 16 MiB pinned buffers, made on first use for the current device and kept
 * for later file calls until the process ends (at most 256 MiB of pinned
 * host memory); file calls are serialised.  With sync the files are
 * flushed to storage (fsync) before the call returns.
 * pp_read_text_files: reads files "<prefix>.0" .. ".<nfiles-1>" back to
 * back into text (device, cap bytes); *nbytes (host) = total.  Both return
 * PP_EINVAL with the system's message for a file that cannot be opened,
 * read or written, and leave the stream idle. */
pp_status pp_tsv_format(int32_t scale, int64_t m, const int64_t *u, const int64_t *v, char *text,
                        int64_t cap, int32_t nsplit, int64_t *split, void *ws, size_t ws_bytes,
                        void *stream);
pp_status pp_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap, int64_t *u,
                       int64_t *v, int64_t *m, void *ws, size_t ws_bytes, void *stream);
pp_status pp_write_text_files(const char *prefix, int32_t nfiles, const char *text,
                              const int64_t *split, int32_t sync, void *stream);
pp_status pp_read_text_files(const char *prefix, int32_t nfiles, char *text, int64_t cap,
                             int64_t *nbytes, void *stream);

/* K3 initial vector (Sec. IV.D, r = rand(1,N); r = r./norm(r,1)): for each
 * right-hand side j < nrhs, k_ij = top 24 bits of word 0 of Philox4x32-10
 * keyed by the seed at counter (i, j, 0, 2); r_ij = k_ij / sum_i k_ij, one
 * IEEE FP64 division of exact integers (FP32: that quotient rounded); if the
 * sum is 0, r_ij = 1/n.  r: n x nrhs, row-major, of the dtype.  The integer
 * sums live in the workspace: any workspace sized for pp_pagerank with the
 * same n, dtype and nrhs is large enough (pp_workspace_bytes(PP_K3, n, 0,
 * dt, nrhs) is the minimum). */
pp_status pp_init_r(int64_t n, int32_t nrhs, uint64_t seed, pp_dtype dt, void *r, void *ws,
                    size_t ws_bytes, void *stream);

/* K3 (Sec. IV.D and the Appendix): `iters` iterations of
 *   r_j <- c * sum_i r_i * A(i,j) + ((1-c)/N) * sum(r)
 * on CSR(A^T) (as written by pp_filter), for nrhs independent right-hand
 * sides stored row-major in r (n x nrhs, in/out).  nrhs = 1 runs the
 * sparse matrix-vector form; nrhs in 2..64 runs the sparse matrix-dense
 * matrix form.  sums (device, (iters+1) x nrhs FP64, may be NULL) receives
 * sum(r) of each right-hand side before every iteration and after the last
 * one.  Dangling rows are not adjusted, so sum(r) may decay.
 * order_weights (device, n int32, may be NULL): per-vertex weights, e.g.
 * pp_filter's d_out.  When given, the iterations run on a copy of the
 * matrix (in the workspace) whose vertices are relabelled by decreasing
 * floor(log2(weight + 1)) for weights > 0, then weights <= 0 with entries
 * in their row of A^T, then weights <= 0 without, ties in label order, so
 * that frequently gathered ranks share cache lines; r is permuted in and out, so inputs and outputs
 * keep the original labels.  When the weights are pp_filter's d_out for
 * this matrix, a segmented run also stores the entries as integer counts
 * and gathers r_i / d_out[i] (the degree-scaled form; see scaled_form in
 * pp_k3_config): A = D^-1 C with C the count matrix of Sec. IV.C, verified
 * entry by entry.  The weights only affect speed and the rounding and order
 * of floating-point operations.  The caller must supply a valid CSR (row_ptr
 * non-decreasing from 0 to nnz, columns in [0, n)); pp_filter's output
 * always is. */
pp_status pp_pagerank(const pp_csr *AT, pp_dtype dt, int32_t nrhs, int32_t iters, double c,
                      const int32_t *order_weights, void *r, double *sums, void *ws,
                      size_t ws_bytes, void *stream);

/* Dangling vertices (rows of A without entries, i.e. d_out == 0): the
 * adjustment applied by pp_pagerank_converge (Sec. IV.C-D name such
 * adjustments; Sec. V asks about a diagonal entry in empty rows). */
typedef enum {
  PP_DANGLING_NONE = 0,    /* the benchmark's iteration: sum(r) decays */
  PP_DANGLING_UNIFORM = 1, /* a dangling vertex's damped mass c*r_i is spread
                              evenly: teleport (1-c)/N*sum(r) + c/N*sum of r
                              over dangling vertices */
  PP_DANGLING_SELF = 2     /* every empty row i of A gets A(i,i) = 1 */
} pp_dangling;

/* K3 run until a convergence test passes (Sec. IV.D: applications iterate
 * until the normed sum of the differences between iterations is small),
 * single right-hand side.  Iteration k computes r_{k+1} from r_k as
 * pp_pagerank does, plus the term of `mode`, then
 *   delta_k = sum_j | r_{k+1,j} / sum(r_{k+1}) - r_{k,j} / sum(r_k) |
 * (FP64; +infinity unless both sums are positive).  It stops after the first
 * k with delta_k <= tol, or after max_iters iterations (tol < 0: never
 * early).  r (device, n values of dt) is r_0 on entry and the last iterate
 * on return; *iters_done (host) = iterations run.  sums (device, max_iters
 * + 1 FP64, may be NULL) gets sum(r_k) for k = 0..*iters_done; deltas
 * (device, max_iters FP64, may be NULL) gets delta_k.  d_out (device, n
 * int32, pp_filter's out-degrees) marks the dangling vertices and is
 * required unless mode is PP_DANGLING_NONE; order_weights as in
 * pp_pagerank.  The workspace is pp_pagerank's for nrhs = 1.  The host
 * reads a stop flag after every iteration, so the call synchronizes the
 * stream once per iteration and returns with it idle.  In FP32 the
 * differences bottom out near the rounding of the iterates (~1e-7), so
 * useful tolerances start around 1e-6. */
pp_status pp_pagerank_converge(const pp_csr *AT, pp_dtype dt, int32_t max_iters, double c,
                               double tol, pp_dangling mode, const int32_t *d_out,
                               const int32_t *order_weights, void *r, double *sums,
                               double *deltas, int32_t *iters_done, void *ws, size_t ws_bytes,
                               void *stream);

/* K3 (Sec. IV.D) for a batch of independent small graphs in one persistent
 * launch: for every graph, r_0 as pp_init_r (right-hand side 0, the graph's
 * seed) followed by `iters` iterations as pp_pagerank, with r and the
 * iterate held in on-chip memory.  graphs is a [host] array of ngraphs
 * descriptors (the arrays they point to are device memory); it is read
 * during the call and copied into the workspace ahead of the launch.
 * Workgroups take graphs in array order, so listing the largest first
 * balances the launch.  Every descriptor is checked on the host before
 * anything is enqueued: n in [1, pp_graphs_max_n(dt)] (PP_ERANGE above it),
 * nnz >= 0, n + nnz < 2^31 (PP_ERANGE), row_ptr and r present, col and val
 * present when nnz > 0 (PP_EINVAL); a failed check launches nothing and
 * leaves every output untouched.  use_graph != 0 records the launch into a
 * hipGraph on first use and replays it on later calls with the same
 * workspace, stream, batch size, iteration count, damping and largest n
 * (stream must not be NULL then); use_graph == 0 launches directly.
 * Workspace: pp_workspace_bytes(PP_K3_GRAPHS, 1, ngraphs, dt, 1); calls
 * sharing a workspace must not overlap. */
pp_status pp_pagerank_graphs(int32_t ngraphs, const pp_graph *graphs, pp_dtype dt, int32_t iters,
                             double c, int32_t use_graph, void *ws, size_t ws_bytes,
                             void *stream);

/* Largest n a pp_pagerank_graphs graph may have with value type dt (the
 * on-chip memory of one workgroup holds two n-vectors). */
int64_t pp_graphs_max_n(pp_dtype dt);

/* pp_pagerank_graphs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, checks, kernels and results as a direct
 * launch (use_graph == 0) of pp_pagerank_graphs, but without a workspace
 * argument.  The queue counter and the descriptor table live in a static
 * device array of the library, sized for pp_graphs_noalloc_max() graphs
 * (65536: 64 B per graph plus 512 B, about 4 MiB), which every GPU the
 * library runs on holds until the process ends; its address is looked up
 * once per device on the first call made with that device current.
 * ngraphs above pp_graphs_noalloc_max() is PP_ERANGE (nothing launched).
 * The call enqueues a fill kernel that resets the queue counter, the copy of
 * the [host] descriptor table and the persistent kernel, and allocates
 * nothing (no hipMalloc, hipFree or allocating library call).  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams or threads) race on it and
 * must be serialised by the caller. */
pp_status pp_pagerank_graphs_noalloc(int32_t ngraphs, const pp_graph *graphs, pp_dtype dt,
                                     int32_t iters, double c, void *stream);

/* Largest batch pp_pagerank_graphs_noalloc accepts. */
int32_t pp_graphs_noalloc_max(void);

/* Launch configuration of pp_pagerank (process-wide; the autotuner in the
 * Python package measures the candidates on a given matrix and sets the
 * fastest).  items_per_thread in {4, 8, 16}: merge-path items per thread of
 * the sparse matrix-vector kernel (a workgroup tile is 256 times that);
 * rhs_lanes: lanes per right-hand-side group of the sparse matrix-dense
 * matrix kernel, 0 = the next power of two >= nrhs, else a power of two in
 * [nrhs, 64].  slab_log2 in [-1, 30]: 0 iterates over the whole matrix
 * in one pass; k > 0 (nrhs == 1 only) cuts the columns into slabs of 2^k
 * vertices (widened until there are at most 256) and stores the matrix
 * slab by slab, so each pass gathers from an L2-sized range of r
 * (column segmenting, Zhang et al., IEEE BigData 2017); -1 chooses: slabs
 * of 2 MiB of r (2^19 FP32 or 2^18 FP64 vertices) once r exceeds 4 MiB,
 * else one pass.  The segmented layout is built inside each pp_pagerank
 * call, which then synchronizes its stream once to read the number of
 * (slab, row) pairs.  scaled_form in {0, 1}: with 1, a pp_pagerank call
 * that relabels (order_weights given) and segments stores each entry as
 * its integer count k = A(i,j) * w[i] instead of its value whenever every
 * entry verifies as A(i,j) == V(k / w[i]) with k in [1, 255] (as for
 * pp_filter's output with its d_out as the weights: Sec. IV.C's counts
 * divided by out-degrees), and the iterations gather r_i / w[i]; any entry
 * that does not verify keeps the values (one more stream synchronisation
 * reads the verdict).  rhs_tile in {0, 2, 4, 8, 16, 32}: with nrhs above
 * it, the sparse matrix-dense matrix form runs the right-hand sides rhs_tile
 * columns at a time, each tile held as an n x rhs_tile block of its own in
 * the workspace (a tile's rows are gathered from a block small enough to
 * stay in the 256 MB Infinity Cache); 0 runs all columns in one pass.
 * Results do not depend on the configuration beyond the rounding of
 * floating-point products and the order of sums.  pp_set_k3_config(NULL)
 * restores the defaults (8, 0, -1, 1, 0). */
typedef struct {
  int32_t items_per_thread;
  int32_t rhs_lanes;
  int32_t slab_log2;
  int32_t scaled_form;
  int32_t rhs_tile;
} pp_k3_config;
pp_status pp_set_k3_config(const pp_k3_config *cfg);
pp_status pp_get_k3_config(pp_k3_config *cfg);

/* Layout the most recent pp_pagerank / pp_pagerank_converge call (in this
 * process) iterated on: bit 0 vertices relabelled, bit 1 columns
 * segmented, bit 2 entries stored as counts (degree-scaled form), bit 3
 * each count packed with its column inside the slab into one 4-byte word.
 * 0 before any call.  Instrumentation for tests and benchmarks. */
int32_t pp_k3_last_layout(void);

/* Benchmark instrumentation.  While enabled (enable != 0), each
 * pp_pagerank call records a pair of HIP events on its stream around every
 * launch of its sparse product kernel (one per iteration); the events are
 * created once by this call and reused.  pp_kernel_times() waits for the
 * last recorded pair and copies up to `cap` durations in milliseconds of
 * the most recent pp_pagerank call into ms [host]; it returns how many were
 * recorded (0 if none, -1 on a HIP error).  Process-wide state, meant for a
 * single benchmarking thread. */
pp_status pp_set_kernel_timing(int enable);
int32_t pp_kernel_times(float *ms, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
