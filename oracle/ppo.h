/*
 * ppo.h -- CPU oracle for the PageRank pipeline kernels K0..K3.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * implementation written from the paper (Dreher et al., "PageRank Pipeline
 * Benchmark", arXiv 1603.01876, Sec. IV.A-IV.D and the Appendix).  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it.
 * It shares no code, header or constant table with the GPU library.
 *
 * Conventions: vertices are 0-based in [0, 2^S); every array is host memory
 * owned by the caller; every function returns 0 on success or a negative
 * PPO_E* code.  Nothing here is multithreaded.
 */
#ifndef PPO_H
#define PPO_H
#include <stdint.h>

#define PPO_OK 0
#define PPO_EINVAL (-1)  /* bad argument (range, NULL, unsorted input) */
#define PPO_ENOMEM (-2)  /* malloc failed */

/* Generator parameters (Sec. IV.A): scale S, edges per vertex k, Kronecker
 * initiator probabilities a,b,c,d and the seed of the counter-based stream. */
typedef struct {
  int32_t scale;
  int32_t edge_factor;
  double a, b, c, d;
  uint64_t seed;
} ppo_kron;

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void ppo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Integer thresholds [T_u, T_v0, T_v1] the generator compares 32-bit draws
 * against. */
int ppo_kron_thresholds(const ppo_kron *p, uint32_t thr[3]);

/* Keyed bijection on S-bit labels used to permute vertex labels. */
int64_t ppo_permute(int32_t scale, uint64_t seed, int64_t x);

/* K0 (Sec. IV.A): edges e in [e0, e0+count) of the M = k*2^S edge list.
 * permute=0 returns the raw Kronecker labels (before relabelling). */
int ppo_generate_range(const ppo_kron *p, int64_t e0, int64_t count, int permute,
                       int64_t *u, int64_t *v);

/* K1 (Sec. IV.B): stable sort of (u,v) by u; ties keep input order. */
int ppo_sort(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
             int64_t *u_out, int64_t *v_out);

/* K1 variant: edges ordered by u, then v (Sec. V's question whether the
 * end vertices should be sorted too).  Same arguments as ppo_sort; v must
 * also lie in [0, 2^scale). */
int ppo_sort_uv(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                int64_t *u_out, int64_t *v_out);

/* K2 (Sec. IV.C): A = sparse(u,v,1,N,N) with counts; d_in = column sums;
 * drop columns with d_in == max(d_in) and with d_in == 1 (both from the
 * original d_in); d_out = row sums of what is left; non-empty rows divided
 * by d_out.  Outputs CSR(A) (columns ascending) and CSR(A^T) (rows = v,
 * columns u ascending).  Arrays: d_in, d_out [N]; *_rp [N+1]; *_col, *_val
 * with capacity m (nnz <= m always).  Any output pointer may be NULL. */
int ppo_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
               int64_t *d_in, int64_t *d_out,
               int64_t *A_rp, int32_t *A_col, double *A_val,
               int64_t *AT_rp, int32_t *AT_col, double *AT_val, int64_t *nnz);

/* K2 at full scale, for a sample of rows of A^T: computes d_in, max, the
 * removal mask and d_out over all m edges, then returns for each requested
 * row j (rows[q], any order) its entries in CSR-like form:
 * out_rp[q+1]-out_rp[q] entries (u ascending) in out_col/out_val, with
 * out_cap the capacity.  Also returns mx and Z (total filtered nnz). */
int ppo_filter_rows(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                    const int64_t *rows, int64_t nrows,
                    int64_t *out_rp, int32_t *out_col, double *out_val, int64_t out_cap,
                    int64_t *out_din, int64_t *out_dout, int64_t *mx, int64_t *nnz);

/* Edge files (Sec. IV.A-C): text with one edge per line, the two labels in
 * decimal separated by a tab, each line ended by a newline.  format writes
 * the m edges into text (cap bytes) and sets *nbytes; parse reads them back
 * (the last newline may be missing), checking every label against
 * [0, 2^scale), and sets *m (at most cap edges). */
int ppo_tsv_format(int64_t m, const int64_t *u, const int64_t *v, char *text, int64_t cap,
                   int64_t *nbytes);
int ppo_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap, int64_t *u,
                  int64_t *v, int64_t *m);

/* K3 init (Sec. IV.D): r_i = k_i / sum(k) with k_i the top 24 bits of a
 * Philox draw; rhs selects an independent vector. */
int ppo_init_r(int64_t n, uint64_t seed, int32_t rhs, double *r);

/* K3 (Sec. IV.D, Appendix): iters times r = ((c*r)*A) + ((1-c)/N)*sum(r),
 * on CSR(A).  sums (iters+1 entries, may be NULL) receives sum(r) before
 * each iteration and after the last.  Every sum is compensated (Neumaier),
 * terms in ascending index order. */
int ppo_pagerank(int64_t n, const int64_t *A_rp, const int32_t *A_col, const double *A_val,
                 int32_t iters, double c, double *r, double *sums);

/* K3 run until a convergence test passes (Sec. IV.D remarks that real
 * applications iterate until the normed sum of the differences between
 * iterations is small), optionally with a term for dangling vertices (rows
 * of A that are empty; Sec. IV.C/IV.D name the adjustments, Sec. V asks
 * about a diagonal entry in empty rows):
 *   PPO_DANGLING_NONE     the benchmark's iteration;
 *   PPO_DANGLING_UNIFORM  a dangling vertex's damped mass c*r_i is spread
 *                         evenly: the teleport becomes (1-c)/N*sum(r) +
 *                         c/N*sum(r over dangling vertices);
 *   PPO_DANGLING_SELF     every empty row i of A gets A(i,i) = 1.
 * Iteration k computes y from r as in ppo_pagerank (plus the mode's term),
 * delta_k = sum_j |y_j/sum(y) - r_j/sum(r)| (infinite if a sum is not
 * positive), sets r = y, and stops after the first k with delta_k <= tol or
 * after max_iters iterations.  *iters_done = iterations run; sums (max_iters
 * + 1 entries, may be NULL) gets sum(r_k) for k = 0..iters_done, deltas
 * (max_iters entries, may be NULL) gets delta_k. */
#define PPO_DANGLING_NONE 0
#define PPO_DANGLING_UNIFORM 1
#define PPO_DANGLING_SELF 2
int ppo_pagerank_converge(int64_t n, const int64_t *A_rp, const int32_t *A_col,
                          const double *A_val, int32_t max_iters, double c, double tol,
                          int32_t mode, double *r, double *sums, double *deltas,
                          int32_t *iters_done);

/* One damped step for a set of output entries, pull form: row q of the
 * given rows-of-A^T (entries rp[q]..rp[q+1], u ascending) yields
 * y[q] = sum_i (c*r_i)*val (i ascending, compensated) + ((1-c)/n)*s.  With rp = the
 * full CSR(A^T) row pointer and nrows = n this is a whole iteration. */
int ppo_step_rows(int64_t n, int64_t nrows, const int64_t *rp, const int32_t *col,
                  const double *val, const double *r, double s, double c, double *y);

/* sum(r) as K3 forms it: compensated (Neumaier), terms in ascending index
 * order.  Lets a caller split one iteration's rows over several
 * ppo_step_rows calls and still reproduce ppo_pagerank bit for bit. */
int ppo_sum_r(int64_t n, const double *r, double *out);

/* Test tooling, not part of any kernel: *out = sum over i < count of
 * mix(x_i XOR mix(index0 + i + 0x9E3779B97F4A7C15)) mod 2^64, with x_i the
 * bit pattern of element i (width 4 or 8 bytes, zero-extended) and mix the
 * SplitMix64 output function.  Order-independent, and additive over
 * consecutive pieces of an array when index0 is the piece's offset. */
int ppo_digest(const void *x, int64_t count, int32_t width, int64_t index0, uint64_t *out);

#endif
