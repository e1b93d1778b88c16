/*
 * ppo.c -- CPU oracle for the PageRank pipeline kernels K0..K3.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded FP64 code that
 * follows the paper (Dreher et al., "PageRank Pipeline Benchmark", arXiv
 * 1603.01876) step by step.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the GPU library never does, and the two share no
 * code.  Built with -O2 -ffp-contract=off and no fast-math, so every floating
 * point operation below is a single IEEE-754 double operation in the order
 * written.
 *
 * Parity pins (what each function is checked against, tests/test_oracle_*):
 *   philox       published known-answer vectors (tests/golden/philox_kat.txt)
 *   thresholds   exact quadrant probabilities a,b,c,d (chi-square per level)
 *   permute      bijection on [0, 2^S) by exhaustive enumeration
 *   generate     range/count; per-level quadrant frequencies; independence
 *                of e-ranges; label multiset invariant under the bijection
 *   sort         numpy stable argsort by u (a library routine)
 *   sort_uv      numpy lexsort by (u, v) (a library routine)
 *   tsv_format   Python's own decimal formatting of the same edges
 *   tsv_parse    round trip; Python's int() on each field; rejects each
 *                malformed line of a list
 *   filter       dense brute force written from Sec. IV.C's Matlab lines;
 *                special graphs (complete, star, permutation) => A = 0;
 *                invariants (sum of counts, rows summing to one)
 *   init_r       exact integer sum => sum(r0) = 1 within N ulp
 *   pagerank     extended-precision (long double) reference iteration;
 *                dense power iteration; closed forms for a permutation
 *                matrix and for A = 0; the sum(r) recurrence; the Perron
 *                vector of c*A.' + (1-c)/N from numpy.linalg.eig (Sec. IV.D)
 *   step_rows    equals one pagerank iteration on every row
 *   sum_r        the sums pagerank reports; extended-precision sum
 *   digest       Python big-integer evaluation of its definition;
 *                order independence; additivity over pieces
 *   filter_rows  blocks of rows put together equal filter's CSR(A^T)
 *   pagerank_converge
 *                Perron vector of the dense matrix of each dangling mode
 *                (numpy.linalg.eig); sum(r) conserved by the two modes
 *                that make A stochastic; closed forms of every iterate
 *                and difference for a permutation matrix and for A = 0
 */
#include "ppo.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the description in Salmon, Moraes, Dror and Shaw,    */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11: ten rounds of two  */
/* 32x32->64 multiplies whose halves are xored into the other counter words */
/* together with a Weyl-sequence key.                                        */
/* ------------------------------------------------------------------------ */
void ppo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {          /* key schedule: add the Weyl constants */
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): advance by the golden  */
/* gamma and apply the variant-13 finaliser.                               */
static uint64_t splitmix64_next(uint64_t *state) {
  *state += 0x9E3779B97F4A7C15ull;
  uint64_t z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* K0 -- Kronecker (Graph500-style) generator, Sec. IV.A.                    */
/* ------------------------------------------------------------------------ */

/* p * 2^32 rounded to nearest (ties up), clamped to [0, 2^32 - 1]. */
static uint32_t prob_to_u32(double p) {
  double x = p * 4294967296.0;
  if (!(x > 0.0)) return 0u;
  double r = x + 0.5;
  if (r >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)r;   /* truncation of x + 0.5 = round half up */
}

static int kron_params_ok(const ppo_kron *p) {
  if (!p) return 0;
  if (p->scale < 1 || p->scale > 30) return 0;
  if (p->edge_factor < 1 || p->edge_factor > 1024) return 0;
  if (!(p->a >= 0 && p->b >= 0 && p->c >= 0 && p->d >= 0)) return 0;
  double s = p->a + p->b + p->c + p->d;
  if (!(s > 0.999999999 && s < 1.000000001)) return 0;
  return 1;
}

int ppo_kron_thresholds(const ppo_kron *p, uint32_t thr[3]) {
  if (!kron_params_ok(p) || !thr) return PPO_EINVAL;
  /* Level choice = quadrant of the 2x2 initiator [a b; c d]:
   *   P(u-bit = 1) = c + d;
   *   P(v-bit = 1 | u-bit = 0) = b / (a + b);
   *   P(v-bit = 1 | u-bit = 1) = d / (c + d). */
  thr[0] = prob_to_u32(p->c + p->d);
  thr[1] = (p->a + p->b > 0.0) ? prob_to_u32(p->b / (p->a + p->b)) : 0u;
  thr[2] = (p->c + p->d > 0.0) ? prob_to_u32(p->d / (p->c + p->d)) : 0u;
  return PPO_OK;
}

/* Four rounds of x = (x*m_r + a_r) mod 2^S; x ^= x >> h on S-bit labels,
 * h = max(1, S/2); m_r odd.  Each round is invertible, so the map is a
 * bijection.  Round constants are SplitMix64 outputs seeded with `seed`. */
static void permute_keys(int32_t scale, uint64_t seed, uint64_t mul[4], uint64_t add[4]) {
  uint64_t mask = (scale >= 64) ? ~0ull : ((1ull << scale) - 1ull);
  uint64_t st = seed;
  for (int r = 0; r < 4; ++r) {
    mul[r] = (splitmix64_next(&st) | 1ull) & mask;
    add[r] = splitmix64_next(&st) & mask;
  }
}

static int64_t permute_with(int32_t scale, const uint64_t mul[4], const uint64_t add[4], int64_t x) {
  uint64_t mask = (1ull << scale) - 1ull;
  int h = scale / 2;
  if (h < 1) h = 1;
  uint64_t y = (uint64_t)x;
  for (int r = 0; r < 4; ++r) {
    y = (y * mul[r] + add[r]) & mask;
    y ^= y >> h;
  }
  return (int64_t)y;
}

int64_t ppo_permute(int32_t scale, uint64_t seed, int64_t x) {
  uint64_t mul[4], add[4];
  permute_keys(scale, seed, mul, add);
  return permute_with(scale, mul, add, x);
}

int ppo_generate_range(const ppo_kron *p, int64_t e0, int64_t count, int permute,
                       int64_t *u, int64_t *v) {
  if (!kron_params_ok(p) || count < 0 || e0 < 0 || (count > 0 && (!u || !v)))
    return PPO_EINVAL;
  int64_t m = (int64_t)p->edge_factor << p->scale;
  if (e0 + count > m) return PPO_EINVAL;
  uint32_t thr[3];
  ppo_kron_thresholds(p, thr);
  uint64_t mul[4], add[4];
  permute_keys(p->scale, p->seed, mul, add);
  uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
  for (int64_t q = 0; q < count; ++q) {
    int64_t e = e0 + q;
    int64_t uu = 0, vv = 0;
    /* Level l uses the draw pair (x, y) = words (2*(l%2), 2*(l%2)+1) of
     * the Philox block with counter (e_lo, e_hi, l/2, 0). */
    for (int32_t j = 0; 2 * j < p->scale; ++j) {
      uint32_t ctr[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), (uint32_t)j, 0u};
      uint32_t w[4];
      ppo_philox4x32_10(ctr, key, w);
      for (int h = 0; h < 2; ++h) {
        int lev = 2 * j + h;
        if (lev >= p->scale) break;
        uint32_t x = w[2 * h], y = w[2 * h + 1];
        int ub = x < thr[0];
        int vb = y < (ub ? thr[2] : thr[1]);
        uu |= (int64_t)ub << lev;
        vv |= (int64_t)vb << lev;
      }
    }
    if (permute) {
      uu = permute_with(p->scale, mul, add, uu);
      vv = permute_with(p->scale, mul, add, vv);
    }
    u[q] = uu;
    v[q] = vv;
  }
  return PPO_OK;
}

/* ------------------------------------------------------------------------ */
/* K1 -- sort by start vertex, Sec. IV.B.  Counting sort over the N vertex   */
/* labels; scanning the input in order makes it stable.                     */
/* ------------------------------------------------------------------------ */
int ppo_sort(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
             int64_t *u_out, int64_t *v_out) {
  if (scale < 1 || scale > 30 || m < 0) return PPO_EINVAL;
  if (m > 0 && (!u || !v || !u_out || !v_out)) return PPO_EINVAL;
  int64_t n = (int64_t)1 << scale;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] < 0 || u[e] >= n) return PPO_EINVAL;
  int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!next) return PPO_ENOMEM;
  for (int64_t e = 0; e < m; ++e) next[u[e] + 1] += 1;
  for (int64_t i = 0; i < n; ++i) next[i + 1] += next[i];
  for (int64_t e = 0; e < m; ++e) {
    int64_t pos = next[u[e]]++;
    u_out[pos] = u[e];
    v_out[pos] = v[e];
  }
  free(next);
  return PPO_OK;
}

static int cmp_i64(const void *a, const void *b);

/* K1 variant (Sec. V asks whether the end vertices should be sorted too):
 * edges ordered by (u, v).  Edges are bucketed by u (counting sort), and
 * each bucket's end vertices are sorted in place; equal (u, v) pairs are
 * identical records, so the order among them needs no rule. */
int ppo_sort_uv(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                int64_t *u_out, int64_t *v_out) {
  int st = ppo_sort(scale, m, u, v, u_out, v_out);
  if (st != PPO_OK) return st;
  int64_t n = (int64_t)1 << scale;
  for (int64_t e = 0; e < m; ++e)
    if (v[e] < 0 || v[e] >= n) return PPO_EINVAL;
  int64_t e0 = 0;
  while (e0 < m) {
    int64_t e1 = e0;
    while (e1 < m && u_out[e1] == u_out[e0]) ++e1;
    qsort(v_out + e0, (size_t)(e1 - e0), sizeof(int64_t), cmp_i64);
    e0 = e1;
  }
  return PPO_OK;
}

/* ------------------------------------------------------------------------ */
/* Edge files, Sec. IV.A-C: one edge per line, "u<TAB>v<LF>", decimal.        */
/* ------------------------------------------------------------------------ */
int ppo_tsv_format(int64_t m, const int64_t *u, const int64_t *v, char *text, int64_t cap,
                   int64_t *nbytes) {
  if (m < 0 || cap < 0 || !nbytes || (m > 0 && (!u || !v || !text))) return PPO_EINVAL;
  int64_t pos = 0;
  char line[64];
  for (int64_t e = 0; e < m; ++e) {
    if (u[e] < 0 || v[e] < 0) return PPO_EINVAL;
    int len = snprintf(line, sizeof line, "%lld\t%lld\n", (long long)u[e], (long long)v[e]);
    if (len < 0 || pos + len > cap) return PPO_EINVAL;
    memcpy(text + pos, line, (size_t)len);
    pos += len;
  }
  *nbytes = pos;
  return PPO_OK;
}

/* Accepted text: lines of one or more decimal digits, a tab, one or more
 * decimal digits, each line ended by a newline except that the last line
 * may end at the end of the text.  Labels must lie in [0, 2^scale).
 * Anything else (empty lines, signs, spaces, other characters, more than
 * cap lines) is an error. */
int ppo_tsv_parse(int32_t scale, const char *text, int64_t nbytes, int64_t cap, int64_t *u,
                  int64_t *v, int64_t *m) {
  if (scale < 1 || scale > 30 || nbytes < 0 || cap < 0 || !m || (nbytes > 0 && !text))
    return PPO_EINVAL;
  int64_t n = (int64_t)1 << scale, count = 0, pos = 0;
  while (pos < nbytes) {
    int64_t val[2];
    for (int f = 0; f < 2; ++f) {
      int64_t x = 0;
      int digits = 0;
      while (pos < nbytes && text[pos] >= '0' && text[pos] <= '9') {
        x = x * 10 + (text[pos] - '0');
        if (x >= n) return PPO_EINVAL;
        ++digits;
        ++pos;
      }
      if (digits == 0) return PPO_EINVAL;
      char want = f == 0 ? '\t' : '\n';
      if (pos < nbytes) {
        if (text[pos] != want) return PPO_EINVAL;
        ++pos;
      } else if (f == 0) {
        return PPO_EINVAL;
      }
      val[f] = x;
    }
    if (count >= cap || !u || !v) return PPO_EINVAL;
    u[count] = val[0];
    v[count] = val[1];
    ++count;
  }
  *m = count;
  return PPO_OK;
}

/* ------------------------------------------------------------------------ */
/* K2 -- filter, Sec. IV.C.                                                  */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Bucket the edges by u (any input order) and sort each bucket by v.  On
 * return row i holds the v labels of its edges in ascending order, in
 * cols[rp[i] .. rp[i+1]). */
static int rows_sorted(int64_t n, int64_t m, const int64_t *u, const int64_t *v,
                       int64_t **rp_out, int64_t **cols_out) {
  int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t *cols = (int64_t *)malloc(((size_t)m + 1) * sizeof(int64_t));
  if (!rp || !fill || !cols) { free(rp); free(fill); free(cols); return PPO_ENOMEM; }
  for (int64_t e = 0; e < m; ++e) rp[u[e] + 1] += 1;
  for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
  memcpy(fill, rp, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) cols[fill[u[e]]++] = v[e];
  free(fill);
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] - rp[i] > 1)
      qsort(cols + rp[i], (size_t)(rp[i + 1] - rp[i]), sizeof(int64_t), cmp_i64);
  *rp_out = rp;
  *cols_out = cols;
  return PPO_OK;
}

int ppo_filter(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
               int64_t *d_in, int64_t *d_out,
               int64_t *A_rp, int32_t *A_col, double *A_val,
               int64_t *AT_rp, int32_t *AT_col, double *AT_val, int64_t *nnz) {
  if (scale < 1 || scale > 30 || m < 0) return PPO_EINVAL;
  if (m > 0 && (!u || !v)) return PPO_EINVAL;
  int64_t n = (int64_t)1 << scale;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return PPO_EINVAL;

  /* Step 1: A = sparse(u, v, 1, N, N).  Repeated (u,v) pairs add up, so an
   * entry holds the number of edges from u to v. */
  int64_t *rp = NULL, *cols = NULL;
  int st = rows_sorted(n, m, u, v, &rp, &cols);
  if (st) return st;
  int64_t *e_rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t *e_col = (int64_t *)malloc(((size_t)m + 1) * sizeof(int64_t));
  int64_t *e_cnt = (int64_t *)malloc(((size_t)m + 1) * sizeof(int64_t));
  int64_t *din = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *dout = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  char *gone = (char *)calloc((size_t)n, 1);
  if (!e_rp || !e_col || !e_cnt || !din || !dout || !gone) { st = PPO_ENOMEM; goto done; }
  int64_t ne = 0;
  e_rp[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      if (q > rp[i] && cols[q] == cols[q - 1]) {
        e_cnt[ne - 1] += 1;
      } else {
        e_col[ne] = cols[q];
        e_cnt[ne] = 1;
        ne += 1;
      }
    }
    e_rp[i + 1] = ne;
  }

  /* Step 2: d_in = sum(A, 1), the column sums of the counts. */
  for (int64_t q = 0; q < ne; ++q) din[e_col[q]] += e_cnt[q];

  /* Step 3: zero the columns whose in-degree equals the maximum (every tied
   * column) and the columns whose in-degree is one.  Both tests read the
   * in-degree computed in step 2. */
  int64_t mx = din[0];
  for (int64_t j = 1; j < n; ++j)
    if (din[j] > mx) mx = din[j];
  for (int64_t j = 0; j < n; ++j) gone[j] = (din[j] == mx) || (din[j] == 1);

  /* Step 4: d_out = sum(A, 2) over what is left; rows with d_out > 0 are
   * divided by it.  Zeroed entries leave the sparse structure. */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = e_rp[i]; q < e_rp[i + 1]; ++q)
      if (!gone[e_col[q]]) dout[i] += e_cnt[q];

  int64_t z = 0;
  for (int64_t q = 0; q < ne; ++q)
    if (!gone[e_col[q]]) z += 1;

  if (A_rp || A_col || A_val) {
    int64_t k = 0;
    if (A_rp) A_rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t q = e_rp[i]; q < e_rp[i + 1]; ++q) {
        if (gone[e_col[q]]) continue;
        if (A_col) A_col[k] = (int32_t)e_col[q];
        if (A_val) A_val[k] = (double)e_cnt[q] / (double)dout[i];
        k += 1;
      }
      if (A_rp) A_rp[i + 1] = k;
    }
  }

  if (AT_rp || AT_col || AT_val) {
    /* Transpose by a counting sort on the column; visiting rows in
     * ascending order leaves each row of A^T with u ascending. */
    int64_t *trp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!trp) { st = PPO_ENOMEM; goto done; }
    for (int64_t q = 0; q < ne; ++q)
      if (!gone[e_col[q]]) trp[e_col[q] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
    if (AT_rp) memcpy(AT_rp, trp, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t q = e_rp[i]; q < e_rp[i + 1]; ++q) {
        int64_t j = e_col[q];
        if (gone[j]) continue;
        int64_t pos = trp[j]++;
        if (AT_col) AT_col[pos] = (int32_t)i;
        if (AT_val) AT_val[pos] = (double)e_cnt[q] / (double)dout[i];
      }
    }
    free(trp);
  }
  if (d_in) memcpy(d_in, din, (size_t)n * sizeof(int64_t));
  if (d_out) memcpy(d_out, dout, (size_t)n * sizeof(int64_t));
  if (nnz) *nnz = z;
  st = PPO_OK;
done:
  free(rp); free(cols); free(e_rp); free(e_col); free(e_cnt);
  free(din); free(dout); free(gone);
  return st;
}

int ppo_filter_rows(int32_t scale, int64_t m, const int64_t *u, const int64_t *v,
                    const int64_t *rows, int64_t nrows,
                    int64_t *out_rp, int32_t *out_col, double *out_val, int64_t out_cap,
                    int64_t *out_din, int64_t *out_dout, int64_t *mx_out, int64_t *nnz) {
  if (scale < 1 || scale > 30 || m < 0 || nrows < 0) return PPO_EINVAL;
  if (m > 0 && (!u || !v)) return PPO_EINVAL;
  if (nrows > 0 && (!rows || !out_rp)) return PPO_EINVAL;
  int64_t n = (int64_t)1 << scale;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return PPO_EINVAL;
  for (int64_t q = 0; q < nrows; ++q)
    if (rows[q] < 0 || rows[q] >= n) return PPO_EINVAL;

  int st = PPO_OK;
  int64_t *din = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *dout = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  char *gone = (char *)calloc((size_t)n, 1);
  int64_t *want = (int64_t *)malloc(((size_t)n) * sizeof(int64_t));
  int64_t *cnt = NULL, *buf = NULL, *bufc = NULL;
  if (!din || !dout || !gone || !want) { st = PPO_ENOMEM; goto done; }

  /* Column sums of the count matrix = number of edges into each vertex. */
  for (int64_t e = 0; e < m; ++e) din[v[e]] += 1;
  int64_t mx = din[0];
  for (int64_t j = 1; j < n; ++j)
    if (din[j] > mx) mx = din[j];
  for (int64_t j = 0; j < n; ++j) gone[j] = (din[j] == mx) || (din[j] == 1);
  for (int64_t e = 0; e < m; ++e)
    if (!gone[v[e]]) dout[u[e]] += 1;

  /* Entries of the requested rows of A^T: for every requested v, the
   * distinct u with an edge u->v, their counts, divided by d_out[u]. */
  for (int64_t j = 0; j < n; ++j) want[j] = -1;
  for (int64_t q = 0; q < nrows; ++q) want[rows[q]] = q;
  cnt = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
  if (!cnt) { st = PPO_ENOMEM; goto done; }
  for (int64_t e = 0; e < m; ++e)
    if (want[v[e]] >= 0) cnt[want[v[e]] + 1] += 1;
  for (int64_t q = 0; q < nrows; ++q) cnt[q + 1] += cnt[q];
  buf = (int64_t *)malloc(((size_t)cnt[nrows] + 1) * sizeof(int64_t));
  bufc = (int64_t *)malloc(((size_t)nrows + 1) * sizeof(int64_t));
  if (!buf || !bufc) { st = PPO_ENOMEM; goto done; }
  memcpy(bufc, cnt, ((size_t)nrows + 1) * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    int64_t q = want[v[e]];
    if (q >= 0) buf[bufc[q]++] = u[e];
  }
  {
    int64_t k = 0;
    out_rp[0] = 0;
    for (int64_t q = 0; q < nrows; ++q) {
      int64_t b0 = cnt[q], b1 = cnt[q + 1];
      /* Every entry of a row of A^T has the same column-of-A (= rows[q]);
       * the whole row is gone when that column was removed. */
      if (!gone[rows[q]] && b1 > b0) {
        qsort(buf + b0, (size_t)(b1 - b0), sizeof(int64_t), cmp_i64);
        for (int64_t t = b0; t < b1;) {
          int64_t t2 = t;
          while (t2 < b1 && buf[t2] == buf[t]) ++t2;
          if (k >= out_cap) { st = PPO_EINVAL; goto done; }
          if (out_col) out_col[k] = (int32_t)buf[t];
          if (out_val) out_val[k] = (double)(t2 - t) / (double)dout[buf[t]];
          k += 1;
          t = t2;
        }
      }
      out_rp[q + 1] = k;
    }
  }

  if (nnz) {
    /* Total filtered nnz = distinct (u,v) pairs whose column survives.
     * Needs the input grouped by u (K1 order); each group is sorted by v
     * to find its distinct pairs. */
    int64_t z = 0;
    int64_t cap = 0;
    int64_t *tmp = NULL;
    for (int64_t e = 0; e < m;) {
      int64_t e2 = e;
      while (e2 < m && u[e2] == u[e]) ++e2;
      if (e2 < m && u[e2] < u[e]) { free(tmp); st = PPO_EINVAL; goto done; }
      int64_t len = e2 - e;
      if (len > cap) {
        free(tmp);
        cap = len;
        tmp = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
        if (!tmp) { st = PPO_ENOMEM; goto done; }
      }
      memcpy(tmp, v + e, (size_t)len * sizeof(int64_t));
      qsort(tmp, (size_t)len, sizeof(int64_t), cmp_i64);
      for (int64_t t = 0; t < len; ++t)
        if ((t == 0 || tmp[t] != tmp[t - 1]) && !gone[tmp[t]]) z += 1;
      e = e2;
    }
    free(tmp);
    *nnz = z;
  }
  if (out_din) memcpy(out_din, din, (size_t)n * sizeof(int64_t));
  if (out_dout) memcpy(out_dout, dout, (size_t)n * sizeof(int64_t));
  if (mx_out) *mx_out = mx;
done:
  free(din); free(dout); free(gone); free(want); free(cnt); free(buf); free(bufc);
  return st;
}

/* ------------------------------------------------------------------------ */
/* K3 -- PageRank, Sec. IV.D and the Appendix.                               */
/* ------------------------------------------------------------------------ */

/* The paper defines K3 in exact arithmetic; its sums (the row-vector times  */
/* matrix product and sum(r)) fix no rounding order.  Plain left-to-right    */
/* FP64 accumulation of ~1e6-term sums and of 1e4-entry columns drifts by    */
/* ~1e-12 over 20 iterations, the size of the tolerance the GPU is held to,  */
/* so every sum here is compensated (Neumaier's variant of Kahan summation):  */
/* the running FP64 sum s plus a correction c that collects each addition's  */
/* exact rounding error.  Terms are still added in ascending index order.    */
typedef struct {
  double s, c;
} csum;

static void csum_add(csum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double csum_value(const csum *a) { return a->s + a->c; }

static double sum_r(int64_t n, const double *r) {
  csum a = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) csum_add(&a, r[i]);
  return csum_value(&a);
}

int ppo_sum_r(int64_t n, const double *r, double *out) {
  if (n < 0 || !out || (n > 0 && !r)) return PPO_EINVAL;
  *out = sum_r(n, r);
  return PPO_OK;
}
int ppo_init_r(int64_t n, uint64_t seed, int32_t rhs, double *r) {
  if (n < 1 || n > ((int64_t)1 << 30) || rhs < 0 || !r) return PPO_EINVAL;
  /* r = rand(1,N); r = r ./ norm(r,1).  Each draw is a 24-bit integer k_i,
   * so the sum K is an exact integer and r_i = k_i / K is one rounding. */
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint64_t big = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)rhs, 0u, 2u};
    uint32_t w[4];
    ppo_philox4x32_10(ctr, key, w);
    uint32_t k = w[0] >> 8;
    r[i] = (double)k;
    big += k;
  }
  if (big == 0) {
    for (int64_t i = 0; i < n; ++i) r[i] = 1.0 / (double)n;
  } else {
    double kk = (double)big;
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] / kk;
  }
  return PPO_OK;
}

int ppo_pagerank(int64_t n, const int64_t *A_rp, const int32_t *A_col, const double *A_val,
                 int32_t iters, double c, double *r, double *sums) {
  if (n < 1 || iters < 0 || !A_rp || !r) return PPO_EINVAL;
  if (A_rp[n] > 0 && (!A_col || !A_val)) return PPO_EINVAL;
  csum *y = (csum *)malloc((size_t)n * sizeof(csum));
  if (!y) return PPO_ENOMEM;
  /* a = ones(1,N) .* (1-c) ./ N */
  double a = (1.0 - c) / (double)n;
  for (int32_t it = 0; it < iters; ++it) {
    double s = sum_r(n, r);
    if (sums) sums[it] = s;
    /* r = ((c .* r) * A) + (a .* sum(r,2)): the row vector c.*r times A,
     * accumulated over i in ascending order, then the teleport term. */
    for (int64_t j = 0; j < n; ++j) y[j].s = y[j].c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double cr = c * r[i];
      for (int64_t q = A_rp[i]; q < A_rp[i + 1]; ++q) csum_add(&y[A_col[q]], cr * A_val[q]);
    }
    double t = a * s;
    for (int64_t j = 0; j < n; ++j) r[j] = csum_value(&y[j]) + t;
  }
  if (sums) sums[iters] = sum_r(n, r);
  free(y);
  return PPO_OK;
}

int ppo_pagerank_converge(int64_t n, const int64_t *A_rp, const int32_t *A_col,
                          const double *A_val, int32_t max_iters, double c, double tol,
                          int32_t mode, double *r, double *sums, double *deltas,
                          int32_t *iters_done) {
  if (n < 1 || max_iters < 0 || mode < PPO_DANGLING_NONE || mode > PPO_DANGLING_SELF || !A_rp ||
      !r || !iters_done)
    return PPO_EINVAL;
  if (A_rp[n] > 0 && (!A_col || !A_val)) return PPO_EINVAL;
  csum *acc = (csum *)malloc((size_t)n * sizeof(csum));
  double *y = (double *)malloc((size_t)n * sizeof(double));
  if (!acc || !y) {
    free(acc);
    free(y);
    return PPO_ENOMEM;
  }
  double a = (1.0 - c) / (double)n;
  double cn = c / (double)n;
  double s = sum_r(n, r);
  if (sums) sums[0] = s;
  int32_t it = 0;
  while (it < max_iters) {
    /* Mass on dangling vertices: those whose row of A is empty. */
    csum dm = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
      if (A_rp[i + 1] == A_rp[i]) csum_add(&dm, r[i]);
    /* The benchmark's step: the row vector c.*r times A, sums over i in
     * ascending order.  Mode SELF gives every empty row i of A the entry
     * A(i,i) = 1, taken at its place i in that order. */
    for (int64_t j = 0; j < n; ++j) acc[j].s = acc[j].c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double cr = c * r[i];
      if (mode == PPO_DANGLING_SELF && A_rp[i + 1] == A_rp[i]) csum_add(&acc[i], cr * 1.0);
      for (int64_t q = A_rp[i]; q < A_rp[i + 1]; ++q) csum_add(&acc[A_col[q]], cr * A_val[q]);
    }
    /* Teleport (1-c)/N * sum(r); mode UNIFORM adds the dangling mass spread
     * evenly, c/N * sum of r over dangling vertices. */
    double t = a * s;
    if (mode == PPO_DANGLING_UNIFORM) t = t + cn * csum_value(&dm);
    for (int64_t j = 0; j < n; ++j) y[j] = csum_value(&acc[j]) + t;
    double s1 = sum_r(n, y);
    /* Normed sum of the differences between the two iterates, each divided
     * by its own sum (the un-adjusted iteration loses mass every step). */
    double delta = INFINITY;
    if (s > 0.0 && s1 > 0.0) {
      csum d = {0.0, 0.0};
      for (int64_t j = 0; j < n; ++j) csum_add(&d, fabs(y[j] / s1 - r[j] / s));
      delta = csum_value(&d);
    }
    for (int64_t j = 0; j < n; ++j) r[j] = y[j];
    s = s1;
    if (deltas) deltas[it] = delta;
    ++it;
    if (sums) sums[it] = s;
    if (delta <= tol) break;
  }
  *iters_done = it;
  free(acc);
  free(y);
  return PPO_OK;
}

int ppo_step_rows(int64_t n, int64_t nrows, const int64_t *rp, const int32_t *col,
                  const double *val, const double *r, double s, double c, double *y) {
  if (n < 1 || nrows < 0 || !r || (nrows > 0 && (!rp || !y))) return PPO_EINVAL;
  double a = (1.0 - c) / (double)n;
  double t = a * s;
  for (int64_t q = 0; q < nrows; ++q) {
    csum acc = {0.0, 0.0};
    for (int64_t k = rp[q]; k < rp[q + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) return PPO_EINVAL;
      csum_add(&acc, (c * r[col[k]]) * val[k]);
    }
    y[q] = csum_value(&acc) + t;
  }
  return PPO_OK;
}

/* ------------------------------------------------------------------------ */
/* Order-independent digest of an array, for comparing arrays too large to  */
/* store: D = sum_i mix(x_i XOR mix(i + g)) mod 2^64, where x_i is element   */
/* i's bit pattern zero-extended to 64 bits, g = 0x9E3779B97F4A7C15 and mix  */
/* is the SplitMix64 output function (Steele, Lea and Flood, "Fast          */
/* splittable pseudorandom number generators", OOPSLA 2014).  Test tooling: */
/* it takes part in no kernel's arithmetic.                                 */
/* ------------------------------------------------------------------------ */
static uint64_t digest_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int ppo_digest(const void *x, int64_t count, int32_t width, int64_t index0, uint64_t *out) {
  if (count < 0 || index0 < 0 || !out || (width != 4 && width != 8) || (count > 0 && !x))
    return PPO_EINVAL;
  uint64_t d = 0;
  for (int64_t i = 0; i < count; ++i) {
    uint64_t bits;
    if (width == 4) {
      uint32_t w;
      memcpy(&w, (const char *)x + 4 * i, 4);
      bits = w;
    } else {
      memcpy(&bits, (const char *)x + 8 * i, 8);
    }
    d += digest_mix(bits ^ digest_mix((uint64_t)(index0 + i) + 0x9E3779B97F4A7C15ull));
  }
  *out = d;
  return PPO_OK;
}
