// k2_transpose.hip -- the row form CSR(A) of K2's matrix (Sec. IV.C builds A
// with rows u, columns v) from the CSR(A^T) that pp_filter writes.
//
// Entry j of CSR(A^T) sits in row v (a column of A) and names its source
// u = col[j].  A stable radix sort of the keys u << 32 | j by u lists the
// entries row by row of A; inside a row they keep the CSR(A^T) order, in
// which v ascends, so every row of A comes out with its columns ascending.
// The column of entry j, i.e. its CSR(A^T) row, is the number of CSR(A^T)
// rows that start at or before j, minus one: a histogram of the row starts
// and one exclusive scan give it for every j.  Values are copied, so CSR(A)
// holds exactly the numbers K2 computed.
#include "pp_common.hpp"

namespace pp {

namespace {

__global__ __launch_bounds__(256) void k_start_hist(const int32_t *__restrict__ rp, int64_t n,
                                                    uint32_t *__restrict__ hist) {
  for (int64_t v = blockIdx.x * int64_t(256) + threadIdx.x; v < n; v += int64_t(gridDim.x) * 256)
    atomicAdd(hist + rp[v], 1u);
}

__global__ __launch_bounds__(256) void k_tr_keys(const int32_t *__restrict__ col, int64_t z,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ rowcnt) {
  for (int64_t j = blockIdx.x * int64_t(256) + threadIdx.x; j < z; j += int64_t(gridDim.x) * 256) {
    const uint32_t u = uint32_t(col[j]);
    keys[j] = (uint64_t(u) << 32) | uint64_t(uint32_t(j));
    atomicAdd(rowcnt + u, 1u);
  }
}

// starts = exclusive scan of the row-start histogram (z + 1 entries), so
// starts[j + 1] is the number of CSR(A^T) rows starting at or before j.
template <typename V>
__global__ __launch_bounds__(256) void k_tr_emit(const uint64_t *__restrict__ keys, int64_t z,
                                                 const uint32_t *__restrict__ starts,
                                                 const V *__restrict__ val_in,
                                                 int32_t *__restrict__ col_out,
                                                 V *__restrict__ val_out) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < z; i += int64_t(gridDim.x) * 256) {
    const uint32_t j = uint32_t(keys[i]);
    col_out[i] = int32_t(starts[j + 1]) - 1;
    val_out[i] = val_in[j];
  }
}

struct Layout {
  uint32_t *starts, *rowcnt, *counts, *scan;
  uint64_t *a, *b;
};

Layout carve(void *ws, int64_t n, int64_t z, size_t *bytes = nullptr) {
  Carve c(ws);
  Layout L{};
  const int64_t zz = z > 0 ? z : 1;
  L.starts = c.take<uint32_t>(size_t(zz + 1));
  L.rowcnt = c.take<uint32_t>(size_t(n + 1));
  L.a = c.take<uint64_t>(size_t(zz));
  L.b = c.take<uint64_t>(size_t(zz));
  const int64_t cnt = int64_t(radix_pingpong_counts(zz));
  L.counts = c.take<uint32_t>(size_t(cnt));
  int64_t sn = zz + 1;
  if (n + 1 > sn) sn = n + 1;
  if (cnt > sn) sn = cnt;
  L.scan = c.take<uint32_t>(size_t(scan_ws_elems(sn)));
  if (bytes) *bytes = c.bytes();
  return L;
}

template <typename V>
pp_status run_transpose(const pp_csr &AT, pp_csr *A, void *ws, hipStream_t s) {
  const int64_t n = AT.n, z = AT.nnz;
  Layout L = carve(ws, n, z);
  pp_status st = fill_i32(reinterpret_cast<int32_t *>(L.rowcnt), n + 1, 0, s);
  if (st != PP_OK) return st;
  if (z > 0) {
    if ((st = fill_i32(reinterpret_cast<int32_t *>(L.starts), z + 1, 0, s)) != PP_OK) return st;
    hipLaunchKernelGGL(k_start_hist, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, AT.row_ptr, n,
                       L.starts);
    hipLaunchKernelGGL(k_tr_keys, dim3(grid_for(z, 256, 16384)), dim3(256), 0, s, AT.col, z, L.a,
                       L.rowcnt);
    PP_LAUNCHED("k_start_hist/k_tr_keys");
    if ((st = exscan_u32(L.starts, L.starts, z + 1, L.scan, nullptr, s)) != PP_OK) return st;
  }
  // Row pointers of A: exclusive scan of the entries per source u.
  st = exscan_u32(L.rowcnt, reinterpret_cast<uint32_t *>(A->row_ptr), n + 1, L.scan, nullptr, s);
  if (st != PP_OK) return st;
  if (z > 0) {
    const int32_t bits = n > 1 ? 32 - __builtin_clz(uint32_t(n - 1)) : 1;
    st = radix_sort_pingpong(L.a, L.b, z, bits, L.counts, L.scan, s);
    if (st != PP_OK) return st;
    hipLaunchKernelGGL(k_tr_emit<V>, dim3(grid_for(z, 256, 16384)), dim3(256), 0, s, L.a, z,
                       L.starts, static_cast<const V *>(AT.val), A->col, static_cast<V *>(A->val));
    PP_LAUNCHED("k_tr_emit");
  }
  A->nnz = z;
  return PP_OK;
}

}  // namespace

size_t transpose_ws_bytes(int64_t n, int64_t z) {
  size_t b = 0;
  carve(nullptr, n, z, &b);
  return b;
}

pp_status launch_transpose(const pp_csr &AT, pp_dtype dt, pp_csr *A, void *ws, size_t ws_bytes,
                           hipStream_t s) {
  if (ws_bytes < transpose_ws_bytes(AT.n, AT.nnz))
    return fail(PP_EWORKSPACE, "pp_transpose: workspace too small");
  return dt == PP_F64 ? run_transpose<double>(AT, A, ws, s) : run_transpose<float>(AT, A, ws, s);
}

}  // namespace pp
