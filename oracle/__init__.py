"""CPU oracle for the PageRank pipeline kernels K0..K3 (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``ppo.c`` -- a plain,
single-threaded FP64 C implementation written from the paper (Dreher et
al., "PageRank Pipeline Benchmark", arXiv 1603.01876, Sec. IV.A-IV.D and the
Appendix) -- with numpy arrays.  It never touches the GPU library.

Parity pins live in ``tests/test_oracle_*.py``; see the header of ppo.c for
which pin covers which function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppo.c")
_LIB = os.path.join(_HERE, "libppo.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)


class _Kron(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_int32), ("edge_factor", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


def build() -> str:
    """Compile ppo.c into oracle/libppo.so (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.ppo_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.ppo_philox4x32_10.restype = None
        L.ppo_kron_thresholds.argtypes = [ctypes.POINTER(_Kron), _u32p]
        L.ppo_permute.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64]
        L.ppo_permute.restype = ctypes.c_int64
        L.ppo_generate_range.argtypes = [ctypes.POINTER(_Kron), ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int, _i64p, _i64p]
        L.ppo_sort.argtypes = [ctypes.c_int32, ctypes.c_int64, _i64p, _i64p, _i64p, _i64p]
        L.ppo_sort_uv.argtypes = [ctypes.c_int32, ctypes.c_int64, _i64p, _i64p, _i64p, _i64p]
        L.ppo_tsv_format.argtypes = [ctypes.c_int64, _i64p, _i64p, ctypes.c_char_p,
                                     ctypes.c_int64, _i64p]
        L.ppo_tsv_parse.argtypes = [ctypes.c_int32, ctypes.c_char_p, ctypes.c_int64,
                                    ctypes.c_int64, _i64p, _i64p, _i64p]
        L.ppo_filter.argtypes = [ctypes.c_int32, ctypes.c_int64, _i64p, _i64p, _i64p, _i64p,
                                 _i64p, _i32p, _f64p, _i64p, _i32p, _f64p, _i64p]
        L.ppo_filter_rows.argtypes = [ctypes.c_int32, ctypes.c_int64, _i64p, _i64p, _i64p,
                                      ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int64,
                                      _i64p, _i64p, _i64p, _i64p]
        L.ppo_init_r.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, _f64p]
        L.ppo_pagerank.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32,
                                   ctypes.c_double, _f64p, _f64p]
        L.ppo_step_rows.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p,
                                    _f64p, ctypes.c_double, ctypes.c_double, _f64p]
        L.ppo_sum_r.argtypes = [ctypes.c_int64, _f64p, _f64p]
        L.ppo_digest.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        L.ppo_pagerank_converge.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                            _f64p, _f64p, _f64p, _i32p]
        _lib = L
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


# --------------------------------------------------------------------------
# K0: generator (Sec. IV.A)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Kron:
    scale: int
    edge_factor: int = 16
    a: float = 0.57
    b: float = 0.19
    c: float = 0.19
    d: float = 0.05
    seed: int = 1603

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def m(self) -> int:
        return self.edge_factor << self.scale

    def _c(self):
        return _Kron(self.scale, self.edge_factor, self.a, self.b, self.c, self.d,
                     self.seed & (2**64 - 1))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ppo_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def kron_thresholds(p: Kron):
    thr = np.zeros(3, dtype=np.uint32)
    _check(lib().ppo_kron_thresholds(ctypes.byref(p._c()), _p(thr, _u32p)), "thresholds")
    return thr


def permute(scale: int, seed: int, x: int) -> int:
    return int(lib().ppo_permute(scale, seed & (2**64 - 1), x))


def generate(p: Kron, e0: int = 0, count: int | None = None, permute: bool = True):
    if count is None:
        count = p.m - e0
    u = np.empty(count, dtype=np.int64)
    v = np.empty(count, dtype=np.int64)
    _check(lib().ppo_generate_range(ctypes.byref(p._c()), e0, count, int(permute),
                                    _p(u, _i64p), _p(v, _i64p)), "generate")
    return u, v


# --------------------------------------------------------------------------
# K1: sort (Sec. IV.B)
# --------------------------------------------------------------------------
def sort(scale: int, u, v):
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    uo = np.empty_like(u)
    vo = np.empty_like(v)
    _check(lib().ppo_sort(scale, u.size, _p(u, _i64p), _p(v, _i64p),
                          _p(uo, _i64p), _p(vo, _i64p)), "sort")
    return uo, vo


def sort_uv(scale: int, u, v):
    """K1 variant: edges ordered by (u, v)."""
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    uo = np.empty_like(u)
    vo = np.empty_like(v)
    _check(lib().ppo_sort_uv(scale, u.size, _p(u, _i64p), _p(v, _i64p),
                             _p(uo, _i64p), _p(vo, _i64p)), "sort_uv")
    return uo, vo


def tsv_format(u, v) -> bytes:
    """Edges as text lines "u<TAB>v<LF>"."""
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    cap = 22 * u.size + 1
    buf = ctypes.create_string_buffer(cap)
    nb = np.zeros(1, np.int64)
    _check(lib().ppo_tsv_format(u.size, _p(u, _i64p), _p(v, _i64p), buf, cap, _p(nb, _i64p)),
           "tsv_format")
    return buf.raw[:int(nb[0])]


def tsv_parse(scale: int, text: bytes, cap: int | None = None):
    """Edges back from text; raises on malformed text or labels >= 2^scale."""
    cap = len(text) // 4 + 1 if cap is None else cap
    u = np.empty(max(cap, 1), np.int64)
    v = np.empty(max(cap, 1), np.int64)
    m = np.zeros(1, np.int64)
    _check(lib().ppo_tsv_parse(scale, text, len(text), cap, _p(u, _i64p), _p(v, _i64p),
                               _p(m, _i64p)), "tsv_parse")
    k = int(m[0])
    return u[:k].copy(), v[:k].copy()


# --------------------------------------------------------------------------
# K2: filter (Sec. IV.C)
# --------------------------------------------------------------------------
@dataclass
class Filtered:
    n: int
    nnz: int
    d_in: np.ndarray
    d_out: np.ndarray
    A_rp: np.ndarray
    A_col: np.ndarray
    A_val: np.ndarray
    AT_rp: np.ndarray
    AT_col: np.ndarray
    AT_val: np.ndarray


def filter(scale: int, u, v) -> Filtered:
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    n = 1 << scale
    m = u.size
    d_in = np.empty(n, np.int64)
    d_out = np.empty(n, np.int64)
    A_rp = np.empty(n + 1, np.int64)
    AT_rp = np.empty(n + 1, np.int64)
    cap = max(m, 1)
    A_col = np.empty(cap, np.int32)
    A_val = np.empty(cap, np.float64)
    AT_col = np.empty(cap, np.int32)
    AT_val = np.empty(cap, np.float64)
    nnz = np.zeros(1, np.int64)
    _check(lib().ppo_filter(scale, m, _p(u, _i64p), _p(v, _i64p), _p(d_in, _i64p),
                            _p(d_out, _i64p), _p(A_rp, _i64p), _p(A_col, _i32p),
                            _p(A_val, _f64p), _p(AT_rp, _i64p), _p(AT_col, _i32p),
                            _p(AT_val, _f64p), _p(nnz, _i64p)), "filter")
    z = int(nnz[0])
    return Filtered(n, z, d_in, d_out, A_rp, A_col[:z].copy(), A_val[:z].copy(),
                    AT_rp, AT_col[:z].copy(), AT_val[:z].copy())


def filter_rows(scale: int, u, v, rows, want_nnz: bool = False):
    """Sampled K2 at any scale: d_in, d_out, mx over all edges plus the
    listed rows of A^T.  Returns (rp, col, val, d_in, d_out, mx, nnz|None)."""
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = 1 << scale
    m = u.size
    # A row of A^T has at most d_in[v] entries; bound the buffer by m.
    cap = int(min(m, max(1, 64 * rows.size + 4096)))
    while True:
        rp = np.empty(rows.size + 1, np.int64)
        col = np.empty(cap, np.int32)
        val = np.empty(cap, np.float64)
        d_in = np.empty(n, np.int64)
        d_out = np.empty(n, np.int64)
        mx = np.zeros(1, np.int64)
        nnz = np.zeros(1, np.int64)
        st = lib().ppo_filter_rows(scale, m, _p(u, _i64p), _p(v, _i64p), _p(rows, _i64p),
                                   rows.size, _p(rp, _i64p), _p(col, _i32p), _p(val, _f64p),
                                   cap, _p(d_in, _i64p), _p(d_out, _i64p), _p(mx, _i64p),
                                   _p(nnz, _i64p) if want_nnz else None)
        if st == -1 and cap < m:
            cap = m
            continue
        _check(st, "filter_rows")
        k = int(rp[-1])
        return (rp, col[:k].copy(), val[:k].copy(), d_in, d_out, int(mx[0]),
                int(nnz[0]) if want_nnz else None)


# --------------------------------------------------------------------------
# K3: PageRank (Sec. IV.D, Appendix)
# --------------------------------------------------------------------------
def init_r(n: int, seed: int, rhs: int = 0):
    r = np.empty(n, np.float64)
    _check(lib().ppo_init_r(n, seed & (2**64 - 1), rhs, _p(r, _f64p)), "init_r")
    return r


def pagerank(n: int, A_rp, A_col, A_val, r0, iters: int = 20, c: float = 0.85):
    """Returns (r_iters, sums) with sums[k] = sum(r_k), k = 0..iters."""
    A_rp = np.ascontiguousarray(A_rp, dtype=np.int64)
    A_col = np.ascontiguousarray(A_col, dtype=np.int32)
    A_val = np.ascontiguousarray(A_val, dtype=np.float64)
    r = np.array(r0, dtype=np.float64, copy=True)
    sums = np.empty(iters + 1, np.float64)
    if A_col.size == 0:
        A_col = np.zeros(1, np.int32)
        A_val = np.zeros(1, np.float64)
    _check(lib().ppo_pagerank(n, _p(A_rp, _i64p), _p(A_col, _i32p), _p(A_val, _f64p),
                              iters, c, _p(r, _f64p), _p(sums, _f64p)), "pagerank")
    return r, sums


DANGLING = {"none": 0, "uniform": 1, "self": 2}


def pagerank_converge(n: int, A_rp, A_col, A_val, r0, max_iters: int, tol: float,
                      mode: str = "none", c: float = 0.85):
    """K3 until the normalised L1 difference of successive iterates is
    <= tol (or max_iters), with a dangling-vertex mode ("none", "uniform",
    "self").  Returns (r, sums[0..k], deltas[0..k-1], k)."""
    A_rp = np.ascontiguousarray(A_rp, dtype=np.int64)
    A_col = np.ascontiguousarray(A_col, dtype=np.int32)
    A_val = np.ascontiguousarray(A_val, dtype=np.float64)
    r = np.array(r0, dtype=np.float64, copy=True)
    sums = np.empty(max_iters + 1, np.float64)
    deltas = np.empty(max(max_iters, 1), np.float64)
    done = np.zeros(1, np.int32)
    if A_col.size == 0:
        A_col = np.zeros(1, np.int32)
        A_val = np.zeros(1, np.float64)
    _check(lib().ppo_pagerank_converge(n, _p(A_rp, _i64p), _p(A_col, _i32p), _p(A_val, _f64p),
                                       max_iters, c, tol, DANGLING[mode], _p(r, _f64p),
                                       _p(sums, _f64p), _p(deltas, _f64p), _p(done, _i32p)),
           "pagerank_converge")
    k = int(done[0])
    return r, sums[:k + 1], deltas[:k], k


def step_rows(n: int, rp, col, val, r, s: float, c: float = 0.85):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    nrows = rp.size - 1
    y = np.empty(max(nrows, 0), np.float64)
    if col.size == 0:
        col = np.zeros(1, np.int32)
        val = np.zeros(1, np.float64)
    _check(lib().ppo_step_rows(n, nrows, _p(rp, _i64p), _p(col, _i32p), _p(val, _f64p),
                               _p(r, _f64p), s, c, _p(y, _f64p)), "step_rows")
    return y


def transpose_csr(n: int, rp, col, val):
    """CSR(A) -> CSR(A^T) by a stable counting sort on the column (numpy;
    used by tests that feed K3 hand-built matrices)."""
    rp = np.asarray(rp, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    order = np.argsort(col, kind="stable")
    trp = np.zeros(n + 1, np.int64)
    np.add.at(trp, col + 1, 1)
    trp = np.cumsum(trp)
    return trp, rows[order].astype(np.int32), np.asarray(val, np.float64)[order]


# --------------------------------------------------------------------------
# Tooling for full-size parity: sums, digests, row blocks
# --------------------------------------------------------------------------
def sum_r(r) -> float:
    """sum(r) exactly as K3 forms it (compensated, ascending index)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(1, np.float64)
    _check(lib().ppo_sum_r(r.size, _p(r, _f64p), _p(out, _f64p)), "sum_r")
    return float(out[0])


def digest(x, index0: int = 0) -> int:
    """Order-independent 64-bit digest of an array's element bit patterns
    (4- or 8-byte elements, zero-extended); see ppo_digest."""
    x = np.ascontiguousarray(x)
    if x.dtype.itemsize not in (4, 8):
        raise ValueError(f"digest of {x.dtype} elements")
    out = ctypes.c_uint64(0)
    ptr = ctypes.c_void_p(x.ctypes.data if x.size else 0)
    _check(lib().ppo_digest(ptr, x.size, x.dtype.itemsize, index0, ctypes.byref(out)), "digest")
    return int(out.value)


def digest_add(*parts: int) -> int:
    """Digests of consecutive pieces add up (mod 2^64) to the whole's."""
    return sum(parts) % (1 << 64)


def _threads(fn, jobs, threads):
    # The oracle's C functions run with the GIL released (ctypes), so
    # independent calls overlap on several cores; each call is itself the
    # plain single-threaded code.
    from concurrent.futures import ThreadPoolExecutor
    if threads <= 1:
        return [fn(j) for j in jobs]
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, jobs))


def generate_parallel(p: Kron, threads: int = 1, chunk: int = 1 << 22):
    """K0's whole edge list, computed in independent edge ranges (each edge is
    a pure function of its index, Sec. IV.A), several ranges at a time."""
    u = np.empty(p.m, dtype=np.int64)
    v = np.empty(p.m, dtype=np.int64)
    starts = list(range(0, p.m, chunk))

    def one(e0):
        k = min(chunk, p.m - e0)
        _check(lib().ppo_generate_range(ctypes.byref(p._c()), e0, k, 1, _p(u[e0:], _i64p),
                                        _p(v[e0:], _i64p)), "generate")

    _threads(one, starts, threads)
    return u, v


def filter_blocks(scale: int, u, v, nblocks: int = 8, threads: int = 1):
    """K2's CSR(A^T) at any scale, built from contiguous blocks of its rows
    with ppo_filter_rows (each block rescans all edges, so peak memory is the
    edges plus one block).  Returns (AT_rp int64, AT_col, AT_val, d_in,
    d_out, mx, nnz) -- the same arrays ppo_filter writes."""
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    n = 1 << scale
    m = u.size
    d_in = np.empty(n, np.int64)
    d_out = np.empty(n, np.int64)
    mx = np.zeros(1, np.int64)
    one = np.zeros(2, np.int64)
    _check(lib().ppo_filter_rows(scale, m, _p(u, _i64p), _p(v, _i64p), None, 0, _p(one, _i64p),
                                 None, None, 0, _p(d_in, _i64p), _p(d_out, _i64p),
                                 _p(mx, _i64p), None), "filter_rows")
    bounds = [n * b // nblocks for b in range(nblocks + 1)]
    caps = [int(d_in[bounds[b]:bounds[b + 1]].sum()) for b in range(nblocks)]
    offs = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
    col = np.empty(max(int(offs[-1]), 1), np.int32)
    val = np.empty(max(int(offs[-1]), 1), np.float64)
    rps = [None] * nblocks

    def block(b):
        j0, j1 = bounds[b], bounds[b + 1]
        rows = np.arange(j0, j1, dtype=np.int64)
        rp = np.empty(j1 - j0 + 1, np.int64)
        o = int(offs[b])
        cap = max(caps[b], 1)
        _check(lib().ppo_filter_rows(scale, m, _p(u, _i64p), _p(v, _i64p), _p(rows, _i64p),
                                     rows.size, _p(rp, _i64p), _p(col[o:], _i32p),
                                     _p(val[o:], _f64p), cap, None, None, None, None),
               "filter_rows")
        rps[b] = rp

    _threads(block, range(nblocks), threads)
    # Close the gaps between blocks in place (block b's entries sit at
    # offs[b] >= their final offset; numpy copies overlapping slices safely).
    AT_rp = np.empty(n + 1, np.int64)
    at = 0
    for b in range(nblocks):
        k = int(rps[b][-1])
        o = int(offs[b])
        if o != at:
            col[at:at + k] = col[o:o + k]
            val[at:at + k] = val[o:o + k]
        AT_rp[bounds[b]:bounds[b + 1]] = rps[b][:-1] + at
        at += k
    AT_rp[n] = at
    return AT_rp, col[:at], val[:at], d_in, d_out, int(mx[0]), at


def pagerank_rows(n: int, AT_rp, AT_col, AT_val, r0, iters: int = 20, c: float = 0.85,
                  threads: int = 1, nblocks: int | None = None):
    """K3 on CSR(A^T): per iteration s = sum_r(r), then ppo_step_rows over
    contiguous row blocks (the blocks only split the rows; every row is
    the oracle's own sum).  Equals pagerank() on CSR(A) bit for bit.
    Returns (r_iters, sums)."""
    AT_rp = np.ascontiguousarray(AT_rp, dtype=np.int64)
    AT_col = np.ascontiguousarray(AT_col, dtype=np.int32)
    AT_val = np.ascontiguousarray(AT_val, dtype=np.float64)
    if AT_col.size == 0:
        AT_col = np.zeros(1, np.int32)
        AT_val = np.zeros(1, np.float64)
    r = np.array(r0, dtype=np.float64, copy=True)
    y = np.empty_like(r)
    sums = np.empty(iters + 1, np.float64)
    nb = nblocks or max(1, 4 * threads)
    bounds = [n * b // nb for b in range(nb + 1)]
    for it in range(iters + 1):
        sums[it] = sum_r(r)
        if it == iters:
            break
        s = sums[it]

        def block(b, r=r, y=y, s=s):
            j0, j1 = bounds[b], bounds[b + 1]
            _check(lib().ppo_step_rows(n, j1 - j0, _p(AT_rp[j0:], _i64p), _p(AT_col, _i32p),
                                       _p(AT_val, _f64p), _p(r, _f64p), s, c,
                                       _p(y[j0:], _f64p)), "step_rows")

        _threads(block, range(nb), threads)
        r, y = y, r
    return r, sums

