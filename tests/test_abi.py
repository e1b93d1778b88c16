"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every entry point include/pp.h declares, and
reject bad arguments on the host before anything is enqueued.
"""
import ctypes
import glob
import os
import re

import pytest

from paper_1603_01876_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(pp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_pipeline():
    names = declared_functions()
    for want in ["pp_generate", "pp_sort", "pp_filter", "pp_init_r", "pp_pagerank",
                 "pp_workspace_bytes", "pp_strerror", "pp_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    L = native.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in native.SIGNATURES, f"binding lacks {name}"


def test_strerror():
    L = native.lib()
    assert L.pp_strerror(0) == b"success"
    assert L.pp_strerror(3).startswith(b"workspace")
    assert L.pp_strerror(5).startswith(b"internal")


def test_workspace_sizes():
    n, m = 1 << 12, 16 << 12
    assert native.workspace_bytes(native.K0, n, m) == 0
    k1 = native.workspace_bytes(native.K1, n, m)
    assert k1 >= 16 * m                      # two 8-byte key buffers
    k2 = native.workspace_bytes(native.K2, n, m)
    assert k2 >= k1
    k3d = native.workspace_bytes(native.K3, n, m, "f64")
    k3f = native.workspace_bytes(native.K3, n, m, "f32")
    assert k3d > k3f > 0
    with pytest.raises(native.PPError):
        native.workspace_bytes(native.K1, 0, m)
    with pytest.raises(native.PPError):
        native.workspace_bytes(native.K1, n, 1 << 31)
    with pytest.raises(native.PPError):
        native.workspace_bytes(native.K3, n, m, "f32", nrhs=65)


def test_generate_rejects_bad_params():
    L = native.lib()
    p = native._Kron(0, 16, 0.57, 0.19, 0.19, 0.05, 1)
    assert L.pp_generate(ctypes.byref(p), 8, 8, None) == native.PP_EINVAL
    p = native._Kron(10, 16, 0.5, 0.5, 0.5, 0.5, 1)
    assert L.pp_generate(ctypes.byref(p), 8, 8, None) == native.PP_EINVAL
    p = native._Kron(10, 16, 0.57, 0.19, 0.19, 0.05, 1)
    assert L.pp_generate(ctypes.byref(p), None, 8, None) == native.PP_EINVAL
    assert b"null" in L.pp_last_error()


def test_sort_rejects_bad_args():
    L = native.lib()
    assert L.pp_sort(31, 10, 8, 8, 16, 16, 8, 1 << 20, None) == native.PP_ERANGE
    assert L.pp_sort(10, 1 << 31, 8, 8, 16, 16, 8, 1 << 20, None) == native.PP_ERANGE
    assert L.pp_sort(10, -1, 8, 8, 16, 16, 8, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_sort(10, 100, None, 8, 16, 24, 8, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_sort(10, 100, 8, 16, 8, 24, 64, 1 << 20, None) == native.PP_EINVAL  # alias
    assert L.pp_sort(10, 100, 8, 16, 24, 32, None, 0, None) == native.PP_EWORKSPACE
    assert L.pp_sort(10, 100, 8, 16, 24, 32, 64, 100, None) == native.PP_EWORKSPACE
    assert L.pp_sort(10, 0, None, None, None, None, None, 0, None) == native.PP_OK


def test_sort_uv_rejects_bad_args():
    L = native.lib()
    assert L.pp_sort_uv(31, 10, 8, 8, 16, 16, 8, 1 << 20, None) == native.PP_ERANGE
    assert L.pp_sort_uv(10, -1, 8, 16, 24, 32, 8, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_sort_uv(10, 100, 8, 16, 8, 24, 64, 1 << 20, None) == native.PP_EINVAL   # alias
    assert L.pp_sort_uv(10, 100, 8, 16, 24, 24, 64, 1 << 20, None) == native.PP_EINVAL  # outputs
    assert L.pp_sort_uv(10, 100, 8, 16, 24, 32, 64, 100, None) == native.PP_EWORKSPACE
    assert L.pp_sort_uv(10, 0, None, None, None, None, None, 0, None) == native.PP_OK


def test_filter_rejects_bad_args():
    L = native.lib()
    c = native._Csr(1 << 10, 0, 1 << 14, 8, 16, 24)
    assert L.pp_filter(10, 1 << 14, 8, 16, 0, ctypes.byref(c), None, None, None, 0,
                       None) == native.PP_EWORKSPACE
    bad_n = native._Csr(1 << 9, 0, 1 << 14, 8, 16, 24)
    assert L.pp_filter(10, 1 << 14, 8, 16, 0, ctypes.byref(bad_n), None, None, 64, 1 << 30,
                       None) == native.PP_EINVAL
    small = native._Csr(1 << 10, 0, 100, 8, 16, 24)
    assert L.pp_filter(10, 1 << 14, 8, 16, 0, ctypes.byref(small), None, None, 64, 1 << 30,
                       None) == native.PP_EINVAL
    assert L.pp_filter(10, 1 << 14, 8, 16, 7, ctypes.byref(c), None, None, 64, 1 << 30,
                       None) == native.PP_EINVAL
    assert L.pp_filter(0, 1 << 14, 8, 16, 0, ctypes.byref(c), None, None, 64, 1 << 30,
                       None) == native.PP_ERANGE


def test_pagerank_rejects_bad_args():
    L = native.lib()
    c = native._Csr(1000, 10, 100, 8, 16, 24)
    assert L.pp_pagerank(ctypes.byref(c), 0, 0, 20, 0.85, None, 8, None, 64, 1 << 30,
                         None) == native.PP_EINVAL
    assert L.pp_pagerank(ctypes.byref(c), 0, 1, -1, 0.85, None, 8, None, 64, 1 << 30,
                         None) == native.PP_EINVAL
    assert L.pp_pagerank(ctypes.byref(c), 0, 1, 20, 1.5, None, 8, None, 64, 1 << 30,
                         None) == native.PP_EINVAL
    assert L.pp_pagerank(ctypes.byref(c), 0, 1, 20, 0.85, None, 8, None, 64, 10,
                         None) == native.PP_EWORKSPACE
    over = native._Csr(1000, 200, 100, 8, 16, 24)
    assert L.pp_pagerank(ctypes.byref(over), 0, 1, 20, 0.85, None, 8, None, 64, 1 << 30,
                         None) == native.PP_EINVAL
    big = native._Csr(1 << 30, (1 << 31) - 10, 1 << 31, 8, 16, 24)
    assert L.pp_pagerank(ctypes.byref(big), 0, 1, 20, 0.85, None, 8, None, 64, 1 << 30,
                         None) == native.PP_ERANGE


def test_pagerank_converge_rejects_bad_args():
    L = native.lib()
    c = native._Csr(1000, 10, 100, 8, 16, 24)
    done = ctypes.c_int32(-5)

    def call(csr=c, dt=0, iters=100, damp=0.85, tol=1e-9, mode=0, d_out=None, r=8, ws=64,
             wsb=1 << 30, done_p=ctypes.byref(done)):
        return L.pp_pagerank_converge(ctypes.byref(csr), dt, iters, damp, tol, mode, d_out, None,
                                      r, None, None, done_p, ws, wsb, None)

    assert call(iters=-1) == native.PP_EINVAL and done.value == 0
    assert call(damp=-0.1) == native.PP_EINVAL
    assert call(dt=7) == native.PP_EINVAL
    assert call(mode=3) == native.PP_EINVAL
    assert call(mode=1) == native.PP_EINVAL          # uniform needs d_out
    assert call(mode=2) == native.PP_EINVAL          # self needs d_out
    assert call(r=None) == native.PP_EINVAL
    assert call(done_p=None) == native.PP_EINVAL
    assert call(wsb=10) == native.PP_EWORKSPACE
    assert call(csr=native._Csr(1000, 200, 100, 8, 16, 24)) == native.PP_EINVAL
    assert call(csr=native._Csr(1 << 30, (1 << 31) - 10, 1 << 31, 8, 16, 24)) == native.PP_ERANGE


def test_pagerank_graphs_rejects_bad_args():
    # Every call below fails a host-side check before anything is enqueued;
    # the descriptors' device addresses are never dereferenced.
    L = native.lib()
    mx = native.graphs_max_n("f32")
    assert mx > 0 and mx % 64 == 0
    assert 0 < native.graphs_max_n("f64") <= mx      # two n-vectors of 8 B instead of 4 B

    def table(*graphs):
        t = (native._Graph * len(graphs))()
        for i, g in enumerate(graphs):
            t[i] = native._Graph(*g)
        return t

    good = (100, 50, 8, 16, 24, 32, 0, 1)        # n, nnz, row_ptr, col, val, r, sums, seed
    ok = table(good, good)

    def call(ng=2, g=ok, dt=1, iters=20, damp=0.85, use_graph=0, ws=64, wsb=1 << 20,
             stream=None):
        gp = None if g is None else ctypes.addressof(g)
        return L.pp_pagerank_graphs(ng, gp, dt, iters, damp, use_graph, ws, wsb, stream)

    assert call(ng=0) == native.PP_EINVAL
    assert call(g=None) == native.PP_EINVAL
    assert call(dt=5) == native.PP_EINVAL
    assert call(iters=-1) == native.PP_EINVAL
    assert call(damp=1.5) == native.PP_EINVAL
    assert call(use_graph=1) == native.PP_EINVAL      # capture needs a stream
    assert call(ws=None) == native.PP_EWORKSPACE
    assert call(wsb=1) == native.PP_EWORKSPACE
    # The workspace holds the descriptor table: it grows with the batch.
    assert native.workspace_bytes(native.K3_GRAPHS, 1, 1000, "f32") > \
        native.workspace_bytes(native.K3_GRAPHS, 1, 10, "f32")
    # Descriptors: above the on-chip bound, empty or negative, over int32,
    # missing arrays.  The bad descriptor may sit anywhere in the table.
    big = (mx + 1,) + good[1:]
    assert call(g=table(good, big)) == native.PP_ERANGE
    assert call(g=table((native.graphs_max_n("f64") + 1,) + good[1:], good), dt=0) == \
        native.PP_ERANGE
    assert call(g=table((0,) + good[1:], good)) == native.PP_EINVAL
    assert call(g=table(good, (100, -1) + good[2:])) == native.PP_EINVAL
    assert call(g=table(good, (100, (1 << 31) - 50) + good[2:])) == native.PP_ERANGE
    assert call(g=table(good, (100, 50, 0) + good[3:])) == native.PP_EINVAL     # no row_ptr
    assert call(g=table(good, (100, 50, 8, 0) + good[4:])) == native.PP_EINVAL  # no col
    assert call(g=table(good, (100, 50, 8, 16, 0) + good[5:])) == native.PP_EINVAL  # no val
    assert call(g=table(good, (100, 50, 8, 16, 24, 0) + good[6:])) == native.PP_EINVAL  # no r
    # A graph without entries needs no col / val: it passes the descriptor
    # checks and fails only on the (too small) workspace.
    assert call(g=table(good, (100, 0, 8, 0, 0, 32, 0, 1)), wsb=1) == native.PP_EWORKSPACE
    assert call(g=table((mx,) + good[1:], good), wsb=1) == native.PP_EWORKSPACE


def test_pagerank_graphs_noalloc_rejects_bad_args():
    # The allocation-free batch call applies the same host checks (nothing is
    # enqueued, no device address is touched) and bounds the batch by its
    # static scratch.
    L = native.lib()
    cap = native.graphs_noalloc_max()
    assert cap == 1 << 16
    mx = native.graphs_max_n("f32")
    good = (100, 50, 8, 16, 24, 32, 0, 1)

    def table(*graphs):
        t = (native._Graph * len(graphs))()
        for i, g in enumerate(graphs):
            t[i] = native._Graph(*g)
        return t

    ok = table(good, good)

    def call(ng=2, g=ok, dt=1, iters=20, damp=0.85):
        gp = None if g is None else ctypes.addressof(g)
        return L.pp_pagerank_graphs_noalloc(ng, gp, dt, iters, damp, None)

    assert call(ng=cap + 1) == native.PP_ERANGE
    assert call(ng=1 << 25) == native.PP_ERANGE
    assert call(ng=0) == native.PP_EINVAL
    assert call(g=None) == native.PP_EINVAL
    assert call(dt=5) == native.PP_EINVAL
    assert call(iters=-1) == native.PP_EINVAL
    assert call(damp=-0.1) == native.PP_EINVAL
    assert call(g=table(good, (mx + 1,) + good[1:])) == native.PP_ERANGE
    assert call(g=table(good, (100, 50, 8, 16, 24, 0) + good[6:])) == native.PP_EINVAL
    assert b"noalloc" in L.pp_last_error()


def test_edge_file_calls_reject_bad_args(tmp_path):
    L = native.lib()
    assert native.workspace_bytes(native.TSV_FORMAT, 0, 32, "f64", 3) > 0
    assert native.workspace_bytes(native.TSV_PARSE, 0, 1 << 35, "f64") > 1 << 21  # > 2^31 bytes ok
    assert native.workspace_bytes(native.TSV_PARSE, 0, 0, "f64") > 0
    assert L.pp_workspace_bytes(native.TSV_FORMAT, 0, 32, 0, 0) == ctypes.c_size_t(-1).value
    split = (ctypes.c_int64 * 3)()
    sp = ctypes.cast(split, ctypes.c_void_p)
    m = ctypes.c_int64(-1)
    assert L.pp_tsv_format(31, 10, 8, 16, 24, 1000, 1, sp, 64, 1 << 20, None) == native.PP_ERANGE
    assert L.pp_tsv_format(10, 10, 8, 16, 24, 1000, 0, sp, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_tsv_format(10, 10, 8, 16, 24, 1000, 1, None, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_tsv_format(10, 10, None, 16, 24, 1000, 1, sp, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_tsv_format(10, 10, 8, 16, 24, 1000, 1, sp, 64, 4, None) == native.PP_EWORKSPACE
    assert L.pp_tsv_parse(10, 8, 100, 10, 16, 24, ctypes.byref(m), 64, 1 << 20,
                          None) == native.PP_EINVAL          # text not 16-byte aligned
    assert m.value == 0
    assert L.pp_tsv_parse(10, 16, -1, 10, 16, 24, ctypes.byref(m), 64, 1 << 20,
                          None) == native.PP_EINVAL
    assert L.pp_tsv_parse(31, 16, 100, 10, 16, 24, ctypes.byref(m), 64, 1 << 20,
                          None) == native.PP_ERANGE
    assert L.pp_tsv_parse(10, 16, 100, 10, 16, 24, None, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_write_text_files(b"x", 0, 16, sp, 0, None) == native.PP_EINVAL
    assert L.pp_write_text_files(None, 2, 16, sp, 0, None) == native.PP_EINVAL
    nb = ctypes.c_int64(-1)
    missing = str(tmp_path / "absent").encode()
    assert L.pp_read_text_files(missing, 1, 16, 100, ctypes.byref(nb), None) == native.PP_EINVAL
    assert b"absent" in L.pp_last_error()


def test_init_r_rejects_bad_args():
    L = native.lib()
    assert L.pp_init_r(0, 1, 1, 0, 8, 64, 1 << 20, None) == native.PP_ERANGE
    assert L.pp_init_r(100, 0, 1, 0, 8, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_init_r(100, 1, 1, 0, None, 64, 1 << 20, None) == native.PP_EINVAL
    assert L.pp_init_r(100, 1, 1, 0, 8, None, 0, None) == native.PP_EWORKSPACE


def test_product_path_has_no_cpu_fallback():
    # The binding imports nothing from the oracle and has no host compute path.
    for f in glob.glob(os.path.join(ROOT, "paper_1603_01876_amd", "*.py")):
        src = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
    src = open(os.path.join(ROOT, "paper_1603_01876_amd", "native.py")).read()
    assert not re.search(r"^\s*import numpy", src, flags=re.M)


def test_k3_config_roundtrip_and_validation():
    native.set_k3_config(16, 0, 19)
    assert native.get_k3_config() == (16, 0, 19, 1, 0)
    native.set_k3_config(16, 0, 19, 0, 8)
    assert native.get_k3_config() == (16, 0, 19, 0, 8)
    for bad in ((8, 0, -2), (8, 0, 31), (5, 0, 0), (8, 3, 0), (8, 128, 0), (8, 0, 0, 2),
                (8, 0, 0, -1), (8, 0, 0, 1, 3), (8, 0, 0, 1, 64), (8, 0, 0, 1, 1),
                (8, 0, 0, 1, -2)):
        with pytest.raises(native.PPError):
            native.set_k3_config(*bad)
    assert native.get_k3_config() == (16, 0, 19, 0, 8)   # a rejected call changes nothing
    native.lib().pp_set_k3_config(None)
    assert native.get_k3_config() == (8, 0, -1, 1, 0)


def test_transpose_validation():
    L = native.lib()
    n = 8
    at = native._Csr(n, 3, 3, 1, 1, 1)
    a_bad_n = native._Csr(n + 1, 0, 3, 1, 1, 1)
    a_small = native._Csr(n, 0, 2, 1, 1, 1)
    for args in ((None, native.F64, ctypes.byref(native._Csr(n, 0, 3, 1, 1, 1))),
                 (ctypes.byref(at), native.F64, ctypes.byref(a_bad_n)),
                 (ctypes.byref(at), native.F64, ctypes.byref(a_small)),
                 (ctypes.byref(at), 7, ctypes.byref(native._Csr(n, 0, 3, 1, 1, 1)))):
        st = L.pp_transpose(*args, None, 0, None)
        assert st in (native.PP_EINVAL, native.PP_ERANGE), st
    # a large enough matrix but no workspace
    st = L.pp_transpose(ctypes.byref(at), native.F64, ctypes.byref(native._Csr(n, 0, 3, 1, 1, 1)),
                        None, 0, None)
    assert st == native.PP_EWORKSPACE
    assert native.workspace_bytes(native.K2_ROWFORM, n, 3) > 0
