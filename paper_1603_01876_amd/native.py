"""Python binding of libpp.so (include/pp.h): argument marshalling only.

Every array is a torch tensor on the GPU; torch provides device memory and
the current stream, nothing else.  Each function calls exactly one C entry
point of the same name; all computation happens in the library's HIP
kernels.  There is no fallback: if libpp.so is missing or fails to load,
every call raises PPError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpp.so")

PP_OK, PP_EINVAL, PP_ERANGE, PP_EWORKSPACE, PP_EHIP, PP_EINTERNAL = range(6)
F64, F32 = 0, 1
K0, K1, K2, K3, K3_GRAPHS, K2_ROWFORM, TSV_FORMAT, TSV_PARSE = range(8)

_TORCH = {F64: torch.float64, F32: torch.float32}
_NAMES = {"f64": F64, "f32": F32, F64: F64, F32: F32,
          torch.float64: F64, torch.float32: F32}


class PPError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class _Kron(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_int32), ("edge_factor", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("cap", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class _K3Config(ctypes.Structure):
    _fields_ = [("items_per_thread", ctypes.c_int32), ("rhs_lanes", ctypes.c_int32),
                ("slab_log2", ctypes.c_int32), ("scaled_form", ctypes.c_int32),
                ("rhs_tile", ctypes.c_int32)]


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("sums", ctypes.c_void_p), ("seed", ctypes.c_uint64)]


_lib = None

# (name, restype, argtypes) of every entry point in include/pp.h.
_VP, _I32, _I64, _U64, _SZ, _D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double)
SIGNATURES = {
    "pp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pp_last_error": (ctypes.c_char_p, []),
    "pp_workspace_bytes": (_SZ, [ctypes.c_int, _I64, _I64, ctypes.c_int, _I32]),
    "pp_generate": (ctypes.c_int, [ctypes.POINTER(_Kron), _VP, _VP, _VP]),
    "pp_sort": (ctypes.c_int, [_I32, _I64, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "pp_sort_uv": (ctypes.c_int, [_I32, _I64, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "pp_tsv_format": (ctypes.c_int, [_I32, _I64, _VP, _VP, _VP, _I64, _I32, _VP, _VP, _SZ,
                                     _VP]),
    "pp_tsv_parse": (ctypes.c_int, [_I32, _VP, _I64, _I64, _VP, _VP, ctypes.POINTER(_I64), _VP,
                                    _SZ, _VP]),
    "pp_write_text_files": (ctypes.c_int, [ctypes.c_char_p, _I32, _VP, _VP, _I32, _VP]),
    "pp_read_text_files": (ctypes.c_int, [ctypes.c_char_p, _I32, _VP, _I64,
                                          ctypes.POINTER(_I64), _VP]),
    "pp_filter": (ctypes.c_int, [_I32, _I64, _VP, _VP, ctypes.c_int, ctypes.POINTER(_Csr),
                                 _VP, _VP, _VP, _SZ, _VP]),
    "pp_transpose": (ctypes.c_int, [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.POINTER(_Csr),
                                    _VP, _SZ, _VP]),
    "pp_init_r": (ctypes.c_int, [_I64, _I32, _U64, ctypes.c_int, _VP, _VP, _SZ, _VP]),
    "pp_pagerank": (ctypes.c_int, [ctypes.POINTER(_Csr), ctypes.c_int, _I32, _I32, _D, _VP,
                                   _VP, _VP, _VP, _SZ, _VP]),
    "pp_pagerank_graphs": (ctypes.c_int, [_I32, _VP, ctypes.c_int, _I32, _D, _I32, _VP, _SZ,
                                          _VP]),
    "pp_pagerank_converge": (ctypes.c_int, [ctypes.POINTER(_Csr), ctypes.c_int, _I32, _D, _D,
                                            ctypes.c_int, _VP, _VP, _VP, _VP, _VP,
                                            ctypes.POINTER(_I32), _VP, _SZ, _VP]),
    "pp_graphs_max_n": (_I64, [ctypes.c_int]),
    "pp_pagerank_graphs_noalloc": (ctypes.c_int, [_I32, _VP, ctypes.c_int, _I32, _D, _VP]),
    "pp_graphs_noalloc_max": (_I32, []),
    "pp_set_k3_config": (ctypes.c_int, [ctypes.c_void_p]),
    "pp_get_k3_config": (ctypes.c_int, [ctypes.c_void_p]),
    "pp_k3_last_layout": (_I32, []),
    "pp_set_kernel_timing": (ctypes.c_int, [ctypes.c_int]),
    "pp_kernel_times": (_I32, [ctypes.POINTER(ctypes.c_float), _I32]),
}


def lib():
    """Loads libpp.so once.  Raises PPError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PPError(-1, "libpp", f"{LIB_PATH} not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != PP_OK:
        L = lib()
        raise PPError(st, where, f"{L.pp_strerror(st).decode()}: {L.pp_last_error().decode()}")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def dtype_code(dtype) -> int:
    return _NAMES[dtype]


def workspace_bytes(kernel: int, n: int, m: int, dtype="f64", nrhs: int = 1) -> int:
    b = lib().pp_workspace_bytes(kernel, n, m, dtype_code(dtype), nrhs)
    if b == ctypes.c_size_t(-1).value:
        raise PPError(PP_ERANGE, "pp_workspace_bytes", f"kernel {kernel}, n {n}, m {m}")
    return int(b)


def _ws(nbytes: int, ws, device):
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise PPError(PP_EWORKSPACE, "workspace", f"needs {nbytes} bytes")
        return ws
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------- K0
def generate(spec, u=None, v=None, device="cuda"):
    """K0: returns (u, v) int64 tensors of M = k*2^S edges."""
    m = spec.edge_factor << spec.scale
    if u is None:
        u = torch.empty(m, dtype=torch.int64, device=device)
    if v is None:
        v = torch.empty(m, dtype=torch.int64, device=device)
    p = _Kron(spec.scale, spec.edge_factor, spec.a, spec.b, spec.c, spec.d,
              spec.seed & (2**64 - 1))
    _check(lib().pp_generate(ctypes.byref(p), _ptr(u), _ptr(v), _stream()), "pp_generate")
    return u, v


# ---------------------------------------------------------------------- K1
def sort(scale: int, u, v, u_out=None, v_out=None, ws=None):
    """K1: stable sort by u.  Returns (u_out, v_out)."""
    m = u.numel()
    if u_out is None:
        u_out = torch.empty_like(u)
    if v_out is None:
        v_out = torch.empty_like(v)
    nbytes = workspace_bytes(K1, 1 << scale, m)
    ws = _ws(nbytes, ws, u.device)
    _check(lib().pp_sort(scale, m, _ptr(u), _ptr(v), _ptr(u_out), _ptr(v_out), _ptr(ws),
                         ws.numel(), _stream()), "pp_sort")
    return u_out, v_out


def sort_uv(scale: int, u, v, u_out=None, v_out=None, ws=None):
    """K1 variant: edges ordered by (u, v).  Returns (u_out, v_out)."""
    m = u.numel()
    if u_out is None:
        u_out = torch.empty_like(u)
    if v_out is None:
        v_out = torch.empty_like(v)
    ws = _ws(workspace_bytes(K1, 1 << scale, m), ws, u.device)
    _check(lib().pp_sort_uv(scale, m, _ptr(u), _ptr(v), _ptr(u_out), _ptr(v_out), _ptr(ws),
                            ws.numel(), _stream()), "pp_sort_uv")
    return u_out, v_out


# ------------------------------------------------------------- edge files
def tsv_format(scale: int, u, v, nsplit: int = 1, text=None, ws=None):
    """Edges as text lines "u<TAB>v<LF>" on the GPU.  Returns (text, split):
    a uint8 device tensor (capacity 22 bytes per edge unless given) and the
    nsplit + 1 byte offsets of nsplit parts of nearly equal edge counts
    (split[-1] = bytes of text)."""
    m = u.numel()
    if text is None:
        text = torch.empty(max(22 * m, 16), dtype=torch.uint8, device=u.device)
    split = (ctypes.c_int64 * (nsplit + 1))()
    ws = _ws(workspace_bytes(TSV_FORMAT, 0, m, F64, nsplit), ws, u.device)
    _check(lib().pp_tsv_format(scale, m, _ptr(u), _ptr(v), _ptr(text), text.numel(), nsplit,
                               ctypes.cast(split, ctypes.c_void_p), _ptr(ws), ws.numel(),
                               _stream()), "pp_tsv_format")
    return text, [int(x) for x in split]


def tsv_parse(scale: int, text, nbytes: int, cap: int | None = None, u=None, v=None, ws=None):
    """Edges back from text (a uint8 device tensor, first nbytes bytes).
    Returns (u, v) cut to the edges read."""
    dev = text.device
    if cap is None:
        cap = u.numel() if u is not None else nbytes // 4 + 1
    if u is None:
        u = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    if v is None:
        v = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    m = ctypes.c_int64(0)
    ws = _ws(workspace_bytes(TSV_PARSE, 0, nbytes, F64), ws, dev)
    _check(lib().pp_tsv_parse(scale, _ptr(text), nbytes, cap, _ptr(u), _ptr(v), ctypes.byref(m),
                              _ptr(ws), ws.numel(), _stream()), "pp_tsv_parse")
    return u[:m.value], v[:m.value]


def write_text_files(prefix: str, text, split, sync: bool = True) -> None:
    """File k = text[split[k]:split[k+1]] for k < len(split) - 1."""
    arr = (ctypes.c_int64 * len(split))(*split)
    _check(lib().pp_write_text_files(prefix.encode(), len(split) - 1, _ptr(text),
                                     ctypes.cast(arr, ctypes.c_void_p), int(sync), _stream()),
           "pp_write_text_files")


def read_text_files(prefix: str, nfiles: int, text) -> int:
    """Reads the files back to back into text (uint8 device tensor); returns
    the number of bytes."""
    nb = ctypes.c_int64(0)
    _check(lib().pp_read_text_files(prefix.encode(), nfiles, _ptr(text), text.numel(),
                                    ctypes.byref(nb), _stream()), "pp_read_text_files")
    return int(nb.value)


# ---------------------------------------------------------------------- K2
@dataclass
class CSR:
    """CSR(A^T) on the device: row v lists the sources u of column v of A."""
    n: int
    nnz: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def dtype(self) -> int:
        return dtype_code(self.val.dtype)

    def _c(self) -> _Csr:
        return _Csr(self.n, self.nnz, self.col.numel(), self.row_ptr.data_ptr(),
                    self.col.data_ptr(), self.val.data_ptr())

    @staticmethod
    def from_arrays(n, row_ptr, col, val, dtype="f64", device="cuda") -> "CSR":
        """Uploads a host CSR (numpy or torch) to the device."""
        rp = torch.as_tensor(row_ptr).to(torch.int32)
        cl = torch.as_tensor(col).to(torch.int32)
        vl = torch.as_tensor(val).to(_TORCH[dtype_code(dtype)])
        nnz = int(rp[-1])
        cap = max(nnz, 1)
        col_d = torch.zeros(cap, dtype=torch.int32, device=device)
        val_d = torch.zeros(cap, dtype=vl.dtype, device=device)
        col_d[:nnz] = cl[:nnz].to(device)
        val_d[:nnz] = vl[:nnz].to(device)
        return CSR(n, nnz, rp.to(device), col_d, val_d)


def filter(scale: int, u, v, dtype="f64", AT: CSR | None = None, d_in=None, d_out=None,
           ws=None, degrees: bool = True):
    """K2: returns (CSR(A^T), d_in, d_out); degrees are None if not asked for."""
    n = 1 << scale
    m = u.numel()
    dt = dtype_code(dtype)
    dev = u.device
    if AT is None:
        cap = max(m, 1)
        AT = CSR(n, 0, torch.empty(n + 1, dtype=torch.int32, device=dev),
                 torch.empty(cap, dtype=torch.int32, device=dev),
                 torch.empty(cap, dtype=_TORCH[dt], device=dev))
    if degrees:
        if d_in is None:
            d_in = torch.empty(n, dtype=torch.int32, device=dev)
        if d_out is None:
            d_out = torch.empty(n, dtype=torch.int32, device=dev)
    ws = _ws(workspace_bytes(K2, n, m), ws, dev)
    c = AT._c()
    _check(lib().pp_filter(scale, m, _ptr(u), _ptr(v), dt, ctypes.byref(c), _ptr(d_in),
                           _ptr(d_out), _ptr(ws), ws.numel(), _stream()), "pp_filter")
    AT.nnz = int(c.nnz)
    return AT, d_in, d_out


def transpose(AT: CSR, A: CSR | None = None, ws=None) -> CSR:
    """Row form CSR(A) of K2's matrix from its CSR(A^T) (see pp_transpose)."""
    dt = AT.dtype
    dev = AT.row_ptr.device
    if A is None:
        cap = max(AT.nnz, 1)
        A = CSR(AT.n, 0, torch.empty(AT.n + 1, dtype=torch.int32, device=dev),
                torch.empty(cap, dtype=torch.int32, device=dev),
                torch.empty(cap, dtype=_TORCH[dt], device=dev))
    ws = _ws(workspace_bytes(K2_ROWFORM, AT.n, AT.nnz, dt), ws, dev)
    ca, cat = A._c(), AT._c()
    _check(lib().pp_transpose(ctypes.byref(cat), dt, ctypes.byref(ca), _ptr(ws), ws.numel(),
                              _stream()), "pp_transpose")
    A.nnz = int(ca.nnz)
    return A


# ---------------------------------------------------------------------- K3
def init_r(n: int, seed: int, dtype="f64", nrhs: int = 1, out=None, ws=None, device="cuda"):
    """K3 initial vector(s): n x nrhs row-major (shape (n,) when nrhs == 1)."""
    dt = dtype_code(dtype)
    if out is None:
        shape = (n,) if nrhs == 1 else (n, nrhs)
        out = torch.empty(shape, dtype=_TORCH[dt], device=device)
    ws = _ws(workspace_bytes(K3, n, 0, dt, nrhs), ws, out.device)
    _check(lib().pp_init_r(n, nrhs, seed & (2**64 - 1), dt, _ptr(out), _ptr(ws), ws.numel(),
                           _stream()), "pp_init_r")
    return out


def pagerank(AT: CSR, r, iters: int = 20, c: float = 0.85, sums=True, ws=None, weights=None):
    """K3: iterates r in place; returns sum(r) per iteration ((iters+1) x nrhs
    FP64 tensor) or None when sums is False.  `weights` (int32 per vertex,
    e.g. d_out from filter()) turns on the locality relabelling."""
    dt = dtype_code(r.dtype)
    if dt != AT.dtype:
        raise PPError(PP_EINVAL, "pagerank", "r and matrix values differ in dtype")
    nrhs = 1 if r.dim() == 1 else r.shape[1]
    if sums is True:
        sums = torch.empty((iters + 1, nrhs) if nrhs > 1 else (iters + 1,),
                           dtype=torch.float64, device=r.device)
    elif sums is False:
        sums = None
    ws = _ws(workspace_bytes(K3, AT.n, AT.nnz, dt, nrhs), ws, r.device)
    cs = AT._c()
    _check(lib().pp_pagerank(ctypes.byref(cs), dt, nrhs, iters, c, _ptr(weights), _ptr(r),
                             _ptr(sums), _ptr(ws), ws.numel(), _stream()), "pp_pagerank")
    return sums


DANGLING = {"none": 0, "uniform": 1, "self": 2}


def pagerank_converge(AT: CSR, r, max_iters: int, tol: float, mode: str = "none", d_out=None,
                      c: float = 0.85, weights=None, ws=None):
    """K3 until the normalised L1 difference between iterates is <= tol (or
    max_iters), with a dangling-vertex mode ("none", "uniform", "self"; the
    last two need d_out).  Iterates r in place; returns (sums, deltas,
    iterations): FP64 tensors of sum(r_k), k = 0..iterations, and of the
    differences, k = 0..iterations-1."""
    dt = dtype_code(r.dtype)
    if dt != AT.dtype:
        raise PPError(PP_EINVAL, "pagerank_converge", "r and matrix values differ in dtype")
    if mode not in DANGLING:
        raise PPError(PP_EINVAL, "pagerank_converge", f"dangling mode {mode!r}")
    sums = torch.empty(max_iters + 1, dtype=torch.float64, device=r.device)
    deltas = torch.empty(max(max_iters, 1), dtype=torch.float64, device=r.device)
    ws = _ws(workspace_bytes(K3, AT.n, AT.nnz, dt, 1), ws, r.device)
    done = ctypes.c_int32(0)
    cs = AT._c()
    _check(lib().pp_pagerank_converge(ctypes.byref(cs), dt, max_iters, c, tol, DANGLING[mode],
                                      _ptr(d_out), _ptr(weights), _ptr(r), _ptr(sums),
                                      _ptr(deltas), ctypes.byref(done), _ptr(ws), ws.numel(),
                                      _stream()), "pp_pagerank_converge")
    k = int(done.value)
    return sums[:k + 1], deltas[:k], k


def graphs_max_n(dtype="f32") -> int:
    """Largest vertex count pagerank_graphs() accepts for this dtype."""
    return int(lib().pp_graphs_max_n(dtype_code(dtype)))


class GraphBatch:
    """A batch for pagerank_graphs(): (CSR, r, sums_or_None, seed) per graph,
    largest graphs first, and their descriptor table (host memory; the
    library copies it into the batch's workspace on every call)."""

    def __init__(self, items, dtype="f32"):
        self.dtype = dtype_code(dtype)
        self.items = sorted(items, key=lambda it: -(it[0].n + it[0].nnz))
        self.table = (_Graph * len(self.items))()
        for i, (AT, r, sums, seed) in enumerate(self.items):
            if AT.dtype != self.dtype or dtype_code(r.dtype) != self.dtype:
                raise PPError(PP_EINVAL, "GraphBatch", "dtype mismatch")
            self.table[i] = _Graph(AT.n, AT.nnz, AT.row_ptr.data_ptr(), AT.col.data_ptr(),
                                   AT.val.data_ptr(), r.data_ptr(), _ptr(sums) or 0,
                                   seed & (2**64 - 1))
        dev = self.items[0][1].device
        self.max_n = max(AT.n for AT, *_ in self.items)
        self.ws = torch.empty(workspace_bytes(K3_GRAPHS, 1, len(self.items), self.dtype),
                              dtype=torch.uint8, device=dev)

    def __len__(self):
        return len(self.items)


def pagerank_graphs(batch: GraphBatch, iters: int = 20, c: float = 0.85, use_graph=True):
    """K3 for every graph of the batch in one persistent launch (r and sums
    filled in place).  With use_graph the launch is recorded once into a
    hipGraph and replayed on later calls; it needs a non-default stream."""
    _check(lib().pp_pagerank_graphs(len(batch), ctypes.addressof(batch.table), batch.dtype,
                                    iters, c, int(bool(use_graph)), batch.ws.data_ptr(),
                                    batch.ws.numel(), _stream()), "pp_pagerank_graphs")


def pagerank_graphs_noalloc(batch: GraphBatch, iters: int = 20, c: float = 0.85):
    """pagerank_graphs() through pp_pagerank_graphs_noalloc: a direct launch
    whose queue and descriptor table live in the library's static device
    array, so the call allocates nothing (batch.ws is not used)."""
    _check(lib().pp_pagerank_graphs_noalloc(len(batch), ctypes.addressof(batch.table),
                                            batch.dtype, iters, c, _stream()),
           "pp_pagerank_graphs_noalloc")


def graphs_noalloc_max() -> int:
    """Largest batch pagerank_graphs_noalloc() accepts."""
    return int(lib().pp_graphs_noalloc_max())


def set_k3_config(items_per_thread: int = 8, rhs_lanes: int = 0, slab_log2: int = -1,
                  scaled_form: int = 1, rhs_tile: int = 0) -> None:
    """Launch configuration of pagerank() (see pp_set_k3_config)."""
    cfg = _K3Config(items_per_thread, rhs_lanes, slab_log2, scaled_form, rhs_tile)
    _check(lib().pp_set_k3_config(ctypes.addressof(cfg)), "pp_set_k3_config")


def get_k3_config() -> tuple[int, int, int, int, int]:
    """(items_per_thread, rhs_lanes, slab_log2, scaled_form, rhs_tile)."""
    cfg = _K3Config()
    _check(lib().pp_get_k3_config(ctypes.addressof(cfg)), "pp_get_k3_config")
    return (int(cfg.items_per_thread), int(cfg.rhs_lanes), int(cfg.slab_log2),
            int(cfg.scaled_form), int(cfg.rhs_tile))


# ------------------------------------------------------------ instrumentation
def k3_last_layout() -> dict:
    """What the last pagerank() call iterated on (see pp_k3_last_layout)."""
    v = int(lib().pp_k3_last_layout())
    return {"relabelled": bool(v & 1), "segmented": bool(v & 2), "scaled": bool(v & 4),
            "packed": bool(v & 8)}


def set_kernel_timing(enable: bool) -> None:
    """Records HIP events around every sparse-product launch of pagerank()."""
    _check(lib().pp_set_kernel_timing(int(enable)), "pp_set_kernel_timing")


def kernel_times(cap: int = 256) -> list[float]:
    """Durations (ms) of the sparse-product launches of the last pagerank()."""
    buf = (ctypes.c_float * cap)()
    n = lib().pp_kernel_times(buf, cap)
    if n < 0:
        raise PPError(PP_EHIP, "pp_kernel_times", lib().pp_last_error().decode())
    return [float(buf[i]) for i in range(n)]
