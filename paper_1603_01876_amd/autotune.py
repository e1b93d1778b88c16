"""Autotuner for the K3 launch configuration.

For a given matrix, value type and number of right-hand sides it measures
every candidate configuration of pagerank() -- SpMV items per thread
(4, 8, 16: the merge-path tile is 256 times that) or SpMM lane-group width
(the next power of two >= nrhs, or 64) -- with the library's HIP-event timing
of the sparse kernel, keeps the fastest and caches it in a JSON file keyed by
device architecture, size bucket, dtype, nrhs and whether vertices are
relabelled.  All candidates compute the same result up to the order of
floating-point sums.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import native as pp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pp_mi355x", "k3_tuning.json")


def candidates(nrhs: int) -> list[tuple[int, int]]:
    if nrhs == 1:
        return [(4, 0), (8, 0), (16, 0)]
    lanes = 2
    while lanes < nrhs:
        lanes *= 2
    return [(8, lanes)] + ([(8, 64)] if lanes < 64 else [])


def key(AT, dtype, nrhs: int, relabel: bool) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
        if torch.cuda.is_available() else "cpu"
    nb = int(math.log2(max(AT.n, 1)))
    zb = int(math.log2(max(AT.nnz, 1)))
    return f"{arch}|n2^{nb}|nnz2^{zb}|{dtype}|k{nrhs}|relabel{int(relabel)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(AT, dtype="f32", nrhs: int = 1, weights=None, iters: int = 4, cache: str | None = None,
         force: bool = False, ws=None) -> dict:
    """Measures the candidates on this matrix, applies the fastest with
    set_k3_config() and returns {"config": [ipt, lanes], "ms": {...}}."""
    cache = cache or DEFAULT_CACHE
    k = key(AT, dtype, nrhs, weights is not None)
    table = _load(cache)
    if not force and k in table:
        best = table[k]["config"]
        pp.set_k3_config(*best)
        return table[k]
    n = AT.n
    shape = (n,) if nrhs == 1 else (n, nrhs)
    tdt = torch.float32 if pp.dtype_code(dtype) == pp.F32 else torch.float64
    r = torch.empty(shape, dtype=tdt, device="cuda")
    if ws is None:
        ws = torch.empty(pp.workspace_bytes(pp.K3, n, AT.nnz, dtype, nrhs), dtype=torch.uint8,
                         device="cuda")
    times = {}
    pp.set_kernel_timing(True)
    try:
        for ipt, lanes in candidates(nrhs):
            pp.set_k3_config(ipt, lanes)
            pp.init_r(n, 1, dtype, nrhs, out=r, ws=ws)
            pp.pagerank(AT, r, iters=1, sums=False, ws=ws, weights=weights)   # warm-up
            pp.kernel_times()
            pp.pagerank(AT, r, iters=iters, sums=False, ws=ws, weights=weights)
            t = sorted(pp.kernel_times())
            times[f"{ipt},{lanes}"] = t[len(t) // 2]
    finally:
        pp.set_kernel_timing(False)
    best = min(times, key=times.get)
    cfg = [int(x) for x in best.split(",")]
    pp.set_k3_config(*cfg)
    entry = {"config": cfg, "ms": times}
    table[k] = entry
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    except OSError:
        pass
    return entry
