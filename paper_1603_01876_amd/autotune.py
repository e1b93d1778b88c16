"""Autotuner for the K3 launch configuration.

For a given matrix, value type, number of right-hand sides and iteration
count it runs pagerank() once per candidate configuration and keeps the one
whose whole call is fastest: per-call set-up (vertex relabelling, the
column-segmented layout) is paid once per call, so it is measured together
with the iterations it serves.  Candidates are

* nrhs == 1: one pass with 8 or 16 SpMV items per thread (the merge-path
  tile is 256 times that), or column slabs of 2^18, 2^19, 2^20 vertices with
  16 items per thread; each with vertex relabelling on or off when the
  caller passes weights;
* nrhs > 1: SpMM lane-group width (the next power of two >= nrhs, or 64)
  with all right-hand sides in one pass, or column tiles of 16 or 8
  right-hand sides (each tile its own n x T block; lanes = T), each with
  relabelling on or off when the caller passes weights.

The choice is applied with set_k3_config() and cached in a JSON file keyed
by device architecture, size bucket, dtype, nrhs, iteration count and
whether weights were offered.  All candidates compute the same result up to
the order of floating-point sums.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import native as pp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pp_mi355x", "k3_tuning.json")
SLABS = (0, 18, 19, 20)


RHS_TILES = (16, 8)


def candidates(nrhs: int, relabel_options=(False,)) -> list[tuple]:
    """(items_per_thread, rhs_lanes, slab_log2, relabel) tuples for one
    right-hand side; (items_per_thread, rhs_lanes, slab_log2, relabel,
    rhs_tile) for several (rhs_tile 0: all columns in one pass)."""
    if nrhs == 1:
        out = []
        for rl in relabel_options:
            out += [(8, 0, 0, rl), (16, 0, 0, rl)]
            out += [(16, 0, slab, rl) for slab in SLABS if slab]
        return out
    lanes = 2
    while lanes < nrhs:
        lanes *= 2
    out = [(8, lanes, 0, rl, 0) for rl in relabel_options]
    if lanes < 64:
        out += [(8, 64, 0, rl, 0) for rl in relabel_options]
    for t in RHS_TILES:
        if t < nrhs:
            out += [(8, 0, 0, rl, t) for rl in relabel_options]
    return out


def config_of(cand) -> list[int]:
    """set_k3_config() arguments of a candidate (degree-scaled form on)."""
    ipt, lanes, slab = (int(x) for x in cand[:3])
    tile = int(cand[4]) if len(cand) > 4 else 0
    return [ipt, lanes, slab, 1, tile]


def name(cand) -> str:
    return ",".join(str(int(x)) for x in cand)


def key(AT, dtype, nrhs: int, relabel: bool, iters: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
        if torch.cuda.is_available() else "cpu"
    nb = int(math.log2(max(AT.n, 1)))
    zb = int(math.log2(max(AT.nnz, 1)))
    return f"{arch}|n2^{nb}|nnz2^{zb}|{dtype}|k{nrhs}|it{iters}|weights{int(relabel)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(AT, dtype="f32", nrhs: int = 1, weights=None, iters: int = 20, cache: str | None = None,
         force: bool = False, ws=None, repeats: int = 2) -> dict:
    """Measures the candidates on this matrix, applies the fastest with
    set_k3_config() and returns {"config": set_k3_config() arguments,
    "relabel": bool, "candidate": its name, "ms": {candidate: ms per call}}.
    The caller passes `weights` to pagerank() only when "relabel" is true."""
    cache = cache or DEFAULT_CACHE
    k = key(AT, dtype, nrhs, weights is not None, iters)
    table = _load(cache)
    if not force and k in table:
        pp.set_k3_config(*table[k]["config"])
        return table[k]
    n = AT.n
    shape = (n,) if nrhs == 1 else (n, nrhs)
    tdt = torch.float32 if pp.dtype_code(dtype) == pp.F32 else torch.float64
    r = torch.empty(shape, dtype=tdt, device="cuda")
    if ws is None:
        ws = torch.empty(pp.workspace_bytes(pp.K3, n, AT.nnz, dtype, nrhs), dtype=torch.uint8,
                         device="cuda")
    opts = (False, True) if weights is not None else (False,)
    times = {}
    for cand in candidates(nrhs, opts):
        rl = bool(cand[3])
        pp.set_k3_config(*config_of(cand))
        w = weights if rl else None
        best = float("inf")
        for rep in range(repeats + 1):
            pp.init_r(n, 1, dtype, nrhs, out=r, ws=ws)
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            pp.pagerank(AT, r, iters=iters, sums=False, ws=ws, weights=w)
            t1.record()
            t1.synchronize()
            if rep > 0:                       # the first call warms up
                best = min(best, t0.elapsed_time(t1))
        times[name(cand)] = best
    win = min(times, key=times.get)
    cand = [int(x) for x in win.split(",")]
    cfg, relabel = config_of(cand), bool(cand[3])
    pp.set_k3_config(*cfg)
    entry = {"config": cfg, "relabel": relabel, "candidate": win, "ms": times}
    table[k] = entry
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    except OSError:
        pass
    return entry
