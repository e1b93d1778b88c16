"""Shared steps of the full-size parity tests (S = 24 and S = 26).

The expected values are tests/golden/kron_s<S>_pipeline.json, written by
tests/golden/make_pipeline_digests.py from the CPU oracle alone: 64-bit
order-independent digests (oracle.digest) of every array the pipeline
produces, K3's sums and sampled ranks.  The GPU side computes the same
digests over its full arrays, so "equal digests" means the whole array
matches bit for bit (up to a 2^-64 chance).  K3 ranks are compared in
full: once the GPU's FP64 CSR(A^T) digests equal the oracle's, the
oracle's K3 runs on the host from that matrix (row blocks on several
threads, bit-identical to the single-threaded iteration, which its r_20
digest against the stored one confirms) and every GPU run is held to the
relative L1 tolerance against it.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import torch

import oracle
from paper_1603_01876_amd import autotune
from paper_1603_01876_amd import native as pp
from paper_1603_01876_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f64": 1e-12, "f32": 1e-5}


def say(tag, msg):
    print(f"[{tag}] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def load(scale: int) -> dict:
    with open(os.path.join(HERE, "golden", f"kron_s{scale}_pipeline.json")) as fh:
        return json.load(fh)


def gpu_digest(t, count: int | None = None, chunk: int = 1 << 26) -> str:
    """oracle.digest of a device array (its first `count` elements), copied
    to the host piece by piece."""
    t = t.reshape(-1)
    count = t.numel() if count is None else count
    total = 0
    for a in range(0, count, chunk):
        b = min(count, a + chunk)
        total += oracle.digest(t[a:b].cpu().numpy(), a)
    return f"0x{total % (1 << 64):016x}"


def host_csr(AT):
    """CSR(A^T) copied to the host in the oracle's types."""
    z = AT.nnz
    rp = AT.row_ptr.cpu().numpy().astype(np.int64)
    col = AT.col[:z].cpu().numpy()
    val = AT.val[:z].cpu().numpy().astype(np.float64)
    return rp, col, val


def oracle_k3(AT64, golden: dict, tag: str):
    """The oracle's r_20 and sums from the GPU's FP64 CSR(A^T), whose digests
    the caller has already matched against the oracle's own."""
    rp, col, val = host_csr(AT64)
    n = AT64.n
    r0 = oracle.init_r(n, golden["r0_seed"])
    threads = max(1, min(16, os.cpu_count() or 1))
    say(tag, f"oracle K3 on the host, {threads} threads")
    r, sums = oracle.pagerank_rows(n, rp, col, val, r0, golden["iterations"], golden["damping"],
                                   threads=threads)
    del rp, col, val
    return r, sums


def k3_configs():
    """The library default plus every candidate the benchmark's tuner may
    time (items per thread, lanes, slab width, relabelling), each with the
    degree-scaled form on (the default; it applies to relabelled, segmented
    runs), plus the relabelled, segmented candidates with it off."""
    cands = [(8, 0, -1, False), (8, 0, -1, True)] + autotune.candidates(1, (False, True))
    on = [c + (1,) for c in cands]
    off = [c + (0,) for c in cands if c[3] and c[2] != 0]
    return on + off


def rel_l1(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def check_k3_configs(AT, dtype, d_out, want_r, want_sums, golden, ws, tag):
    """Runs K3 (init + iterations) in every configuration and holds r_20 and
    the sums to the tolerance against the oracle's; returns the errors."""
    n = AT.n
    iters = golden["iterations"]
    errs = {}
    saved = pp.get_k3_config()
    rows = np.asarray(golden["r20_rows"], np.int64)
    try:
        for cfg in k3_configs():
            pp.set_k3_config(*cfg[:3], cfg[4])
            r = pp.init_r(n, golden["r0_seed"], dtype, ws=ws)
            sums = pp.pagerank(AT, r, iters=iters, c=golden["damping"], ws=ws,
                               weights=d_out if cfg[3] else None)
            got = r.cpu().numpy().astype(np.float64)
            gs = sums.cpu().numpy()
            e = rel_l1(got, want_r)
            es = float(np.abs(gs / want_sums - 1).max())
            errs[autotune.name(cfg[:4]) + f",scaled{cfg[4]}"] = e
            say(tag, f"{dtype} config {autotune.name(cfg[:4])},scaled{cfg[4]}: rel L1 {e:.3e}, "
                     f"sums {es:.3e}")
            assert e <= TOL[dtype], (cfg, e)
            assert es <= TOL[dtype], (cfg, es)
            # The stored samples agree too (they are the same oracle run).
            assert rel_l1(got[rows], want_r[rows]) <= TOL[dtype]
            del r, sums, got
    finally:
        pp.set_k3_config(*saved)
    return errs
