"""Writes tests/golden/kron_s<S>_pipeline.json: what the CPU oracle computes
for the benchmark's Kronecker pipeline at scale S (seed 1603, edge factor
16, initiator 0.57/0.19/0.19/0.05, K3 from r_0 of seed 1603, c = 0.85, 20
iterations), as order-independent 64-bit digests of every array (ppo_digest)
plus K3's sums and sampled ranks.  It calls nothing but the oracle package;
the GPU tests compare the library's full arrays against these values.

    python tests/golden/make_pipeline_digests.py 24 26 [--threads T]

Each edge range of K0, each block of rows of K2 (ppo_filter_rows) and each
block of rows of a K3 iteration (ppo_step_rows) is the oracle's own
single-threaded code; threads only run independent ranges side by side (the
tooling tests pin the row-block forms against ppo_filter and ppo_pagerank).
At S = 26 the run needs about 40 GB of host memory and several minutes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1603_01876_amd import workloads  # noqa: E402

SAMPLE_ROWS = 1024
TOP_ROWS = 64
RANK_BLOCKS = 256


def say(t0, msg):
    print(f"[{time.time() - t0:7.1f} s] {msg}", flush=True)


def dig(x) -> str:
    return f"0x{oracle.digest(x):016x}"


def run(scale: int, threads: int) -> dict:
    t0 = time.time()
    spec = workloads.pipeline(scale)
    p = oracle.Kron(**spec.as_dict())
    n, m = spec.n, spec.m
    out = {"scale": scale, "vertices": n, "edges": m, "edge_factor": spec.edge_factor,
           "initiator": [spec.a, spec.b, spec.c, spec.d], "seed": spec.seed,
           "r0_seed": workloads.BASE_SEED, "damping": workloads.DAMPING,
           "iterations": workloads.ITERATIONS, "digest": {}}
    d = out["digest"]
    say(t0, f"S={scale}: K0, {m} edges")
    u, v = oracle.generate_parallel(p, threads)
    d["u"], d["v"] = dig(u), dig(v)
    say(t0, "K1")
    us, vs = oracle.sort(scale, u, v)
    del u, v
    d["u_sorted"], d["v_sorted"] = dig(us), dig(vs)
    say(t0, "K2")
    if scale <= 24:
        f = oracle.filter(scale, us, vs)
        rp, col, val, d_in, d_out, nnz = f.AT_rp, f.AT_col, f.AT_val, f.d_in, f.d_out, f.nnz
        mx = int(d_in.max())
        d["A_row_ptr"], d["A_col"], d["A_val_f64"] = dig(f.A_rp), dig(f.A_col), dig(f.A_val)
        del f
    else:
        rp, col, val, d_in, d_out, mx, nnz = oracle.filter_blocks(scale, us, vs, nblocks=16,
                                                                  threads=min(threads, 3))
    del us, vs
    out["nnz"] = int(nnz)
    out["max_in_degree"] = int(mx)
    d["d_in"], d["d_out"] = dig(d_in), dig(d_out)
    d["AT_row_ptr"], d["AT_col"] = dig(rp), dig(col)
    d["AT_val_f64"] = dig(val)
    d["AT_val_f32"] = dig(val.astype(np.float32))
    out["empty_rows_of_A"] = int((d_out == 0).sum())
    del d_in, d_out
    say(t0, f"K3 (nnz {nnz})")
    r0 = oracle.init_r(n, workloads.BASE_SEED)
    d["r0_f64"], d["r0_f32"] = dig(r0), dig(r0.astype(np.float32))
    r, sums = oracle.pagerank_rows(n, rp, col, val, r0, workloads.ITERATIONS,
                                   workloads.DAMPING, threads=threads)
    out["sums"] = [float(x).hex() for x in sums]
    rng = np.random.default_rng(2026)
    rows = np.unique(np.concatenate([rng.integers(0, n, SAMPLE_ROWS),
                                     np.argsort(r, kind="stable")[-TOP_ROWS:]]))
    out["r20_rows"] = [int(x) for x in rows]
    out["r20_values"] = [float(x).hex() for x in r[rows]]
    out["r20_l1"] = float(np.abs(r).sum()).hex()
    blk = r.reshape(RANK_BLOCKS, -1) if n % RANK_BLOCKS == 0 else None
    if blk is not None:
        out["r20_block_sums"] = [float(x).hex() for x in blk.sum(axis=1)]
    d["r20_f64"] = dig(r)
    say(t0, "done")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("scales", type=int, nargs="+")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for s in a.scales:
        res = run(s, a.threads)
        path = os.path.join(HERE, f"kron_s{s}_pipeline.json")
        with open(path, "w") as fh:
            # One key per line, each value compact.
            fh.write("{\n" + ",\n".join(f" {json.dumps(k)}: {json.dumps(v)}"
                                         for k, v in res.items()) + "\n}\n")
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
