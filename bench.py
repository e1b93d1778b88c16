#!/usr/bin/env python3
"""PageRank pipeline benchmark on one MI355X; prints one JSON line.

A step is one pass of the whole pipeline over one synthetic Kronecker graph
held in HBM: K0 generate, K1 sort, K2 filter (into CSR(A^T)), K3 PageRank
(initial vector + 20 damped iterations).  The headline metric is the
paper's K3 rate, 20*M / t_K3 edges per second (Sec. IV.D), on the largest
single-GPU instance (S = 26, M = 2^30 edges) at the paper's precision (FP64
values and ranks).  K1 and K2 rates (M/t, Sec. IV.B and IV.C) and the FP32
form (FP32 values and ranks, compensated row sums, FP64 sum(r) and
teleport) on the same graph are reported beside it, each with its error
against the oracle's ranks stored for this graph.  The roofline object
prices the SpMV iteration's algorithmic HBM bytes against its average
duration, timed with HIP events on its stream.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# L2 tag lookups: 16 channels per XCD, 8 XCDs, one 128 B lookup per channel
# per clock at the 2.4 GHz peak engine clock (a model figure, not measured).
L2_REQ_PEAK = 16 * 8 * 2.4e9
METRIC = "K3 PageRank edges/s (M\u00b720/t) + HBM GB/s, FP64 vs FP32 vs batched-RHS"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--dtype", default="f64", choices=["f32", "f64"],
                    help="value type of the timed run (the other one runs beside it)")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side-by-side run in the other value type")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-k12-scale", type=int, default=21,
                    help="graph scale of the oracle's K1/K2 timing")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-RHS form (S=22, 32 right-hand sides)")
    ap.add_argument("--batched-scale", type=int, default=22)
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the run-to-convergence form (dangling modes uniform and self)")
    ap.add_argument("--converge-tol", type=float, default=1e-6)
    ap.add_argument("--converge-max-iters", type=int, default=300)
    ap.add_argument("--no-k1-uv", action="store_true",
                    help="skip timing K1 ordered by (u, v)")
    ap.add_argument("--no-files", action="store_true",
                    help="skip the file-backed K1/K2 form (edge files on local storage)")
    ap.add_argument("--files-scale", type=int, default=22)
    ap.add_argument("--nfiles", type=int, default=16)
    ap.add_argument("--no-graphs", action="store_true",
                    help="skip the many-small-graphs form (512 graphs, S uniform on 8..14)")
    ap.add_argument("--ngraphs", type=int, default=512)
    ap.add_argument("--no-tune", action="store_true", help="keep the default K3 launch config")
    ap.add_argument("--k3-config", default=None,
                    help="K3 launch config 'items_per_thread,rhs_lanes,slab_log2' applied before "
                         "any run (with --no-tune it is the one timed)")
    ap.add_argument("--no-relabel", action="store_true",
                    help="iterate on K2's labels (no degree-ordered relabelling inside K3)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB three times (reference for rocprofv3 byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain device copy of known size: rocprofv3's FETCH_SIZE / WRITE_SIZE
    read for it gives the factor that turns those counters into bytes."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": 1 << 30, "copies": 3}), flush=True)


def measured_traffic(scale: int, dtype: str, cfg, relabel: bool):
    """From the committed rocprofv3 counter summary for this workload: HBM
    bytes per K3 iteration ("traffic", GB) and the raw SpMV's L1-to-L2 read
    requests per launch with its traced duration ("l2"); None when there is
    no summary, when it was taken with another launch configuration, or when
    the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k3_spmv_kron_s{scale}_{dtype}_counters.md")
    src = os.path.join(ROOT, "paper_1603_01876_amd", "csrc", "k3_pagerank.hip")
    if not os.path.exists(path):
        return None
    keys = ("kernel_source_sha256", "fetch_bytes_per_launch", "write_bytes_per_launch",
            "k3_config", "relabel", "spmv_l2_read_requests_per_launch", "spmv_launch_us")
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in keys:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha:
        return None
    if fields.get("k3_config") != ",".join(str(x) for x in cfg) or \
            fields.get("relabel") != str(int(relabel)):
        return None
    out = {"traffic": (float(fields["fetch_bytes_per_launch"]) +
                       float(fields["write_bytes_per_launch"])) / 1e9}
    if "spmv_l2_read_requests_per_launch" in fields and "spmv_launch_us" in fields:
        req = float(fields["spmv_l2_read_requests_per_launch"])
        us = float(fields["spmv_launch_us"])
        out["l2"] = {"kernel": "k_spmv raw (column-segmented)",
                     "read_requests_per_launch": req, "launch_us": us,
                     "requests_per_s": req / (us * 1e-6),
                     "source": os.path.basename(path)}
    return out


def limiter(mt):
    """What binds the dominant kernel, from the committed counters: the raw
    SpMV's L1-to-L2 read requests per second against the L2's tag-lookup
    rate, beside its HBM bytes.  None without a matching summary."""
    if not mt or "l2" not in mt:
        return None
    l2 = mt["l2"]
    return {"resource": "L2 request rate (one request per gathered value of r)",
            "requests_per_s": l2["requests_per_s"], "model_peak_requests_per_s": L2_REQ_PEAK,
            "frac": l2["requests_per_s"] / L2_REQ_PEAK, "source": l2["source"]}


def copy_ceiling(torch, nbytes=1 << 31, reps=5):
    """Streaming-copy bandwidth of the device (read + write bytes per second
    of a plain device-to-device copy), the practical ceiling beside the
    8 TB/s vendor figure."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


def spmv_label(cfg, dt, layout=None):
    v = "float" if dt == "f32" else "double"
    if cfg[2] > 0:
        ent = ""
        if layout and layout.get("scaled"):
            ent = ",packed" if layout.get("packed") else ",uint8"
        form = {"": "", ",uint8": " (degree-scaled form: entries stored as counts)",
                ",packed": " (degree-scaled form: each entry one 4-byte word, column inside the slab"
                           " and count)"}[ent]
        return (f"segmented SpMV iteration, slabs of 2^{cfg[2]} columns{form}: "
                f"k_spmv<{v},{cfg[0]},raw{ent}> + k_fix_raw<{v}> + k_seg_combine<{v}> + "
                f"k_sum_blocks")
    return f"k_spmv<{v},{cfg[0]}> + k_finish<{v}>"


def form_bytes(n: int, nnz: int, dtype: str, layout) -> int | None:
    """Bytes one iteration of the degree-scaled form must move at the
    least: row pointers 4(N+1), columns 4Z, one count byte per entry, the
    gathered vector once and the next one written, and the out-degrees the
    combine divides by (4N).  Packed with the column: 4 bytes per entry.
    None for the value form (spmv_bytes)."""
    if not layout or not layout.get("scaled"):
        return None
    w = 8 if dtype == "f64" else 4
    per = 4 if layout.get("packed") else 5
    return 4 * (n + 1) + per * nnz + 2 * w * n + 4 * n


def batched_form(args, pp, workloads, torch):
    """K3 with nrhs independent vectors on one S=22 matrix (one SpMM per
    iteration) beside nrhs times the single-vector run, in FP32 and in FP64
    (the batched form's speed-up and error against each)."""
    S, k, dev = args.batched_scale, args.nrhs, "cuda"
    spec = workloads.pipeline(S)
    n, m = spec.n, spec.m
    u, v = pp.generate(spec)
    us, vs = pp.sort(S, u, v)
    del u, v
    AT, _, d_out = pp.filter(S, us, vs, "f32")
    AT64, _, _ = pp.filter(S, us, vs, "f64", degrees=False)
    del us, vs
    w = None if args.no_relabel else d_out
    ws = torch.empty(max(pp.workspace_bytes(pp.K3, n, AT.nnz, "f32", k),
                         pp.workspace_bytes(pp.K3, n, AT.nnz, "f64", 1)),
                     dtype=torch.uint8, device=dev)
    tuned = None
    if not args.no_tune:
        from paper_1603_01876_amd import autotune
        tuned = autotune.tune(AT, "f32", k, w, ws=ws, iters=args.iters, force=True)
        if not tuned["relabel"]:
            w = None
    rk = torch.empty((n, k), dtype=torch.float32, device=dev)
    r1 = torch.empty(n, dtype=torch.float32, device=dev)

    def timed(fn, reps=3):
        ts, kt = [], []
        pp.set_kernel_timing(True)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            kt += pp.kernel_times()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        pp.set_kernel_timing(False)
        return sum(ts) / len(ts), sum(kt) / len(kt) / 1e3

    def run_k():
        pp.init_r(n, workloads.BASE_SEED, "f32", k, out=rk, ws=ws)
        pp.pagerank(AT, rk, iters=args.iters, c=workloads.DAMPING, sums=False, ws=ws, weights=w)

    run_k()
    tk, kk = timed(run_k)
    saved = pp.get_k3_config()
    w1 = w
    if not args.no_tune:
        from paper_1603_01876_amd import autotune
        t1cfg = autotune.tune(AT, "f32", 1, w, ws=ws, iters=args.iters, force=True)
        w1 = w if t1cfg["relabel"] else None

    def run_1():
        pp.init_r(n, workloads.BASE_SEED, "f32", 1, out=r1, ws=ws)
        pp.pagerank(AT, r1, iters=args.iters, c=workloads.DAMPING, sums=False, ws=ws, weights=w1)

    run_1()
    t1, k1 = timed(run_1)
    # The same single vector at the paper's precision (FP64 values and ranks).
    r64 = torch.empty(n, dtype=torch.float64, device=dev)
    w64 = w
    if not args.no_tune:
        t64cfg = autotune.tune(AT64, "f64", 1, w, ws=ws, iters=args.iters, force=True)
        w64 = w if t64cfg["relabel"] else None

    def run_64():
        pp.init_r(n, workloads.BASE_SEED, "f64", 1, out=r64, ws=ws)
        pp.pagerank(AT64, r64, iters=args.iters, c=workloads.DAMPING, sums=False, ws=ws,
                    weights=w64)

    run_64()
    t64, _ = timed(run_64)
    pp.set_k3_config(*saved)
    err = float((rk[:, 0].double() - r1.double()).abs().sum() / r1.double().abs().sum())
    err64 = float((rk[:, 0].double() - r64).abs().sum() / r64.abs().sum())
    nbytes = 4 * (n + 1) + 8 * AT.nnz + 8 * n * k
    out = {"workload": f"kron-s{S}-f32-rhs{k}", "nrhs": k, "nnz_filtered": AT.nnz,
           "k3_ms": tk * 1e3, "rhs_edges_per_s": args.iters * m * k / tk,
           "single_rhs_k3_ms": t1 * 1e3, "single_rhs_edges_per_s": args.iters * m / t1,
           "per_rhs_speedup_over_single": t1 * k / tk,
           "single_rhs_f64_k3_ms": t64 * 1e3,
           "per_rhs_speedup_over_single_f64": t64 * k / tk,
           "rel_l1_rhs0_vs_single_f64": err64,
           "spmm_avg_ms": kk * 1e3, "spmm_GBps": nbytes / kk / 1e9,
           "spmm_frac_of_peak": nbytes / kk / 1e9 / HBM_PEAK_GBS,
           "spmm_algorithmic_bytes_per_launch": nbytes,
           "rel_l1_rhs0_vs_single_f32": err,
           "spmm_config": None if tuned is None else tuned}
    del AT, AT64, ws, rk, r1, r64, d_out
    torch.cuda.empty_cache()
    return out


def graphs_form(args, pp, workloads, torch):
    """K3 for many independent small graphs: one persistent launch recorded
    into a hipGraph and replayed, beside one pp_pagerank call per graph."""
    specs = workloads.batch(args.ngraphs, 8, 14, workloads.BASE_SEED)
    items, edges, nnz = [], 0, 0
    for i, sp in enumerate(specs):
        u, v = pp.generate(sp)
        us, vs = pp.sort(sp.scale, u, v)
        AT, _, _ = pp.filter(sp.scale, us, vs, "f32", degrees=False)
        r = torch.empty(AT.n, dtype=torch.float32, device="cuda")
        items.append((AT, r, None, 7000 + i))
        edges += sp.m
        nnz += AT.nnz
    gb = pp.GraphBatch(items, "f32")
    stream = torch.cuda.Stream()
    ts = []
    with torch.cuda.stream(stream):
        pp.pagerank_graphs(gb, iters=args.iters, c=workloads.DAMPING, use_graph=True)
        stream.synchronize()
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pp.pagerank_graphs(gb, iters=args.iters, c=workloads.DAMPING, use_graph=True)
            e1.record()
            stream.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        r_persist = [r.clone() for _, r, _, _ in gb.items]
        # The same work as one pp_init_r + pp_pagerank call per graph.
        ws = torch.empty(pp.workspace_bytes(pp.K3, 1 << 14, 1 << 19, "f32"), dtype=torch.uint8,
                         device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for AT, r, _, seed in gb.items:
            pp.init_r(AT.n, seed, "f32", out=r, ws=ws)
            pp.pagerank(AT, r, iters=args.iters, c=workloads.DAMPING, sums=False, ws=ws)
        e1.record()
        stream.synchronize()
        t_calls = e0.elapsed_time(e1) / 1e3
        err = max(float((a.double() - r.double()).abs().sum() / r.double().abs().sum())
                  for a, (_, r, _, _) in zip(r_persist, gb.items))
    t = min(ts)
    # Algorithmic bytes as for one SpMV per graph and iteration (8Z + 12N + 4
    # in FP32); each graph's CSR is read from HBM once and from L2 in its
    # later iterations, r and y never leave LDS.
    alg = sum(spmv_bytes(AT.n, AT.nnz, "f32") for AT, *_ in gb.items) * args.iters
    once = sum(4 * (AT.n + 1) + 8 * AT.nnz for AT, *_ in gb.items)
    roof = {"bound": "hbm", "kernel": "k_graphs<float> (one persistent launch)",
            "achieved": alg / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg / t / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg,
            "csr_bytes_read_once": once, "csr_once_GBps": once / t / 1e9}
    return {"workload": f"kron-batch{args.ngraphs}-s8to14-f32", "graphs": args.ngraphs,
            "edges_total": edges, "nnz_total": nnz, "k3_ms": t * 1e3, "roofline": roof,
            "k3_ms_mean": sum(ts) / len(ts) * 1e3,
            "edges_per_s": args.iters * edges / t,
            "per_graph_calls_ms": t_calls * 1e3,
            "speedup_over_per_graph_calls": t_calls / t,
            "max_rel_l1_vs_per_graph_calls": err,
            "launch": "one persistent kernel, replayed from a hipGraph"}


def converge_form(args, pp, workloads, torch, AT, d_out, r, ws, m, relabel, plain_ms):
    """K3 run to a convergence test on the benchmark's matrix: for dangling
    modes uniform and self, iterations until the normalised L1 difference
    is <= tol, timed from pp_init_r to the end (HIP events, best of two
    calls after one warm-up); rate = iterations * M / t like the K3 metric."""
    n = AT.n
    dt = pp.dtype_code(r.dtype)
    out = {"workload": f"kron-s{args.scale}-{args.dtype}-converge", "tol": args.converge_tol,
           "max_iters": args.converge_max_iters, "relabel": relabel,
           "plain_iteration_ms": plain_ms}
    for mode in ("uniform", "self"):
        best = None
        for rep in range(3):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            pp.init_r(n, workloads.BASE_SEED, dt, out=r, ws=ws)
            sums, deltas, k = pp.pagerank_converge(
                AT, r, args.converge_max_iters, args.converge_tol, mode, d_out=d_out,
                c=workloads.DAMPING, weights=d_out if relabel else None, ws=ws)
            t1.record()
            t1.synchronize()
            ms = t0.elapsed_time(t1)
            if rep > 0 and (best is None or ms < best[0]):
                best = (ms, k, float(deltas[-1]) if k else None,
                        float(abs(sums[-1] / sums[0] - 1)))
        ms, k, last, drift = best
        out[mode] = {"iterations": k, "ms": ms, "edges_per_s": k * m / (ms / 1e3) if k else 0.0,
                     "ms_per_iteration": ms / k if k else None, "last_delta": last,
                     "sum_r_rel_drift": drift}
    return out


def fs_type(path: str) -> str:
    """File system type of the mount holding path (from /proc/mounts)."""
    best, kind = "", "unknown"
    try:
        with open("/proc/mounts") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 3 and path.startswith(parts[1]) and len(parts[1]) > len(best):
                    best, kind = parts[1], parts[2]
    except OSError:
        pass
    return kind


def files_form(args, pp, workloads, torch):
    """The paper's file-backed K1 and K2 (Sec. IV.B-C): K0 writes the edges
    as text files (untimed); K1 reads them, parses, sorts, formats and
    writes the sorted edges (fsync: non-volatile storage); K2 reads those,
    parses and filters.  Rates are M / t with every step inside t."""
    import shutil
    import tempfile
    S = args.files_scale
    spec = workloads.pipeline(S)
    n, m = spec.n, spec.m
    dev = "cuda"
    u = torch.empty(m, dtype=torch.int64, device=dev)
    v = torch.empty(m, dtype=torch.int64, device=dev)
    us = torch.empty_like(u)
    vs = torch.empty_like(v)
    text = torch.empty(22 * m, dtype=torch.uint8, device=dev)
    ws1 = torch.empty(pp.workspace_bytes(pp.K1, n, m), dtype=torch.uint8, device=dev)
    wsf = torch.empty(pp.workspace_bytes(pp.TSV_FORMAT, 0, m, "f64", args.nfiles),
                      dtype=torch.uint8, device=dev)
    wsp = torch.empty(pp.workspace_bytes(pp.TSV_PARSE, 0, 22 * m, "f64"), dtype=torch.uint8,
                      device=dev)
    AT = pp.CSR(n, 0, torch.empty(n + 1, dtype=torch.int32, device=dev),
                torch.empty(m, dtype=torch.int32, device=dev),
                torch.empty(m, dtype=torch.float32, device=dev))
    ws2 = torch.empty(pp.workspace_bytes(pp.K2, n, m), dtype=torch.uint8, device=dev)
    d_in = torch.empty(n, dtype=torch.int32, device=dev)
    d_out = torch.empty(n, dtype=torch.int32, device=dev)
    root = tempfile.mkdtemp(prefix="pp_edges_")
    k0, k1 = os.path.join(root, "k0"), os.path.join(root, "k1")
    F = args.nfiles
    try:
        pp.generate(spec, u, v)
        t, split = pp.tsv_format(S, u, v, nsplit=F, text=text, ws=wsf)
        pp.write_text_files(k0, text, split)
        text_bytes = split[-1]
        best = None
        for rep in range(2):   # the faster of two runs
            st = {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nb = pp.read_text_files(k0, F, text)
            t1 = time.perf_counter()
            pu, pv = pp.tsv_parse(S, text, nb, cap=m, u=u, v=v, ws=wsp)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            pp.sort(S, pu, pv, us, vs, ws=ws1)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            _, split1 = pp.tsv_format(S, us, vs, nsplit=F, text=text, ws=wsf)
            t4 = time.perf_counter()
            pp.write_text_files(k1, text, split1, sync=True)
            t5 = time.perf_counter()
            st["k1"] = {"read_ms": (t1 - t0) * 1e3, "parse_ms": (t2 - t1) * 1e3,
                        "sort_ms": (t3 - t2) * 1e3, "format_ms": (t4 - t3) * 1e3,
                        "write_fsync_ms": (t5 - t4) * 1e3, "total_ms": (t5 - t0) * 1e3}
            torch.cuda.synchronize()
            t6 = time.perf_counter()
            nb2 = pp.read_text_files(k1, F, text)
            t7 = time.perf_counter()
            qu, qv = pp.tsv_parse(S, text, nb2, cap=m, u=u, v=v, ws=wsp)
            torch.cuda.synchronize()
            t8 = time.perf_counter()
            pp.filter(S, qu, qv, "f32", AT=AT, d_in=d_in, d_out=d_out, ws=ws2)
            torch.cuda.synchronize()
            t9 = time.perf_counter()
            st["k2"] = {"read_ms": (t7 - t6) * 1e3, "parse_ms": (t8 - t7) * 1e3,
                        "filter_ms": (t9 - t8) * 1e3, "total_ms": (t9 - t6) * 1e3}
            tot = st["k1"]["total_ms"] + st["k2"]["total_ms"]
            if best is None or tot < best[0]:
                best = (tot, st)
        best = best[1]
        out = {"workload": f"kron-s{S}-files", "edges": m, "files": F, "text_bytes": text_bytes,
               "fsync": True, "filesystem": fs_type(root), "nnz_filtered": AT.nnz}
        for k in ("k1", "k2"):
            out[k] = best[k]
            out[k]["edges_per_s"] = m / (best[k]["total_ms"] / 1e3)
        out["k1"]["read_GBps"] = text_bytes / best["k1"]["read_ms"] / 1e6
        out["k1"]["write_GBps"] = text_bytes / best["k1"]["write_fsync_ms"] / 1e6
        out["k1"]["parse_GBps"] = text_bytes / best["k1"]["parse_ms"] / 1e6
        return out
    finally:
        shutil.rmtree(root, ignore_errors=True)


def spmv_bytes(n: int, nnz: int, dtype: str) -> int:
    """Algorithmic HBM bytes of one pull-form SpMV launch: row pointers
    4(N+1), columns 4Z, values Z*sizeof(val), x read once N*sizeof(val), y
    written once N*sizeof(val)."""
    w = 8 if dtype == "f64" else 4
    return 4 * (n + 1) + (4 + w) * nnz + 2 * w * n


def host_cpu() -> dict:
    """The host's CPU model and core counts (from /proc/cpuinfo and the
    scheduler's affinity mask)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model or platform.processor() or platform.machine(),
            "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(AT, scale: int, m: int, budget_s: float, k12_scale: int):
    """The oracle (single thread, FP64) timed on the host: K3 as one damped
    iteration over a contiguous block of rows of the benchmark's CSR(A^T)
    (scaled to K3 edges/s: the rows hold a fraction f of the nnz, so the
    rate is f*M / t_rows, one iteration processing M edges in the paper's
    metric), and K1 / K2 (M/t) over the whole pipeline of a smaller graph
    of the same family (scale k12_scale: the oracle's K1 and K2 at the
    benchmark's scale take minutes).  K0 is untimed, as in the paper."""
    import numpy as np
    import oracle

    n, z = AT.n, AT.nnz
    rp = AT.row_ptr.cpu().numpy().astype(np.int64)
    # Calibrate on a small block, then size the sample to the budget.
    r = np.full(n, 1.0 / n)
    target = max(1, min(z, 2_000_000))
    rows = int(np.searchsorted(rp, target))
    rows = max(1, min(rows, n))
    t0 = time.perf_counter()
    _run_rows(oracle, AT, rp, r, 0, rows)
    t_cal = time.perf_counter() - t0
    per_nnz = t_cal / max(1, rp[rows])
    want = int(min(z, budget_s / max(per_nnz, 1e-12)))
    rows2 = int(np.searchsorted(rp, want))
    rows2 = max(rows, min(rows2, n))
    t0 = time.perf_counter()
    _run_rows(oracle, AT, rp, r, 0, rows2)
    t = time.perf_counter() - t0
    f = float(rp[rows2]) / float(max(z, 1))
    value = f * m / t
    del rp, r
    # K1 and K2 of the oracle on a whole graph of the same family.
    from paper_1603_01876_amd import workloads
    spec = workloads.pipeline(k12_scale)
    p = oracle.Kron(**spec.as_dict())
    info = host_cpu()
    u, v = oracle.generate_parallel(p, threads=max(1, min(16, info["usable_cpus"] or 1)))
    t1 = time.perf_counter()
    us, vs = oracle.sort(k12_scale, u, v)
    t2 = time.perf_counter()
    del u, v
    fl = oracle.filter(k12_scale, us, vs)
    t3 = time.perf_counter()
    del us, vs, fl
    return {"value": value, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": (f"K3: oracle ppo_step_rows (FP64, 1 thread) on rows [0, {rows2}) of the "
                       f"S={scale} CSR(A^T): {int(f * z)} of {z} nnz ({100*f:.1f}%), one "
                       f"iteration, {t:.1f} s; rate = fraction * M / t.  K1/K2: oracle ppo_sort "
                       f"and ppo_filter (1 thread) on the whole S={k12_scale} graph "
                       f"({spec.m} edges)"),
            "k1": {"edges_per_s": spec.m / (t2 - t1), "s": t2 - t1, "scale": k12_scale},
            "k2": {"edges_per_s": spec.m / (t3 - t2), "s": t3 - t2, "scale": k12_scale},
            "host_cpu": info}


def oracle_error(r, scale: int, iters: int, seed: int) -> dict | None:
    """Error of the GPU's r_iters against the oracle's ranks for the same
    graph, as stored by tests/golden/make_pipeline_digests.py (an oracle-only
    script): relative L1 over the stored sample of rows (random rows plus the
    64 largest ranks), over the 256 block sums of r, and of sum(r); None when
    no stored values match this workload."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"kron_s{scale}_pipeline.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    if g["iterations"] != iters or g["r0_seed"] != seed:
        return None
    got = r.double().cpu().numpy()
    rows = np.asarray(g["r20_rows"], np.int64)
    want = np.array([float.fromhex(x) for x in g["r20_values"]])
    out = {"sampled_rows": int(rows.size),
           "sampled_rel_l1": float(np.abs(got[rows] - want).sum() / np.abs(want).sum())}
    if "r20_block_sums" in g:
        wb = np.array([float.fromhex(x) for x in g["r20_block_sums"]])
        gb = got.reshape(wb.size, -1).sum(axis=1)
        out["block_sums_rel_l1"] = float(np.abs(gb - wb).sum() / np.abs(wb).sum())
    wl1 = float.fromhex(g["r20_l1"])
    out["l1_rel"] = float(abs(np.abs(got).sum() / wl1 - 1))
    out["source"] = os.path.relpath(path, ROOT)
    return out


def _run_rows(oracle, AT, rp, r, r0, r1):
    import numpy as np
    a, b = int(rp[r0]), int(rp[r1])
    col = AT.col[a:b].cpu().numpy()
    val = AT.val[a:b].cpu().numpy().astype(np.float64)
    sub = (rp[r0:r1 + 1] - a).astype(np.int64)
    return oracle.step_rows(AT.n, sub, col, val, r, 1.0, 0.85)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU path is a design, not a build", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1603_01876_amd import native as pp
    from paper_1603_01876_amd import workloads

    torch.cuda.set_device(0)
    dev = "cuda"
    if args.k3_config:
        pp.set_k3_config(*[int(x) for x in args.k3_config.split(",")])
    S, dt = args.scale, args.dtype
    spec = workloads.pipeline(S)
    n, m = spec.n, spec.m
    tdt = torch.float32 if dt == "f32" else torch.float64
    log(f"S={S} N={n} M={m} dtype={dt}: allocating")

    u = torch.empty(m, dtype=torch.int64, device=dev)
    v = torch.empty(m, dtype=torch.int64, device=dev)
    us = torch.empty(m, dtype=torch.int64, device=dev)
    vs = torch.empty(m, dtype=torch.int64, device=dev)
    ws12 = torch.empty(max(pp.workspace_bytes(pp.K1, n, m), pp.workspace_bytes(pp.K2, n, m)),
                       dtype=torch.uint8, device=dev)
    AT = pp.CSR(n, 0, torch.empty(n + 1, dtype=torch.int32, device=dev),
                torch.empty(m, dtype=torch.int32, device=dev),
                torch.empty(m, dtype=tdt, device=dev))
    d_in = torch.empty(n, dtype=torch.int32, device=dev)
    d_out = torch.empty(n, dtype=torch.int32, device=dev)
    r = torch.empty(n, dtype=tdt, device=dev)
    sums = torch.empty(args.iters + 1, dtype=torch.float64, device=dev)
    ws3 = torch.empty(pp.workspace_bytes(pp.K3, n, m, dt), dtype=torch.uint8, device=dev)
    rseed = workloads.BASE_SEED
    state = {"relabel": not args.no_relabel}

    def step(timed):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        pp.generate(spec, u, v)
        ev[1].record()
        pp.sort(S, u, v, us, vs, ws=ws12)
        ev[2].record()
        pp.filter(S, us, vs, dt, AT=AT, d_in=d_in, d_out=d_out, ws=ws12)
        ev[3].record()
        pp.init_r(n, rseed, dt, out=r, ws=ws3)
        pp.pagerank(AT, r, iters=args.iters, c=workloads.DAMPING, sums=sums, ws=ws3,
                    weights=d_out if state["relabel"] else None)
        ev[4].record()
        return ev

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup step {i} done (nnz={AT.nnz})")
        if i == 0 and not args.no_tune:
            from paper_1603_01876_amd import autotune
            tuned = autotune.tune(AT, dt, 1, None if args.no_relabel else d_out, ws=ws3,
                                  iters=args.iters, force=True)
            state["relabel"] = tuned["relabel"]
            log(f"autotuned K3 config {tuned['config']} relabel={tuned['relabel']} "
                f"from {tuned['ms']}")

    pp.set_kernel_timing(True)
    spmv_ms = []
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs.append(step(True))
        spmv_ms += pp.kernel_times()      # waits for this step's last SpMV
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pp.set_kernel_timing(False)
    layout = pp.k3_last_layout()
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s (K3 layout {layout})")

    k = {name: [] for name in ("k0", "k1", "k2", "k3")}
    for ev in evs:
        for j, name in enumerate(("k0", "k1", "k2", "k3")):
            k[name].append(ev[j].elapsed_time(ev[j + 1]) / 1e3)
    mean = {key: sum(val) / len(val) for key, val in k.items()}
    z = AT.nnz
    value = args.iters * m / mean["k3"]
    spmv_avg_s = sum(spmv_ms) / len(spmv_ms) / 1e3
    nbytes = spmv_bytes(n, z, dt)
    achieved = nbytes / spmv_avg_s / 1e9
    sums_h = sums.cpu().numpy()

    copy_bw = copy_ceiling(torch)
    mt = measured_traffic(S, dt, pp.get_k3_config(), state["relabel"])
    log(f"device copy ceiling {copy_bw:.0f} GB/s")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": (t1 - t0) / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic Kronecker graph (seeded counter-based generator, K0 on the GPU)",
        "config": {"workload": f"kron-s{S}-{dt}", "scale": S, "vertices": n, "edges": m,
                   "edge_factor": spec.edge_factor, "initiator": [spec.a, spec.b, spec.c, spec.d],
                   "nnz_filtered": z, "iterations": args.iters, "damping": workloads.DAMPING,
                   "parallelism": "single GPU"},
        "kernels": {
            "k0_ms": mean["k0"] * 1e3, "k1_ms": mean["k1"] * 1e3, "k2_ms": mean["k2"] * 1e3,
            "k3_ms": mean["k3"] * 1e3,
            "k1_edges_per_s": m / mean["k1"], "k2_edges_per_s": m / mean["k2"],
            "k3_edges_per_s": value,
            "spmv_avg_ms": spmv_avg_s * 1e3, "spmv_launches": len(spmv_ms),
        },
        "roofline": {"bound": "hbm", "kernel": spmv_label(pp.get_k3_config(), dt, layout),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "form_bytes_per_launch": form_bytes(n, z, dt, layout),
                     "traffic": (mt or {}).get("traffic"),
                     "traffic_unit": "GB per iteration (rocprofv3 FETCH_SIZE + WRITE_SIZE over the iteration's launches, copy-calibrated)",
                     "algorithmic_bytes_per_launch": nbytes,
                     "copy_GBps": copy_bw, "frac_of_copy": achieved / copy_bw,
                     "l2_requests": (mt or {}).get("l2"),
                     "limiter": limiter(mt)},
        "sum_r": {"first": float(sums_h[0]), "last": float(sums_h[-1])},
        "k3_config": {"items_per_thread": pp.get_k3_config()[0],
                      "slab_log2": pp.get_k3_config()[2],
                      "scaled_form": pp.get_k3_config()[3],
                      "relabel": state["relabel"], "layout": layout,
                      "tuned": None if args.no_tune or args.warmup < 1 else tuned["ms"]},
    }

    # K1 with end vertices sorted too (Sec. V): same edges, same buffers.
    tk = []
    for rep in range(0 if args.no_k1_uv else 3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        pp.sort_uv(S, u, v, us, vs, ws=ws12)
        e1.record()
        e1.synchronize()
        tk.append(e0.elapsed_time(e1) / 1e3)
    if tk:
        t_uv = min(tk[1:])
        out.setdefault("forms", {})["k1_sorted_uv"] = {
            "workload": f"kron-s{S}", "k1_uv_ms": t_uv * 1e3, "k1_uv_edges_per_s": m / t_uv,
            "k1_u_ms": mean["k1"] * 1e3, "cost_over_u_only": t_uv / mean["k1"]}

    out["error_vs_oracle"] = {dt: oracle_error(r, S, args.iters, rseed)}
    if not args.no_side:
        other = "f32" if dt == "f64" else "f64"
        log(f"{other.upper()} side by side")
        odt = torch.float32 if other == "f32" else torch.float64
        r_main = r.double().clone()
        ATo = pp.CSR(n, 0, torch.empty(n + 1, dtype=torch.int32, device=dev),
                     torch.empty(m, dtype=torch.int32, device=dev),
                     torch.empty(m, dtype=odt, device=dev))
        pp.filter(S, us, vs, other, AT=ATo, d_in=d_in, d_out=d_out, ws=ws12)
        need = pp.workspace_bytes(pp.K3, n, m, other)
        wso = ws3 if ws3.numel() >= need else torch.empty(need, dtype=torch.uint8, device=dev)
        ro = torch.empty(n, dtype=odt, device=dev)
        sums_o = torch.empty(args.iters + 1, dtype=torch.float64, device=dev)
        saved = pp.get_k3_config()
        wo = None if args.no_relabel else d_out
        tuned_o = None
        if not args.no_tune:
            from paper_1603_01876_amd import autotune
            tuned_o = autotune.tune(ATo, other, 1, wo, ws=wso, iters=args.iters, force=True)
            if not tuned_o["relabel"]:
                wo = None
        cfg_o = pp.get_k3_config()
        times = []
        pp.set_kernel_timing(True)
        spmv_o = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pp.init_r(n, rseed, other, out=ro, ws=wso)
            pp.pagerank(ATo, ro, iters=args.iters, c=workloads.DAMPING, sums=sums_o, ws=wso,
                        weights=wo)
            e1.record()
            spmv_o += pp.kernel_times()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        pp.set_kernel_timing(False)
        layout_o = pp.k3_last_layout()
        pp.set_k3_config(*saved)
        t_o = sum(times) / len(times)
        s_o = sum(spmv_o) / len(spmv_o) / 1e3
        b_o = spmv_bytes(n, ATo.nnz, other)
        out.setdefault("forms", {})[other] = {
            "workload": f"kron-s{S}-{other}", "k3_edges_per_s": args.iters * m / t_o,
            "k3_ms": t_o * 1e3, "spmv_avg_ms": s_o * 1e3, "spmv_GBps": b_o / s_o / 1e9,
            "spmv_frac_of_peak": b_o / s_o / 1e9 / HBM_PEAK_GBS,
            "kernel": spmv_label(cfg_o, other, layout_o), "relabel": wo is not None,
            "k3_config": list(cfg_o), "layout": layout_o,
            "form_bytes_per_launch": form_bytes(n, ATo.nnz, other, layout_o),
            "tuned": None if tuned_o is None else tuned_o["ms"]}
        t32, t64 = (mean["k3"], t_o) if dt == "f32" else (t_o, mean["k3"])
        r32, r64 = (r_main, ro.double()) if dt == "f32" else (ro.double(), r_main)
        out["f32_speedup_over_f64"] = t64 / t32
        out["f32_rel_l1_vs_f64_gpu"] = float((r32 - r64).abs().sum() / r64.abs().sum())
        out["error_vs_oracle"][other] = oracle_error(ro, S, args.iters, rseed)
        del ATo, ro, r_main, r32, r64
        if wso is not ws3:
            del wso
        torch.cuda.empty_cache()

    if not args.no_converge:
        log("run to convergence")
        if not args.no_tune and args.warmup >= 1:
            pp.set_k3_config(*tuned["config"])
        elif args.k3_config is None:
            pp.set_k3_config()
        out.setdefault("forms", {})["converge"] = converge_form(
            args, pp, workloads, torch, AT, d_out, r, ws3, m, state["relabel"], spmv_avg_s * 1e3)

    if not args.no_batched:
        log("batched right-hand sides")
        torch.cuda.empty_cache()
        out.setdefault("forms", {})["batched_rhs"] = batched_form(args, pp, workloads, torch)

    if not args.no_files:
        log("file-backed K1/K2")
        torch.cuda.empty_cache()
        out.setdefault("forms", {})["files"] = files_form(args, pp, workloads, torch)

    if not args.no_graphs:
        log("many small graphs")
        out.setdefault("forms", {})["graphs"] = graphs_form(args, pp, workloads, torch)

    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(AT, S, m, args.cpu_seconds, args.cpu_k12_scale)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
