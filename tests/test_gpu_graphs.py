"""GPU parity for K3 on a batch of small graphs in one persistent launch.

Every graph's ranks and sums must match the oracle's K3 for that graph
within the FP32 / FP64 tolerance; a recorded hipGraph must reproduce the
eager launch bit for bit on every replay.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1603_01876_amd import native as pp
from paper_1603_01876_amd import workloads

pytestmark = pytest.mark.gpu

C = workloads.DAMPING
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pp.lib()
    yield


def okron(s):
    return oracle.Kron(**s.as_dict())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l1(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())


# ------------------------------------------------- K3 many small graphs
def small_batch(count, lo, hi, dtype, seed=77):
    """Pipeline K0-K2 on the GPU for `count` graphs plus their oracle K3."""
    specs = workloads.batch(count, lo, hi, seed)
    batch, want = [], []
    for i, sp in enumerate(specs):
        u, v = pp.generate(sp)
        us, vs = pp.sort(sp.scale, u, v)
        AT, _, _ = pp.filter(sp.scale, us, vs, dtype, degrees=False)
        r = torch.empty(AT.n, dtype=torch.float32 if dtype == "f32" else torch.float64,
                        device="cuda")
        sums = torch.empty(21, dtype=torch.float64, device="cuda")
        rseed = 1000 + i
        batch.append((AT, r, sums, rseed))
        ou, ov = oracle.generate(okron(sp))
        ous, ovs = oracle.sort(sp.scale, ou, ov)
        f = oracle.filter(sp.scale, ous, ovs)
        want.append(oracle.pagerank(f.n, f.A_rp, f.A_col, f.A_val, oracle.init_r(f.n, rseed), 20, C))
    return batch, want


def check_batch(batch, want, dtype):
    for (AT, r, sums, _), (wr, ws) in zip(batch, want):
        assert rel_l1(host(r), wr) <= TOL[dtype]
        assert np.abs(host(sums) / ws - 1).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graphs_batch_matches_oracle(dtype):
    hi = 12 if dtype == "f64" else 14
    items, want = small_batch(40, 2, hi, dtype)
    gb = pp.GraphBatch(items, dtype)
    assert gb.max_n <= pp.graphs_max_n(dtype)
    pp.pagerank_graphs(gb, use_graph=False)
    check_batch(items, want, dtype)


def test_graphs_hipgraph_replays():
    # Record once, replay three times with eager work and synchronisation
    # in between; every replay reproduces the eager result bit for bit.
    items, want = small_batch(24, 3, 12, "f32", seed=5)
    gb = pp.GraphBatch(items, "f32")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pp.pagerank_graphs(gb, use_graph=False)
        stream.synchronize()
        eager = [host(r).copy() for _, r, _, _ in items]
        for rep in range(3):
            for _, r, _, _ in items:
                r.zero_()
            junk = torch.randn(1 << 20, device="cuda").sum()       # unrelated eager work
            pp.pagerank_graphs(gb, use_graph=True)
            stream.synchronize()
            assert float(junk) == float(junk)
            for (_, r, _, _), e in zip(items, eager):
                assert np.array_equal(host(r), e), rep
    check_batch(items, want, "f32")


def test_graphs_reject_oversized_and_malformed():
    # Descriptors are checked on the host: a graph above the on-chip bound,
    # or one that lacks an array, fails the whole call before any launch,
    # and every output stays as it was.  The valid part of the batch then
    # runs and matches the oracle.
    items, want = small_batch(3, 6, 8, "f32", seed=9)
    limit = pp.graphs_max_n("f32")
    s = workloads.GraphSpec(scale=limit.bit_length())
    assert s.n > limit
    u, v = pp.generate(s)
    us, vs = pp.sort(s.scale, u, v)
    AT, _, _ = pp.filter(s.scale, us, vs, "f32", degrees=False)
    big = torch.empty(AT.n, dtype=torch.float32, device="cuda")
    for _, r, _, _ in items:
        r.fill_(-1.0)
    big.fill_(-1.0)
    gb = pp.GraphBatch(items + [(AT, big, None, 1)], "f32")
    with pytest.raises(pp.PPError) as e:
        pp.pagerank_graphs(gb, use_graph=False)
    assert e.value.status == pp.PP_ERANGE
    gb = pp.GraphBatch(items, "f32")
    k = next(i for i in range(len(gb)) if gb.table[i].nnz > 0)
    keep = gb.table[k].col
    gb.table[k].col = 0                      # entries but no column array
    with pytest.raises(pp.PPError) as e:
        pp.pagerank_graphs(gb, use_graph=False)
    assert e.value.status == pp.PP_EINVAL
    torch.cuda.synchronize()
    for _, r, _, _ in items:
        assert bool((r == -1.0).all())
    assert bool((big == -1.0).all())
    gb.table[k].col = keep
    pp.pagerank_graphs(gb, use_graph=False)
    check_batch(items, want, "f32")


# ------------------------------------------- structured small graphs
def csr_from_edges(n, edges):
    """Row form of A (rows u, values 1/out-degree) from (u, v) pairs."""
    edges = sorted(set(edges))
    rp = np.zeros(n + 1, np.int64)
    for u, _ in edges:
        rp[u + 1] += 1
    rp = np.cumsum(rp)
    col = np.array([v for _, v in edges], np.int64)
    deg = np.diff(rp)
    val = np.array([1.0 / deg[u] for u, _ in edges], np.float64)
    return rp, col, val


def structured_cases():
    rng = np.random.default_rng(11)
    cases = {}
    n = 5000
    cases["hub-row"] = (n, [(u, 0) for u in range(1, n)])             # one row of A^T holds every entry
    cases["hub-column"] = (n, [(0, v) for v in range(1, n)])          # n - 1 rows of one entry
    cases["no-entries"] = (300, [])
    cases["one-vertex"] = (1, [])
    cases["one-self-loop"] = (1, [(0, 0)])
    lens = [255, 256, 257, 0, 1, 511, 512, 513, 0, 0, 2]               # rows across 256-item rounds
    n = 2000
    edges = []
    for v in range(n):
        k = lens[v % len(lens)]
        for u in rng.choice(n, size=min(k, n), replace=False):
            edges.append((int(u), v))
    cases["round-edges"] = (n, edges)
    n = 4096
    live = rng.choice(n, size=64, replace=False)                        # most rows empty
    cases["sparse-rows"] = (n, [(int(u), int(v)) for v in live for u in rng.choice(n, 40, replace=False)])
    return cases


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graphs_structured_match_oracle(dtype):
    # Rows that span lanes, rounds and waves, empty graphs, one vertex and
    # empty rows, all in one batch; each graph against the oracle's K3.
    items, want = [], []
    for i, (name, (n, edges)) in enumerate(sorted(structured_cases().items())):
        rp, col, val = csr_from_edges(n, edges)
        trp, tcol, tval = oracle.transpose_csr(n, rp, col, val)
        AT = pp.CSR.from_arrays(n, trp, tcol, tval, dtype)
        r = torch.empty(n, dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")
        sums = torch.empty(21, dtype=torch.float64, device="cuda")
        items.append((AT, r, sums, 500 + i))
        want.append(oracle.pagerank(n, rp, col, val, oracle.init_r(n, 500 + i), 20, C))
    assert max(AT.n for AT, *_ in items) <= pp.graphs_max_n(dtype)
    gb = pp.GraphBatch(items, dtype)
    pp.pagerank_graphs(gb, use_graph=False)
    check_batch(items, want, dtype)
