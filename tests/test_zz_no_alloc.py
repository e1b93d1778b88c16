"""The allocation-free batch entry point, pp_pagerank_graphs_noalloc, against
the workspace form pp_pagerank_graphs (direct launch) on the same batches:
same kernels, so ranks and sums must agree bit for bit, and both must meet
the oracle's tolerance.  Two calls in a row, the second with a smaller batch
of another value type, so the second call starts from whatever the first
left in the library's static scratch (its queue counter in particular).
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


def batch(count, lo, hi, dtype, seed):
    specs = workloads.batch(count, lo, hi, seed)
    items, want = [], []
    tdt = torch.float32 if dtype == "f32" else torch.float64
    for i, sp in enumerate(specs):
        u, v = pp.generate(sp)
        us, vs = pp.sort(sp.scale, u, v)
        AT, _, _ = pp.filter(sp.scale, us, vs, dtype, degrees=False)
        r = torch.full((AT.n,), -1.0, dtype=tdt, device="cuda")
        sums = torch.full((21,), -1.0, dtype=torch.float64, device="cuda")
        rseed = 500 + 7 * i
        items.append((AT, r, sums, rseed))
        ou, ov = oracle.generate(oracle.Kron(**sp.as_dict()))
        ous, ovs = oracle.sort(sp.scale, ou, ov)
        f = oracle.filter(sp.scale, ous, ovs)
        want.append(oracle.pagerank(f.n, f.A_rp, f.A_col, f.A_val, oracle.init_r(f.n, rseed),
                                    20, C))
    return pp.GraphBatch(items, dtype), want, specs


def outputs(gb):
    torch.cuda.synchronize()
    return [(r.cpu().numpy().copy(), s.cpu().numpy().copy()) for _, r, s, _ in gb.items]


def reset(gb):
    for _, r, s, _ in gb.items:
        r.fill_(-1.0)
        s.fill_(-1.0)


def rel_l1(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def check_pair(gb, want, dtype, tag):
    print(f"[no_alloc] {tag}: {len(gb)} graphs {dtype}, workspace form", flush=True)
    reset(gb)
    pp.pagerank_graphs(gb, use_graph=False)
    ref = outputs(gb)
    print(f"[no_alloc] {tag}: allocation-free form", flush=True)
    reset(gb)
    pp.pagerank_graphs_noalloc(gb)
    got = outputs(gb)
    assert len(got) == len(ref) == len(gb)
    for (rg, sg), (rr, sr) in zip(got, ref):
        assert np.array_equal(rg, rr)
        assert np.array_equal(sg, sr)
    # GraphBatch lists graphs largest first; the seed names the oracle run.
    for (AT, r, s, seed), (rg, sg) in zip(gb.items, got):
        k = (seed - 500) // 7
        wr, ws = want[k]
        assert rel_l1(rg, wr) <= TOL[dtype]
        assert np.abs(sg / ws - 1).max() <= TOL[dtype]


def test_noalloc_matches_workspace_form_twice():
    assert torch.cuda.is_available()
    gb1, want1, _ = batch(24, 3, 13, "f32", seed=31)
    check_pair(gb1, want1, "f32", "first call")
    gb2, want2, _ = batch(5, 2, 9, "f64", seed=32)
    assert len(gb2) < len(gb1) and gb2.max_n < gb1.max_n
    check_pair(gb2, want2, "f64", "second call, smaller batch")
    # Over the static bound nothing is launched and the outputs stay as they were.
    reset(gb2)
    big = pp.GraphBatch([gb2.items[0]] * 2, "f64")
    big.table = (pp._Graph * (pp.graphs_noalloc_max() + 1))(*([gb2.table[0]] *
                                                              (pp.graphs_noalloc_max() + 1)))
    big.items = [gb2.items[0]] * (pp.graphs_noalloc_max() + 1)
    with pytest.raises(pp.PPError) as e:
        pp.pagerank_graphs_noalloc(big)
    assert e.value.status == pp.PP_ERANGE
    torch.cuda.synchronize()
    for _, r, s, _ in gb2.items:
        assert bool((r == -1.0).all()) and bool((s == -1.0).all())
