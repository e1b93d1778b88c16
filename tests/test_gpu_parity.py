"""GPU parity: every kernel of libpp.so against the CPU oracle.

Integer work (edges, sort order, degrees, nnz, row pointers, columns) and
the K2 values (one IEEE division each side) must match bit for bit; K3
ranks must match within 1e-12 relative L1 (FP64) or 1e-5 (FP32 with
compensated sums), the tolerances the workload definition states.  Sizes
run from degenerate (S = 1, m = 0, empty matrices) through ragged tails to
S = 20 (16M edges), all on seeded synthetic inputs.
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
    torch.cuda.synchronize()


def spec(scale, k=16, seed=workloads.BASE_SEED):
    return workloads.GraphSpec(scale=scale, edge_factor=k, seed=seed)


def okron(s):
    return oracle.Kron(**s.as_dict())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def dev(a, dtype=torch.int64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def rel_l1(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())


# ----------------------------------------------------------------------- K0
@pytest.mark.parametrize("scale,k", [(1, 16), (2, 1), (5, 3), (10, 16), (16, 16), (20, 16)])
def test_generate_matches_oracle(scale, k):
    s = spec(scale, k)
    u, v = pp.generate(s)
    ou, ov = oracle.generate(okron(s))
    assert np.array_equal(host(u), ou)
    assert np.array_equal(host(v), ov)


def test_generate_other_initiator_and_seed():
    s = workloads.GraphSpec(scale=11, edge_factor=7, a=0.45, b=0.15, c=0.15, d=0.25,
                            seed=2**63 + 12345)
    u, v = pp.generate(s)
    ou, ov = oracle.generate(okron(s))
    assert np.array_equal(host(u), ou) and np.array_equal(host(v), ov)


# ----------------------------------------------------------------------- K1
@pytest.mark.parametrize("scale", [1, 3, 10, 16, 20])
def test_sort_pipeline_matches_oracle(scale):
    s = spec(scale)
    u, v = pp.generate(s)
    us, vs = pp.sort(scale, u, v)
    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort(scale, ou, ov)
    assert np.array_equal(host(us), ous)
    assert np.array_equal(host(vs), ovs)


@pytest.mark.parametrize("scale,m,skew", [(12, 12345, False), (3, 1, False), (3, 4097, True),
                                          (16, 100003, True), (9, 4096, False),
                                          (24, 70001, False)])
def test_sort_random_inputs(scale, m, skew):
    rng = np.random.default_rng(scale * 7 + m)
    n = 1 << scale
    if skew:
        u = np.minimum(rng.geometric(0.01, m) - 1, n - 1)
    else:
        u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    us, vs = pp.sort(scale, dev(u), dev(v))
    ous, ovs = oracle.sort(scale, u, v)
    assert np.array_equal(host(us), ous)
    assert np.array_equal(host(vs), ovs)


def test_sort_is_stable_on_equal_keys():
    m = 50000
    u = np.full(m, 5, np.int64)
    v = np.arange(m, dtype=np.int64) % 1024
    us, vs = pp.sort(10, dev(u), dev(v))
    assert np.array_equal(host(vs), v)


def test_sort_rejects_out_of_range():
    u = dev(np.array([0, 1, 1024, 3]))
    v = dev(np.array([0, 1, 2, 3]))
    with pytest.raises(pp.PPError) as e:
        pp.sort(10, u, v)
    assert e.value.status == pp.PP_EINVAL


@pytest.mark.parametrize("where", [0, 4095, 4096, 3 * 4096 + 16])
@pytest.mark.parametrize("which", ["u", "v", "negative"])
def test_sort_rejects_bad_label_in_any_tile(where, which):
    # One bad label anywhere in four 4096-key tiles (the last one ragged) is
    # caught, and the check does not stick: a valid call right after works.
    m = 3 * 4096 + 17
    rng = np.random.default_rng(where)
    u = rng.integers(0, 1 << 12, m)
    v = rng.integers(0, 1 << 12, m)
    if which == "u":
        u[where] = 1 << 12
    elif which == "v":
        v[where] = 1 << 12
    else:
        u[where] = -1
    with pytest.raises(pp.PPError) as e:
        pp.sort(12, dev(u), dev(v))
    assert e.value.status == pp.PP_EINVAL
    u[where] = v[where] = 7
    us, vs = pp.sort(12, dev(u), dev(v))
    ous, ovs = oracle.sort(12, u, v)
    assert np.array_equal(host(us), ous) and np.array_equal(host(vs), ovs)


# ----------------------------------------------------- K1 ordered by (u, v)
@pytest.mark.parametrize("scale", [1, 3, 8, 9, 10, 16, 20])
def test_sort_uv_pipeline_matches_oracle(scale):
    # 8 and 9: the second radix sort is forced to two passes below 9 bits
    s = spec(scale)
    u, v = pp.generate(s)
    us, vs = pp.sort_uv(scale, u, v)
    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort_uv(scale, ou, ov)
    assert np.array_equal(host(us), ous)
    assert np.array_equal(host(vs), ovs)


@pytest.mark.parametrize("scale,m,skew", [(12, 12345, False), (3, 1, False), (3, 4097, True),
                                          (16, 100003, True), (24, 70001, False)])
def test_sort_uv_random_inputs(scale, m, skew):
    rng = np.random.default_rng(scale * 11 + m)
    n = 1 << scale
    u = np.minimum(rng.geometric(0.01, m) - 1, n - 1) if skew else rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    us, vs = pp.sort_uv(scale, dev(u), dev(v))
    ous, ovs = oracle.sort_uv(scale, u, v)
    assert np.array_equal(host(us), ous) and np.array_equal(host(vs), ovs)


def test_sort_uv_feeds_the_same_filter():
    s = spec(14)
    u, v = pp.generate(s)
    (A, ain, aout), (B, bin_, bout) = (pp.filter(14, *srt(14, u, v), "f64")
                                       for srt in (pp.sort, pp.sort_uv))
    z = A.nnz
    assert B.nnz == z and torch.equal(A.row_ptr, B.row_ptr)
    assert torch.equal(A.col[:z], B.col[:z]) and torch.equal(A.val[:z], B.val[:z])
    assert torch.equal(ain, bin_) and torch.equal(aout, bout)


def test_sort_uv_rejects_out_of_range():
    u = dev(np.array([0, 1, 2, 3]))
    v = dev(np.array([0, 1, 1024, 3]))
    with pytest.raises(pp.PPError) as e:
        pp.sort_uv(10, u, v)
    assert e.value.status == pp.PP_EINVAL


# ----------------------------------------------------------------------- K2
def check_filter(scale, u_sorted, v_sorted, dtype):
    f = oracle.filter(scale, u_sorted, v_sorted)
    AT, d_in, d_out = pp.filter(scale, dev(u_sorted), dev(v_sorted), dtype)
    assert AT.nnz == f.nnz
    assert np.array_equal(host(d_in), f.d_in)
    assert np.array_equal(host(d_out), f.d_out)
    assert np.array_equal(host(AT.row_ptr), f.AT_rp)
    z = f.nnz
    assert np.array_equal(host(AT.col)[:z], f.AT_col)
    want = f.AT_val if dtype == "f64" else f.AT_val.astype(np.float32)
    assert np.array_equal(host(AT.val)[:z], want)
    # the row form CSR(A), bit for bit
    A = pp.transpose(AT)
    assert A.nnz == z
    assert np.array_equal(host(A.row_ptr), f.A_rp)
    assert np.array_equal(host(A.col)[:z], f.A_col)
    want = f.A_val if dtype == "f64" else f.A_val.astype(np.float32)
    assert np.array_equal(host(A.val)[:z], want)
    return AT, f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scale", [1, 4, 10, 16, 20])
def test_filter_matches_oracle(scale, dtype):
    s = spec(scale)
    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort(scale, ou, ov)
    check_filter(scale, ous, ovs, dtype)


@pytest.mark.parametrize("seed", range(4))
def test_filter_random_multigraphs(seed):
    rng = np.random.default_rng(100 + seed)
    scale = 9
    n = 1 << scale
    m = int(rng.integers(1, 30000))
    u = np.minimum(rng.geometric(0.02, m) - 1, n - 1)
    v = np.minimum(rng.geometric(0.03, m) - 1, n - 1)
    us, vs = oracle.sort(scale, u, v)
    check_filter(scale, us, vs, "f64")


def test_filter_special_graphs():
    # complete graph, star, permutation: every column is removed -> A = 0
    n = 1 << 6
    cu, cv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cases = [(cu.ravel(), cv.ravel()),
             (np.arange(n), np.zeros(n, np.int64)),
             (np.arange(n), np.random.default_rng(2).permutation(n))]
    for u, v in cases:
        us, vs = oracle.sort(6, u, v)
        AT, f = check_filter(6, us, vs, "f64")
        assert AT.nnz == 0


def test_filter_empty_edge_list():
    AT, d_in, d_out = pp.filter(5, dev(np.zeros(0)), dev(np.zeros(0)), "f64")
    assert AT.nnz == 0
    assert (host(AT.row_ptr) == 0).all() and (host(d_in) == 0).all()
    A = pp.transpose(AT)
    assert A.nnz == 0 and (host(A.row_ptr) == 0).all()


def test_filter_rejects_unsorted_input():
    u = dev(np.array([3, 1, 2]))
    v = dev(np.array([0, 1, 2]))
    with pytest.raises(pp.PPError) as e:
        pp.filter(4, u, v)
    assert e.value.status == pp.PP_EINVAL


@pytest.mark.parametrize("where", [1, 64, 4095, 4096, 2 * 4096 + 5])
def test_filter_rejects_one_descent_at_any_position(where):
    # u sorted except u[where-1] > u[where] (inside a wave, across waves and
    # across 4096-key tiles); the sorted input right after is filtered as the
    # oracle filters it.
    m = 3 * 4096 + 17
    rng = np.random.default_rng(where)
    u = np.sort(rng.integers(0, 4000, m))
    v = rng.integers(0, 1 << 12, m)
    bad = u.copy()
    bad[where - 1] = u[where] + 1
    with pytest.raises(pp.PPError) as e:
        pp.filter(12, dev(bad), dev(v))
    assert e.value.status == pp.PP_EINVAL
    us, vs = oracle.sort(12, u, v)
    check_filter(12, us, vs, "f32")


# ---------------------------------------------------------------- K3 init
@pytest.mark.parametrize("n,nrhs", [(1, 1), (1000, 1), (1 << 20, 1), (5000, 8), (777, 64)])
def test_init_r_matches_oracle(n, nrhs):
    r64 = host(pp.init_r(n, 4242, "f64", nrhs))
    r32 = host(pp.init_r(n, 4242, "f32", nrhs))
    for j in range(nrhs):
        want = oracle.init_r(n, 4242, j)
        got = r64 if nrhs == 1 else r64[:, j]
        assert np.array_equal(got, want)
        got32 = r32 if nrhs == 1 else r32[:, j]
        assert np.array_equal(got32, want.astype(np.float32))


# --------------------------------------------------------------- K3 iterate
def run_k3(n, A_rp, A_col, A_val, dtype, iters=20, seed=7, weights=None):
    """GPU K3 on CSR(A^T) built from the oracle's CSR(A); returns the GPU
    ranks, GPU sums and the oracle's ranks and sums.  `weights` (host
    array) turns on the vertex relabelling inside K3."""
    trp, tcol, tval = oracle.transpose_csr(n, A_rp, A_col, A_val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, dtype)
    r = pp.init_r(n, seed, dtype)
    w = None if weights is None else dev(weights, torch.int32)
    sums = pp.pagerank(AT, r, iters=iters, c=C, weights=w)
    want, wsums = oracle.pagerank(n, A_rp, A_col, A_val, oracle.init_r(n, seed), iters, C)
    return host(r), host(sums), want, wsums


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scale", [1, 4, 10, 16, 20])
def test_pagerank_on_kronecker_matrix(scale, dtype):
    s = spec(scale)
    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    got, sums, want, wsums = run_k3(f.n, f.A_rp, f.A_col, f.A_val, dtype)
    assert rel_l1(got, want) <= TOL[dtype]
    assert np.abs(sums / wsums - 1).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scale,kind", [(16, "d_out"), (16, "random"), (10, "negative"),
                                        (20, "d_out"), (1, "d_out")])
def test_pagerank_relabelled(scale, kind, dtype):
    # Relabelling by weights only changes speed and summation order.
    s = spec(scale)
    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    rng = np.random.default_rng(scale)
    w = {"d_out": f.d_out,
         "random": rng.integers(0, 1 << 20, f.n),
         "negative": rng.integers(-5, 5, f.n)}[kind]
    got, sums, want, wsums = run_k3(f.n, f.A_rp, f.A_col, f.A_val, dtype, weights=w)
    assert rel_l1(got, want) <= TOL[dtype]
    assert np.abs(sums / wsums - 1).max() <= TOL[dtype]


def random_matrix(n, rng, long_rows=(), density=3.0):
    """CSR(A) with ~density entries per row plus a few very long columns of
    A (= long rows of A^T) and rows left empty."""
    rows, cols = [], []
    k = rng.poisson(density, n)
    k[rng.random(n) < 0.4] = 0
    for i in range(n):
        if k[i]:
            cs = np.unique(rng.integers(0, n, k[i]))
            rows.append(np.full(cs.size, i))
            cols.append(cs)
    for j, length in long_rows:
        src = rng.choice(n, min(length, n), replace=False)
        rows.append(src)
        cols.append(np.full(src.size, j))
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
    val = rng.random(rows.size) / np.maximum(1, np.diff(rp))[rows]
    return rp, cols.astype(np.int32), val


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["long-rows", "tiny", "single", "dense-ish", "ragged"])
def test_pagerank_structured_matrices(case, dtype):
    rng = np.random.default_rng({"long-rows": 1, "tiny": 2, "single": 3, "dense-ish": 4,
                                 "ragged": 5}[case])
    if case == "long-rows":        # rows of A^T spanning many workgroups
        n = 60000
        rp, col, val = random_matrix(n, rng, long_rows=[(5, 50000), (n - 1, 30000), (777, 4097)])
    elif case == "tiny":
        n = 3
        rp, col, val = random_matrix(n, rng, density=2.0)
    elif case == "single":
        n = 1
        rp, col, val = np.array([0, 1]), np.array([0], np.int32), np.array([0.5])
    elif case == "dense-ish":
        n = 700
        rp, col, val = random_matrix(n, rng, density=200.0)
    else:
        n = 12345
        rp, col, val = random_matrix(n, rng, long_rows=[(0, 2048), (1, 2049), (2, 2047)])
    got, sums, want, wsums = run_k3(n, rp, col, val, dtype)
    assert rel_l1(got, want) <= TOL[dtype]
    assert np.abs(sums / wsums - 1).max() <= TOL[dtype]
    w = np.bincount(col, minlength=n)          # gather counts as weights
    got, sums, want, wsums = run_k3(n, rp, col, val, dtype, weights=w)
    assert rel_l1(got, want) <= TOL[dtype]
    assert np.abs(sums / wsums - 1).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pagerank_closed_form_permutation(dtype):
    n = 100003
    perm = np.random.default_rng(5).permutation(n)
    rp = np.arange(n + 1)
    col = perm.astype(np.int32)
    val = np.ones(n)
    got, sums, want, wsums = run_k3(n, rp, col, val, dtype)
    r0 = oracle.init_r(n, 7)
    x = r0.copy()
    for _ in range(20):
        y = np.empty(n)
        y[perm] = x
        x = y
    closed = C**20 * x + (1 - C**20) * r0.sum() / n
    assert rel_l1(got, closed) <= TOL[dtype]
    assert np.abs(sums - sums[0]).max() <= 64 * TOL[dtype] * sums[0]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pagerank_zero_matrix(dtype):
    n = 4099
    got, sums, want, wsums = run_k3(n, np.zeros(n + 1), np.zeros(0, np.int32), np.zeros(0), dtype)
    r0 = oracle.init_r(n, 7)
    closed = (1 - C) ** 20 * r0.sum() / n
    assert np.abs(got / closed - 1).max() <= TOL[dtype]


@pytest.mark.parametrize("iters", [0, 1, 2, 7])
def test_pagerank_iteration_counts(iters):
    n = 5000
    rng = np.random.default_rng(iters)
    rp, col, val = random_matrix(n, rng)
    got, sums, want, wsums = run_k3(n, rp, col, val, "f64", iters=iters)
    assert rel_l1(got, want) <= 1e-12
    assert np.abs(sums / wsums - 1).max() <= 1e-12


def test_pagerank_is_deterministic():
    s = spec(14)
    u, v = pp.generate(s)
    us, vs = pp.sort(14, u, v)
    AT, _, _ = pp.filter(14, us, vs, "f32")
    outs = []
    for _ in range(2):
        r = pp.init_r(AT.n, 3, "f32")
        sums = pp.pagerank(AT, r)
        outs.append((host(r).tobytes(), host(sums).tobytes()))
    assert outs[0] == outs[1]


# ------------------------------------------------------------ whole pipeline
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scale", [10, 20])
def test_pipeline_end_to_end(scale, dtype):
    s = spec(scale)
    u, v = pp.generate(s)
    us, vs = pp.sort(scale, u, v)
    AT, d_in, d_out = pp.filter(scale, us, vs, dtype)
    r = pp.init_r(AT.n, 11, dtype)
    sums = pp.pagerank(AT, r, weights=d_out)

    ou, ov = oracle.generate(okron(s))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    want, wsums = oracle.pagerank(f.n, f.A_rp, f.A_col, f.A_val, oracle.init_r(f.n, 11), 20, C)
    assert np.array_equal(host(us), ous) and np.array_equal(host(vs), ovs)
    assert AT.nnz == f.nnz
    assert np.array_equal(host(AT.row_ptr), f.AT_rp)
    assert np.array_equal(host(AT.col)[:f.nnz], f.AT_col)
    assert np.array_equal(host(d_in), f.d_in) and np.array_equal(host(d_out), f.d_out)
    assert rel_l1(host(r), want) <= TOL[dtype]
    assert np.abs(host(sums) / wsums - 1).max() <= TOL[dtype]


# ------------------------------------------------------- K3 batched (SpMM)
def run_k3_multi(n, A_rp, A_col, A_val, dtype, nrhs, iters=20, seed=9, weights=None):
    trp, tcol, tval = oracle.transpose_csr(n, A_rp, A_col, A_val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, dtype)
    r = pp.init_r(n, seed, dtype, nrhs)
    w = None if weights is None else dev(weights, torch.int32)
    sums = host(pp.pagerank(AT, r, iters=iters, c=C, weights=w))
    got = host(r).reshape(n, nrhs)
    sums = sums.reshape(iters + 1, nrhs)
    for j in range(nrhs):
        want, wsums = oracle.pagerank(n, A_rp, A_col, A_val, oracle.init_r(n, seed, j), iters, C)
        assert rel_l1(got[:, j], want) <= TOL[dtype], j
        assert np.abs(sums[:, j] / wsums - 1).max() <= TOL[dtype], j


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nrhs", [2, 3, 8, 32, 64])
def test_spmm_matches_independent_runs(nrhs, dtype):
    scale = 12
    ou, ov = oracle.generate(okron(spec(scale)))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    run_k3_multi(f.n, f.A_rp, f.A_col, f.A_val, dtype, nrhs)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nrhs,tile", [(32, 8), (32, 16), (12, 8), (17, 16), (5, 2), (64, 16)])
@pytest.mark.parametrize("relabel", [False, True])
def test_spmm_column_tiles(nrhs, tile, relabel, dtype):
    # Right-hand sides run `tile` columns at a time (the last tile narrower
    # when nrhs is not a multiple), each tile an n x T block of its own; every
    # column must still match its independent oracle run, with the caller's
    # r and sums in their usual row-major layout.
    scale = 12
    ou, ov = oracle.generate(okron(spec(scale)))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    pp.set_k3_config(8, 0, 0, 1, tile)
    try:
        run_k3_multi(f.n, f.A_rp, f.A_col, f.A_val, dtype, nrhs,
                     weights=f.d_out if relabel else None)
        if not relabel:
            run_k3_multi(f.n, f.A_rp, f.A_col, f.A_val, dtype, nrhs, iters=1)
    finally:
        pp.set_k3_config()


def test_spmm_column_tiles_zero_iterations():
    # No iteration: the tiled copy of r goes back unchanged.
    n, k = 5000, 24
    rng = np.random.default_rng(8)
    rp, col, val = random_matrix(n, rng)
    trp, tcol, tval = oracle.transpose_csr(n, rp, col, val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, "f32")
    r = pp.init_r(n, 4, "f32", k)
    before = host(r).copy()
    pp.set_k3_config(8, 0, 0, 1, 8)
    try:
        pp.pagerank(AT, r, iters=0, c=C)
    finally:
        pp.set_k3_config()
    assert host(r).tobytes() == before.tobytes()


@pytest.mark.parametrize("nrhs", [5, 32])
def test_spmm_relabelled_and_long_rows(nrhs):
    rng = np.random.default_rng(nrhs)
    n = 30000
    rp, col, val = random_matrix(n, rng, long_rows=[(3, 20000), (n - 2, 9000)])
    run_k3_multi(n, rp, col, val, "f32", nrhs, weights=np.bincount(col, minlength=n))
    run_k3_multi(n, rp, col, val, "f64", nrhs, iters=7)


def test_spmm_kronecker_s16_relabelled():
    scale = 16
    ou, ov = oracle.generate(okron(spec(scale)))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    run_k3_multi(f.n, f.A_rp, f.A_col, f.A_val, "f32", 32, weights=f.d_out)


# ------------------------------------------------------------ launch configs
@pytest.mark.parametrize("ipt", [4, 8, 16])
def test_spmv_configs_agree(ipt):
    scale = 14
    ou, ov = oracle.generate(okron(spec(scale)))
    ous, ovs = oracle.sort(scale, ou, ov)
    f = oracle.filter(scale, ous, ovs)
    pp.set_k3_config(ipt, 0)
    try:
        got, sums, want, wsums = run_k3(f.n, f.A_rp, f.A_col, f.A_val, "f64", weights=f.d_out)
        assert rel_l1(got, want) <= 1e-12
        got, sums, want, wsums = run_k3(f.n, f.A_rp, f.A_col, f.A_val, "f32")
        assert rel_l1(got, want) <= 1e-5
    finally:
        pp.set_k3_config()


def test_spmm_lane_width_and_autotuner(tmp_path):
    from paper_1603_01876_amd import autotune
    rng = np.random.default_rng(3)
    n = 20000
    rp, col, val = random_matrix(n, rng, long_rows=[(1, 9000)])
    pp.set_k3_config(8, 64)
    try:
        run_k3_multi(n, rp, col, val, "f32", 12)
    finally:
        pp.set_k3_config()
    trp, tcol, tval = oracle.transpose_csr(n, rp, col, val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, "f32")
    cache = str(tmp_path / "tune.json")
    weights = torch.as_tensor(np.bincount(col, minlength=n)).to(torch.int32).cuda()
    for k, w in ((1, None), (1, weights), (12, None)):
        entry = autotune.tune(AT, "f32", k, weights=w, iters=5, cache=cache)
        opts = (False, True) if w is not None else (False,)
        names = {autotune.name(cand) for cand in autotune.candidates(k, opts)}
        assert set(entry["ms"]) == names
        assert entry["candidate"] in names
        assert pp.get_k3_config() == tuple(entry["config"])
        again = autotune.tune(AT, "f32", k, weights=w, iters=5, cache=cache)   # from the cache
        assert again == entry
    pp.set_k3_config()
