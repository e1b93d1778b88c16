"""Pins for the oracle's K1 sort (Sec. IV.B) and K2 filter (Sec. IV.C).

K1 is pinned to a library routine (numpy's stable argsort).  K2 is pinned to
a dense brute force that spells out the paper's Matlab lines on an N x N
array, to special graphs whose filtered matrix is known to be empty, and to
invariants the text states (entries sum to M, fewer than M non-zeros,
normalised rows sum to one, removed columns are empty).
"""
import numpy as np
import pytest

from paper_1603_01876_amd import workloads


def kron(scale, seed=workloads.BASE_SEED):
    import oracle
    return oracle.Kron(**workloads.pipeline(scale, seed).as_dict())


# ----------------------------------------------------------------------- K1
@pytest.mark.parametrize("scale,m", [(1, 0), (1, 1), (1, 37), (4, 1000), (10, 16384), (12, 12345)])
def test_sort_matches_stable_argsort(ora, scale, m):
    rng = np.random.default_rng(scale * 1000 + m)
    n = 1 << scale
    u = rng.integers(0, n, m).astype(np.int64)
    v = rng.integers(0, n, m).astype(np.int64)
    uo, vo = ora.sort(scale, u, v)
    order = np.argsort(u, kind="stable")
    assert np.array_equal(uo, u[order]) and np.array_equal(vo, v[order])


def test_sort_generated_graph(ora):
    p = kron(12)
    u, v = ora.generate(p)
    uo, vo = ora.sort(12, u, v)
    assert (np.diff(uo) >= 0).all()
    order = np.argsort(u, kind="stable")
    assert np.array_equal(vo, v[order])


@pytest.mark.parametrize("scale,m", [(1, 0), (1, 1), (1, 37), (4, 1000), (10, 16384), (12, 12345)])
def test_sort_uv_matches_lexsort(ora, scale, m):
    # K1 with end vertices sorted too: numpy lexsort by (u, v).
    rng = np.random.default_rng(scale * 1000 + m + 1)
    n = 1 << scale
    u = rng.integers(0, n, m).astype(np.int64)
    v = rng.integers(0, n, m).astype(np.int64)
    uo, vo = ora.sort_uv(scale, u, v)
    order = np.lexsort((v, u))
    assert np.array_equal(uo, u[order]) and np.array_equal(vo, v[order])


def test_sort_uv_feeds_the_same_filter(ora):
    # K2 builds its matrix from the multiset of edges, so the order of the
    # end vertices within a start vertex cannot change its output.
    p = kron(11)
    u, v = ora.generate(p)
    a = ora.filter(11, *ora.sort(11, u, v))
    b = ora.filter(11, *ora.sort_uv(11, u, v))
    for name in ("AT_rp", "AT_col", "AT_val", "A_rp", "A_col", "A_val", "d_in", "d_out"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    with pytest.raises(RuntimeError):
        ora.sort_uv(3, np.array([1], np.int64), np.array([8], np.int64))


def test_sort_rejects_out_of_range(ora):
    with pytest.raises(RuntimeError):
        ora.sort(3, np.array([8], np.int64), np.array([0], np.int64))


# ----------------------------------------------------------------------- K2
def dense_filter(n, u, v):
    """Sec. IV.C written out on a dense array, one Matlab line at a time."""
    A = np.zeros((n, n), dtype=np.float64)
    np.add.at(A, (u, v), 1.0)                   # A = sparse(u,v,1,N,N)
    d_in = A.sum(axis=0)                        # d_in = sum(A,1)
    A[:, d_in == d_in.max()] = 0                # A(:,d_in == max(d_in)) = 0
    A[:, d_in == 1] = 0                         # A(:,d_in == 1) = 0
    d_out = A.sum(axis=1)                       # d_out = sum(A,2)
    i = d_out > 0                               # i = d_out > 0
    A[i, :] = A[i, :] / d_out[i][:, None]       # A(i,:) = A(i,:) ./ d_out(i)
    return A, d_in.astype(np.int64), d_out.astype(np.int64)


def csr_to_dense(n, rp, col, val):
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    D[rows, col] = val
    return D


def check_against_dense(ora, scale, u, v):
    n = 1 << scale
    f = ora.filter(scale, u, v)
    A, d_in, d_out = dense_filter(n, u, v)
    assert np.array_equal(f.d_in, d_in)
    assert np.array_equal(f.d_out, d_out)
    assert f.nnz == int((A != 0).sum())
    # Bit-exact values: both sides compute count / d_out in IEEE double.
    assert np.array_equal(csr_to_dense(n, f.A_rp, f.A_col, f.A_val), A)
    assert np.array_equal(csr_to_dense(n, f.AT_rp, f.AT_col, f.AT_val), A.T)
    # Canonical order: columns strictly ascending inside every row.
    for rp, col in ((f.A_rp, f.A_col), (f.AT_rp, f.AT_col)):
        for i in range(n):
            seg = col[rp[i]:rp[i + 1]]
            assert (np.diff(seg) > 0).all()
    return f


@pytest.mark.parametrize("scale", [4, 6, 8, 10])
def test_filter_matches_dense_on_kronecker(ora, scale):
    p = kron(scale)
    u, v = ora.generate(p)
    us, vs = ora.sort(scale, u, v)
    check_against_dense(ora, scale, us, vs)


@pytest.mark.parametrize("seed", range(6))
def test_filter_matches_dense_on_random_multigraphs(ora, seed):
    rng = np.random.default_rng(seed)
    scale = 5
    n = 1 << scale
    m = int(rng.integers(0, 400))
    # A skewed distribution gives many duplicate pairs and degree ties.
    u = np.minimum(rng.geometric(0.15, m) - 1, n - 1).astype(np.int64)
    v = np.minimum(rng.geometric(0.2, m) - 1, n - 1).astype(np.int64)
    check_against_dense(ora, scale, u, v)


def test_filter_unsorted_input_same_result(ora):
    p = kron(9)
    u, v = ora.generate(p)
    us, vs = ora.sort(9, u, v)
    a = ora.filter(9, u, v)
    b = ora.filter(9, us, vs)
    assert a.nnz == b.nnz
    assert np.array_equal(a.AT_col, b.AT_col) and np.array_equal(a.AT_val, b.AT_val)


def test_complete_graph_filters_to_zero(ora):
    # Every column has the same in-degree, which is the maximum.
    scale = 3
    n = 1 << scale
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = ora.filter(scale, u.ravel(), v.ravel())
    assert f.nnz == 0 and (f.d_out == 0).all() and (f.d_in == n).all()


def test_star_filters_to_zero(ora):
    scale = 4
    n = 1 << scale
    u = np.arange(n, dtype=np.int64)
    v = np.zeros(n, np.int64)
    f = ora.filter(scale, u, v)
    assert f.nnz == 0 and f.d_in[0] == n


def test_permutation_filters_to_zero(ora):
    # Every in-degree is one, which is also the maximum.
    scale = 6
    n = 1 << scale
    v = np.random.default_rng(1).permutation(n).astype(np.int64)
    f = ora.filter(scale, np.arange(n, dtype=np.int64), v)
    assert f.nnz == 0


def test_multiplicity_counts_toward_in_degree(ora):
    # Column 1 has a single distinct entry of count two: d_in = 2, kept.
    # Column 2 has in-degree 3 (the maximum) and column 3 in-degree 1.
    u = np.array([0, 0, 1, 2, 3, 4], np.int64)
    v = np.array([1, 1, 2, 2, 2, 3], np.int64)
    f = ora.filter(3, u, v)
    assert list(f.d_in[:4]) == [0, 2, 3, 1]
    assert f.nnz == 1
    assert list(f.A_rp[:3]) == [0, 1, 1] and f.A_col[0] == 1 and f.A_val[0] == 1.0


def test_ties_at_max_all_removed(ora):
    u = np.array([0, 1, 2, 3, 4, 5, 6, 7], np.int64)
    v = np.array([1, 1, 2, 2, 3, 3, 3, 3], np.int64)
    u = np.concatenate([u, [0, 1, 2, 3]])
    v = np.concatenate([v, [4, 4, 4, 4]])
    f = ora.filter(3, u, v)
    # d_in: col1=2, col2=2, col3=4, col4=4 -> cols 3 and 4 are both maxima.
    assert f.d_in[3] == f.d_in[4] == 4
    assert f.AT_rp[5] - f.AT_rp[3] == 0           # rows 3 and 4 of A^T empty
    assert f.nnz == 4


def test_invariants_generated(ora):
    scale = 12
    p = kron(scale)
    u, v = ora.generate(p)
    us, vs = ora.sort(scale, u, v)
    f = ora.filter(scale, us, vs)
    n, m = p.n, p.m
    assert f.d_in.sum() == m                      # entries of A sum to M
    assert 0 < f.nnz < m                          # fewer than M non-zeros
    mx = f.d_in.max()
    gone = (f.d_in == mx) | (f.d_in == 1)
    assert (np.diff(f.AT_rp)[gone] == 0).all()    # removed columns empty
    rowsum = np.add.reduceat(f.A_val, f.A_rp[:-1][np.diff(f.A_rp) > 0])
    assert np.abs(rowsum - 1.0).max() <= 64 * np.finfo(float).eps
    nonempty = np.diff(f.A_rp) > 0
    assert np.array_equal(nonempty, f.d_out > 0)
    # Sum of surviving counts per row equals d_out: val * d_out is an integer.
    rows = np.repeat(np.arange(n), np.diff(f.A_rp))
    cnt = f.A_val * f.d_out[rows]
    assert np.abs(cnt - np.rint(cnt)).max() < 1e-9
    assert np.array_equal(np.bincount(rows, weights=np.rint(cnt), minlength=n).astype(np.int64),
                          f.d_out)
    # A^T is the transpose of A.
    trp, tcol, tval = ora.transpose_csr(n, f.A_rp, f.A_col, f.A_val)
    assert np.array_equal(trp, f.AT_rp) and np.array_equal(tcol, f.AT_col)
    assert np.array_equal(tval, f.AT_val)


def test_filter_rows_matches_full_filter(ora):
    scale = 11
    p = kron(scale)
    u, v = ora.generate(p)
    us, vs = ora.sort(scale, u, v)
    f = ora.filter(scale, us, vs)
    rng = np.random.default_rng(3)
    rows = rng.choice(p.n, 300, replace=False)
    rows = np.concatenate([rows, [int(np.argmax(np.diff(f.AT_rp)))]])
    rp, col, val, d_in, d_out, mx, nnz = ora.filter_rows(scale, us, vs, rows, want_nnz=True)
    assert np.array_equal(d_in, f.d_in) and np.array_equal(d_out, f.d_out)
    assert mx == f.d_in.max() and nnz == f.nnz
    for q, j in enumerate(rows):
        a, b = f.AT_rp[j], f.AT_rp[j + 1]
        assert np.array_equal(col[rp[q]:rp[q + 1]], f.AT_col[a:b])
        assert np.array_equal(val[rp[q]:rp[q + 1]], f.AT_val[a:b])
