"""Pins for the oracle's K3 PageRank (Sec. IV.D and the Appendix).

Pinned by: a dense power iteration (numpy matmul, the formula of Sec. IV.D
with the teleport (1-c)/N * sum(r) of the Appendix); closed forms for a
permutation matrix and for A = 0; the exact recurrence of sum(r) (constant
when no row is empty); the eigenvector check the paper itself proposes
(Perron vector of c*A.' + (1-c)/N); and the exact integer construction of
the initial vector.
"""
import numpy as np
import pytest

from paper_1603_01876_amd import workloads

C = workloads.DAMPING


def kron(scale, seed=workloads.BASE_SEED):
    import oracle
    return oracle.Kron(**workloads.pipeline(scale, seed).as_dict())


def relL1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def pipeline_matrix(ora, scale, seed=workloads.BASE_SEED):
    p = kron(scale, seed)
    u, v = ora.generate(p)
    us, vs = ora.sort(scale, u, v)
    return p, ora.filter(scale, us, vs)


def dense_A(n, rp, col, val):
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), col] = val
    return A


# ------------------------------------------------------------------ init
@pytest.mark.parametrize("n", [1, 2, 1000, 1 << 16])
def test_init_r_exact_normalisation(ora, n):
    r = ora.init_r(n, 1603)
    assert (r >= 0).all()
    assert abs(r.sum() - 1.0) <= n * np.finfo(float).eps
    # r_i * K are the 24-bit draws: integers below 2^24 (K = their sum).
    draws = np.array([ora.philox4x32_10([i, 0, 0, 2], [1603, 0])[0] >> 8 for i in range(min(n, 500))],
                     dtype=np.float64)
    if n <= 500:
        assert np.array_equal(r, draws / draws.sum())
    else:
        # r_i / k_i is the same constant 1/K for every i.
        ratio = r[:500] / draws
        assert np.abs(ratio / ratio[0] - 1).max() <= 4 * np.finfo(float).eps


def test_init_r_rhs_independent(ora):
    a = ora.init_r(4096, 7, 0)
    b = ora.init_r(4096, 7, 1)
    assert not np.array_equal(a, b)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.1


# ------------------------------------------------------------------ dense
@pytest.mark.parametrize("scale", [6, 8, 10])
def test_pagerank_matches_dense_power_iteration(ora, scale):
    p, f = pipeline_matrix(ora, scale)
    n = p.n
    A = dense_A(n, f.A_rp, f.A_col, f.A_val)
    r0 = ora.init_r(n, 99)
    r, sums = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r0, iters=20, c=C)
    x = r0.copy()
    for _ in range(20):
        x = (C * x) @ A + (1 - C) / n * x.sum()
    assert relL1(r, x) <= 1e-14
    assert abs(sums[0] - r0.sum()) <= 1e-15


def test_transposed_operand_would_fail(ora):
    # Guard: on this matrix r*A and r*A.' differ far beyond the tolerance,
    # so the dense pin distinguishes the orientation.
    p, f = pipeline_matrix(ora, 8)
    n = p.n
    A = dense_A(n, f.A_rp, f.A_col, f.A_val)
    r0 = ora.init_r(n, 99)
    r, _ = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r0, iters=3, c=C)
    x = r0.copy()
    for _ in range(3):
        x = (C * x) @ A.T + (1 - C) / n * x.sum()
    assert relL1(r, x) > 1e-3


# ------------------------------------------------------------ closed forms
def test_closed_form_permutation(ora):
    n = 1000
    perm = np.random.default_rng(5).permutation(n)
    rp = np.arange(n + 1, dtype=np.int64)
    col = perm.astype(np.int32)
    val = np.ones(n)
    r0 = ora.init_r(n, 3)
    s0 = r0.sum()
    x = r0.copy()
    for k in range(1, 21):
        r, _ = ora.pagerank(n, rp, col, val, r0, iters=k, c=C)
        y = np.empty(n)
        y[perm] = x            # (x P)_j = x_i where j = perm[i]
        x = y
        want = C**k * x + (1 - C**k) * s0 / n
        assert relL1(r, want) <= 1e-14, k


def test_closed_form_zero_matrix(ora):
    n = 777
    rp = np.zeros(n + 1, np.int64)
    r0 = ora.init_r(n, 4)
    s0 = r0.sum()
    for k in (1, 2, 5, 20):
        r, sums = ora.pagerank(n, rp, np.zeros(0, np.int32), np.zeros(0), r0, iters=k, c=C)
        want = (1 - C)**k * s0 / n
        assert np.abs(r / want - 1).max() <= 1e-13
        assert abs(sums[k] / ((1 - C)**k * s0) - 1) <= 1e-13


# --------------------------------------------------------------- invariants
def test_sum_recurrence(ora):
    # sum(r_{k+1}) = sum(r_k) - c * sum of r_k over rows of A that are empty.
    p, f = pipeline_matrix(ora, 12)
    n = p.n
    dangling = np.diff(f.A_rp) == 0
    r = ora.init_r(n, 11)
    for k in range(5):
        r1, sums = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r, iters=1, c=C)
        want = r.sum() - C * r[dangling].sum()
        assert abs(sums[1] - want) <= 1e-13 * want
        r = r1


def test_sum_invariant_without_empty_rows(ora):
    # Every row non-empty: a ring plus random extra edges, rows normalised.
    n = 2048
    rng = np.random.default_rng(8)
    rows, cols = [], []
    for i in range(n):
        extra = rng.integers(0, n, rng.integers(0, 6))
        cs = np.unique(np.concatenate([[(i + 1) % n], extra]))
        rows += [i] * cs.size
        cols += list(cs)
    rows = np.array(rows)
    cols = np.array(cols, np.int32)
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
    val = 1.0 / np.diff(rp)[rows]
    r0 = ora.init_r(n, 2)
    r, sums = ora.pagerank(n, rp, cols, val, r0, iters=20, c=C)
    assert np.abs(sums - sums[0]).max() <= 1e-13


# -------------------------------------------------------------- eigenvector
@pytest.mark.parametrize("scale", [6, 8])
def test_eigenvector_check(ora, scale):
    # Sec. IV.D: r./norm(r,1) equals the leading eigenvector of
    # c*A.' + (1-c)/N, normalised the same way.  Twenty iterations do not
    # converge (0.85^20 ~ 0.04), so iterate until the normalised vector is
    # stationary to 1e-15 and compare with numpy's eigensolver.
    p, f = pipeline_matrix(ora, scale)
    n = p.n
    A = dense_A(n, f.A_rp, f.A_col, f.A_val)
    G = C * A.T + (1 - C) / n
    w, V = np.linalg.eig(G)
    k = int(np.argmax(w.real))
    r1 = np.abs(V[:, k].real)
    r1 /= r1.sum()
    r, _ = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, ora.init_r(n, 1), iters=400, c=C)
    r = r / np.abs(r).sum()
    assert np.abs(r - r1).sum() <= 1e-10


# ----------------------------------------------------------------- step rows
def test_step_rows_equals_one_iteration(ora):
    p, f = pipeline_matrix(ora, 10)
    n = p.n
    r0 = ora.init_r(n, 21)
    r1, sums = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r0, iters=1, c=C)
    y = ora.step_rows(n, f.AT_rp, f.AT_col, f.AT_val, r0, sums[0], C)
    assert np.array_equal(y, r1)       # same summation order: bit-exact


# ------------------------------------------------------- accuracy of the sums
@pytest.mark.parametrize("scale", [12, 16])
def test_pagerank_matches_extended_precision(ora, scale):
    # The iteration computed in x87 extended precision (64-bit significand)
    # with numpy: the oracle's compensated FP64 sums must agree to ~1e-16,
    # far inside the 1e-12 FP64 tolerance the GPU is held to.
    p, f = pipeline_matrix(ora, scale)
    n = p.n
    r0 = ora.init_r(n, 7)
    r, sums = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r0, iters=20, c=C)
    rows = np.repeat(np.arange(n), np.diff(f.AT_rp))
    x = r0.astype(np.longdouble)
    val = f.AT_val.astype(np.longdouble)
    cl = np.longdouble(C)
    a = (np.longdouble(1) - cl) / np.longdouble(n)
    for _ in range(20):
        y = np.zeros(n, np.longdouble)
        np.add.at(y, rows, x[f.AT_col] * val)
        x = cl * y + a * x.sum()
    err = float(np.abs(r.astype(np.longdouble) - x).sum() / np.abs(x).sum())
    assert err <= 1e-15
    assert abs(float(sums[-1] / x.sum()) - 1.0) <= 1e-15


# ------------------------------------------------- run to convergence (Sec. IV.D)
# The convergence test is the normed sum of the differences between two
# iterates, each divided by its sum; dangling modes: "none" (the benchmark),
# "uniform" (a dangling vertex spreads c*r_i evenly), "self" (A(i,i) = 1 in
# every empty row of A, Sec. V).
def mode_matrix(n, A, mode):
    """Dense matrix whose leading eigenvector the converged r must be."""
    d = (np.abs(A).sum(axis=1) == 0).astype(float)
    if mode == "uniform":
        A = A + np.outer(d, np.ones(n)) / n
    elif mode == "self":
        A = A + np.diag(d)
    return C * A.T + (1 - C) / n


@pytest.mark.parametrize("mode", ["none", "uniform", "self"])
@pytest.mark.parametrize("scale", [6, 8])
def test_converge_eigenvector(ora, scale, mode):
    p, f = pipeline_matrix(ora, scale)
    n = p.n
    A = dense_A(n, f.A_rp, f.A_col, f.A_val)
    assert (np.diff(f.A_rp) == 0).sum() > n // 10       # plenty of dangling vertices
    w, V = np.linalg.eig(mode_matrix(n, A, mode))
    k = int(np.argmax(w.real))
    r1 = np.abs(V[:, k].real)
    r1 /= r1.sum()
    r, sums, deltas, done = ora.pagerank_converge(n, f.A_rp, f.A_col, f.A_val, ora.init_r(n, 1),
                                                  max_iters=2000, tol=1e-13, mode=mode, c=C)
    assert done < 2000 and deltas[-1] <= 1e-13 and (deltas[:-1] > 1e-13).all()
    assert np.abs(r / r.sum() - r1).sum() <= 1e-10
    if mode != "none":
        assert abs(w[k].real - 1.0) <= 1e-12              # stochastic: eigenvalue 1


@pytest.mark.parametrize("mode", ["uniform", "self"])
def test_converge_stochastic_modes_keep_sum(ora, mode):
    p, f = pipeline_matrix(ora, 12)
    n = p.n
    r, sums, deltas, done = ora.pagerank_converge(n, f.A_rp, f.A_col, f.A_val, ora.init_r(n, 5),
                                                  max_iters=30, tol=-1.0, mode=mode, c=C)
    assert done == 30
    assert np.abs(sums / sums[0] - 1).max() <= 1e-13


def test_converge_none_sum_recurrence(ora):
    # Without an adjustment each step loses c * (mass on dangling vertices).
    p, f = pipeline_matrix(ora, 11)
    n = p.n
    dangling = np.diff(f.A_rp) == 0
    r = ora.init_r(n, 6)
    for k in range(4):
        r1, sums, _, done = ora.pagerank_converge(n, f.A_rp, f.A_col, f.A_val, r, max_iters=1,
                                                  tol=-1.0, mode="none", c=C)
        want = r.sum() - C * r[dangling].sum()
        assert done == 1 and abs(sums[1] - want) <= 1e-13 * want
        r = r1


def test_converge_none_is_the_benchmark_iteration(ora):
    # With a test that never passes, mode "none" runs exactly the fixed
    # iterations of the benchmark's K3.
    p, f = pipeline_matrix(ora, 10)
    n = p.n
    r0 = ora.init_r(n, 9)
    want, wsums = ora.pagerank(n, f.A_rp, f.A_col, f.A_val, r0, iters=20, c=C)
    r, sums, deltas, done = ora.pagerank_converge(n, f.A_rp, f.A_col, f.A_val, r0, max_iters=20,
                                                  tol=-1.0, mode="none", c=C)
    assert done == 20 and np.array_equal(r, want) and np.array_equal(sums, wsums)
    r, sums, deltas, done = ora.pagerank_converge(n, f.A_rp, f.A_col, f.A_val, r0, max_iters=0,
                                                  tol=1.0, mode="none", c=C)
    assert done == 0 and np.array_equal(r, r0) and deltas.size == 0


@pytest.mark.parametrize("mode", ["none", "uniform", "self"])
def test_converge_closed_form_permutation(ora, mode):
    # A permutation matrix has no empty row, so every mode is the same:
    # r_k = c^k r0 P^k + (1 - c^k) s0/N, sum(r_k) = s0, and delta_k is the
    # L1 norm of r_{k+1} - r_k over s0.  The run stops after the first k
    # with delta_k <= tol.
    n = 1000
    perm = np.random.default_rng(6).permutation(n)
    rp = np.arange(n + 1, dtype=np.int64)
    col = perm.astype(np.int32)
    val = np.ones(n)
    r0 = ora.init_r(n, 12)
    s0 = r0.sum()
    xs, x = [r0], r0
    for k in range(200):
        y = np.empty(n)
        y[perm] = x
        x = y
        xs.append(x)
    rk = [C**k * xs[k] + (1 - C**k) * s0 / n for k in range(201)]
    want_d = np.array([np.abs(rk[k + 1] - rk[k]).sum() / s0 for k in range(200)])
    tol = float(np.sqrt(want_d[60] * want_d[61]))       # between two iterates, far from both
    stop = int(np.argmax(want_d <= tol)) + 1
    r, sums, deltas, done = ora.pagerank_converge(n, rp, col, val, r0, max_iters=200, tol=tol,
                                                  mode=mode, c=C)
    assert done == stop == 62
    assert np.abs(deltas / want_d[:done] - 1).max() <= 1e-9
    assert relL1(r, rk[done]) <= 1e-14
    assert np.abs(sums / s0 - 1).max() <= 1e-14


def test_converge_closed_form_zero_matrix(ora):
    # A = 0: every vertex dangling.
    n = 777
    rp = np.zeros(n + 1, np.int64)
    z32, z = np.zeros(0, np.int32), np.zeros(0)
    r0 = ora.init_r(n, 13)
    s0 = r0.sum()
    d0 = np.abs(1.0 / n - r0 / s0).sum()
    # none: r_k = (1-c)^k s0/N (uniform from the first step), so delta_0 is
    # the distance of r0/s0 from uniform and delta_1 vanishes.
    r, sums, deltas, done = ora.pagerank_converge(n, rp, z32, z, r0, 50, 1e-12, "none", C)
    assert done == 2 and abs(deltas[0] / d0 - 1) <= 1e-12 and deltas[1] <= 1e-15
    assert np.abs(r / ((1 - C)**2 * s0 / n) - 1).max() <= 1e-13
    # uniform: all mass is respread, r_k = s0/N.
    r, sums, deltas, done = ora.pagerank_converge(n, rp, z32, z, r0, 50, 1e-12, "uniform", C)
    assert done == 2 and abs(deltas[0] / d0 - 1) <= 1e-12
    assert np.abs(r / (s0 / n) - 1).max() <= 1e-13 and np.abs(sums / s0 - 1).max() <= 1e-14
    # self: A = I, r_k = c^k r0 + (1 - c^k) s0/N, delta_k = c^k (1-c) d0.
    r, sums, deltas, done = ora.pagerank_converge(n, rp, z32, z, r0, 30, -1.0, "self", C)
    k = np.arange(30)
    assert done == 30 and np.abs(deltas / (C**k * (1 - C) * d0) - 1).max() <= 1e-11
    assert relL1(r, C**30 * r0 + (1 - C**30) * s0 / n) <= 1e-14
