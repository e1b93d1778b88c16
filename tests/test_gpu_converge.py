"""GPU parity of K3 run to a convergence test (pp_pagerank_converge).

Each step is the benchmark's iteration plus a dangling-vertex term ("none",
"uniform": a dangling vertex's damped mass spread evenly, "self": A(i,i) = 1
in every empty row of A), followed by the normed L1 difference of the two
iterates, each divided by its sum; the run stops after the first difference
<= tol.  Against the oracle (pinned in test_oracle_k3.py): the same number
of iterations, r within the K3 tolerances (1e-12 FP64, 1e-5 FP32 relative
L1), sum(r_k) and the differences along the way.  Tolerances are placed
between two consecutive oracle differences (at least a factor ~1/c apart), so the
stopping iteration is decided far from rounding.  Covered: the one-pass
and the column-segmented iteration, with and without relabelling, closed
forms (A = 0, a permutation), max_iters = 0, tests that never pass, and
reproducibility.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1603_01876_amd import native as pp
from paper_1603_01876_amd import workloads
from test_gpu_parity import TOL, host, okron, rel_l1, spec

pytestmark = pytest.mark.gpu

C = workloads.DAMPING
MODES = ["none", "uniform", "self"]


@pytest.fixture(autouse=True)
def restore_config():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield
    pp.set_k3_config()


def kron_matrix(scale):
    ou, ov = oracle.generate(okron(spec(scale)))
    ous, ovs = oracle.sort(scale, ou, ov)
    return oracle.filter(scale, ous, ovs)


def oracle_run(n, rp, col, val, mode, max_iters, tol, seed=7):
    return oracle.pagerank_converge(n, rp, col, val, oracle.init_r(n, seed), max_iters, tol,
                                    mode, C)


def pick_tol(deltas, target):
    """A tolerance between two consecutive differences around `target`."""
    k = int(np.argmax(deltas <= target))
    assert deltas[k] <= target and k > 0
    return float(np.sqrt(deltas[k - 1] * deltas[k])), k + 1


def gpu_run(AT, n, dtype, max_iters, tol, mode, d_out, weights=None, slab=None, seed=7):
    if slab is not None:
        pp.set_k3_config(8, 0, slab)
    r = pp.init_r(n, seed, dtype)
    dt = None if d_out is None else torch.as_tensor(np.asarray(d_out)).to(torch.int32).cuda()
    w = None if weights is None else torch.as_tensor(np.asarray(weights)).to(torch.int32).cuda()
    sums, deltas, k = pp.pagerank_converge(AT, r, max_iters, tol, mode, d_out=dt, c=C, weights=w)
    return host(r), host(sums), host(deltas), k


def check_against_oracle(n, rp, col, val, d_out, dtype, mode, target, weights=None, slab=None,
                         max_iters=400):
    _, _, all_d, _ = oracle_run(n, rp, col, val, mode, max_iters, -1.0)
    tol, stop = pick_tol(all_d, target)
    want, wsums, wdeltas, k = oracle_run(n, rp, col, val, mode, max_iters, tol)
    assert k == stop
    trp, tcol, tval = oracle.transpose_csr(n, rp, col, val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, dtype)
    got, sums, deltas, kg = gpu_run(AT, n, dtype, max_iters, tol, mode, d_out, weights, slab)
    assert kg == k, (kg, k)
    assert rel_l1(got, want) <= TOL[dtype], rel_l1(got, want)
    assert np.abs(sums / wsums - 1).max() <= TOL[dtype]
    # differences: each term is a difference of nearly equal values, so
    # rounding of the iterates (FP64 ~1e-16, FP32 ~1e-7 absolute in the
    # normalised sum) shows relative to delta itself
    dtol = 1e-5 if dtype == "f64" else 2e-2
    assert np.abs(deltas / wdeltas - 1).max() <= dtol
    return k


@pytest.mark.parametrize("dtype,target", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("scale", [10, 14])
def test_converge_kronecker(scale, mode, dtype, target):
    f = kron_matrix(scale)
    k = check_against_oracle(f.n, f.A_rp, f.A_col, f.A_val, f.d_out, dtype, mode, target)
    assert k > (30 if mode == "self" else 4)


@pytest.mark.parametrize("dtype,target", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("mode", MODES)
def test_converge_relabelled_and_segmented(mode, dtype, target):
    # Dangling flags follow the relabelling; slabs of 2^8 columns at S = 14
    # run the segmented iteration, 0 the one-pass one.
    f = kron_matrix(14)
    for slab in (8, 0):
        check_against_oracle(f.n, f.A_rp, f.A_col, f.A_val, f.d_out, dtype, mode, target,
                             weights=f.d_out, slab=slab)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_converge_zero_matrix_closed_forms(dtype):
    n = 777
    AT = pp.CSR.from_arrays(n, np.zeros(n + 1), np.zeros(0, np.int32), np.zeros(0), dtype)
    d_out = np.zeros(n, np.int32)
    r0 = oracle.init_r(n, 7)
    s0 = r0.sum()
    d0 = np.abs(1.0 / n - r0 / s0).sum()
    for mode in ("none", "uniform"):       # uniform after one step, then stationary
        r, sums, deltas, k = gpu_run(AT, n, dtype, 50, 1e-6, mode, d_out)
        assert k == 2 and abs(deltas[0] / d0 - 1) <= 1e-6 and deltas[1] <= 1e-6
        want = (1 - C)**2 * s0 / n if mode == "none" else s0 / n
        assert np.abs(r / want - 1).max() <= TOL[dtype]
    # self: A = I, r_k = c^k r0 + (1 - c^k) s0/N, delta_k = c^k (1-c) d0
    r, sums, deltas, k = gpu_run(AT, n, dtype, 30, -1.0, "self", d_out)
    kk = np.arange(30)
    assert k == 30
    assert np.abs(deltas / (C**kk * (1 - C) * d0) - 1).max() <= (1e-10 if dtype == "f64" else 1e-3)
    assert rel_l1(r, C**30 * r0 + (1 - C**30) * s0 / n) <= TOL[dtype]
    assert np.abs(sums / s0 - 1).max() <= TOL[dtype]


@pytest.mark.parametrize("mode", MODES)
def test_converge_permutation_closed_form(mode):
    # No empty row: every mode is r_k = c^k r0 P^k + (1 - c^k) s0/N.
    n = 5000
    perm = np.random.default_rng(6).permutation(n)
    rp = np.arange(n + 1, dtype=np.int64)
    col = perm.astype(np.int32)
    val = np.ones(n)
    r0 = oracle.init_r(n, 7)
    s0 = r0.sum()
    xs, x = [r0], r0
    for _ in range(200):
        y = np.empty(n)
        y[perm] = x
        x = y
        xs.append(x)
    rk = [C**k * xs[k] + (1 - C**k) * s0 / n for k in range(201)]
    want_d = np.array([np.abs(rk[k + 1] - rk[k]).sum() / s0 for k in range(200)])
    tol, stop = pick_tol(want_d, 1e-8)
    trp, tcol, tval = oracle.transpose_csr(n, rp, col, val)
    AT = pp.CSR.from_arrays(n, trp, tcol, tval, "f64")
    r, sums, deltas, k = gpu_run(AT, n, "f64", 200, tol, mode, np.ones(n, np.int32))
    assert k == stop
    assert np.abs(deltas / want_d[:k] - 1).max() <= 1e-6
    assert rel_l1(r, rk[k]) <= 1e-12 and np.abs(sums / s0 - 1).max() <= 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_converge_edges(dtype):
    f = kron_matrix(10)
    AT = pp.CSR.from_arrays(f.n, f.AT_rp, f.AT_col, f.AT_val, dtype)
    r0 = host(pp.init_r(f.n, 7, dtype))
    # max_iters = 0: nothing runs, r unchanged (also through the relabelling)
    r, sums, deltas, k = gpu_run(AT, f.n, dtype, 0, 1.0, "uniform", f.d_out, weights=f.d_out)
    assert k == 0 and r.tobytes() == r0.tobytes() and deltas.size == 0 and sums.size == 1
    # a test that never passes runs max_iters; mode "none" is then the
    # benchmark's iteration (sums of y formed in another fixed order)
    r, sums, deltas, k = gpu_run(AT, f.n, dtype, 20, -1.0, "none", None)
    rb = pp.init_r(f.n, 7, dtype)
    bsums = host(pp.pagerank(AT, rb, iters=20, c=C))
    assert k == 20 and rel_l1(r, host(rb)) <= TOL[dtype]
    assert np.abs(sums / bsums - 1).max() <= TOL[dtype]
    # tol = NaN never passes either
    _, _, _, k = gpu_run(AT, f.n, dtype, 7, float("nan"), "self", f.d_out)
    assert k == 7


def test_converge_is_reproducible():
    f = kron_matrix(14)
    AT = pp.CSR.from_arrays(f.n, f.AT_rp, f.AT_col, f.AT_val, "f32")
    runs = [gpu_run(AT, f.n, "f32", 200, 1e-6, "uniform", f.d_out, weights=f.d_out, slab=8)
            for _ in range(2)]
    assert runs[0][3] == runs[1][3]
    for a, b in zip(runs[0][:3], runs[1][:3]):
        assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("mode", MODES)
def test_converge_eigenvector_check(mode):
    # Sec. IV.D's own validation, GPU against an eigensolver (no oracle in
    # between): the converged r / sum(r) is the leading eigenvector of
    # c*A.' + (1-c)/N, with the mode's dangling adjustment in A.
    f = kron_matrix(10)
    n = f.n
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(f.A_rp)), f.A_col] = f.A_val
    d = (np.diff(f.A_rp) == 0).astype(float)
    if mode == "uniform":
        A = A + np.outer(d, np.ones(n)) / n
    elif mode == "self":
        A = A + np.diag(d)
    w, V = np.linalg.eig(C * A.T + (1 - C) / n)
    r1 = np.abs(V[:, int(np.argmax(w.real))].real)
    r1 /= r1.sum()
    AT = pp.CSR.from_arrays(n, f.AT_rp, f.AT_col, f.AT_val, "f64")
    r, sums, deltas, k = gpu_run(AT, n, "f64", 2000, 1e-13, mode, f.d_out, weights=f.d_out)
    assert k < 2000
    assert np.abs(r / r.sum() - r1).sum() <= 1e-10
