"""Pins for the oracle tooling that full-size parity rests on.

- ppo_digest against a big-integer evaluation of its definition, its
  order independence and its additivity over pieces of an array, and that a
  single changed element or swapped pair changes it;
- ppo_sum_r against the sums ppo_pagerank reports and an exactly rounded
  sum (math.fsum);
- the row-block K2 (filter_blocks: ppo_filter_rows over contiguous blocks of
  rows of A^T) against the whole-matrix ppo_filter;
- the row-split K3 (pagerank_rows: ppo_sum_r + ppo_step_rows over blocks of
  rows of A^T) against ppo_pagerank on CSR(A), bit for bit.
"""
import math

import numpy as np
import pytest

from paper_1603_01876_amd import workloads

M64 = (1 << 64) - 1
GOLD = 0x9E3779B97F4A7C15


def py_mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def py_digest(x, index0=0):
    bits = np.ascontiguousarray(x).view(np.uint32 if x.dtype.itemsize == 4 else np.uint64)
    d = 0
    for i, b in enumerate(bits.tolist()):
        d = (d + py_mix(int(b) ^ py_mix((index0 + i + GOLD) & M64))) & M64
    return d


@pytest.mark.parametrize("dtype", [np.int32, np.int64, np.float32, np.float64])
def test_digest_matches_definition(ora, dtype):
    rng = np.random.default_rng(3)
    if np.issubdtype(dtype, np.integer):
        x = rng.integers(0, 2**31 - 1, 777).astype(dtype)
    else:
        x = rng.random(777).astype(dtype)
    assert ora.digest(x) == py_digest(x)
    assert ora.digest(x[100:], index0=100) == py_digest(x[100:], 100)
    assert ora.digest(x[:0]) == 0


def test_digest_mix_is_splitmix64_output(ora):
    # mix is SplitMix64's output function: from state 0 the generator's first
    # output is mix(gamma) = 0xE220A8397B1DCDAF (published test vector).  One
    # element at index 0 contributes mix(x ^ mix(gamma)), so x = that output
    # gives mix(0) = 0, and x = output ^ gamma gives mix(gamma) itself.
    first = 0xE220A8397B1DCDAF
    assert ora.digest(np.array([first], np.uint64)) == 0
    assert ora.digest(np.array([first ^ GOLD], np.uint64)) == first


def test_digest_additive_and_order_free(ora):
    rng = np.random.default_rng(5)
    x = rng.integers(0, 1 << 40, 10_000).astype(np.int64)
    whole = ora.digest(x)
    parts = [ora.digest(x[a:b], index0=a) for a, b in [(0, 1), (1, 4000), (4000, 10_000)]]
    assert ora.digest_add(*parts) == whole
    # Pieces taken in another order give the same sum.
    assert ora.digest_add(*reversed(parts)) == whole
    # Any single change, or swapping two different elements, changes it.
    y = x.copy()
    y[1234] ^= 1
    assert ora.digest(y) != whole
    y = x.copy()
    y[[10, 20]] = y[[20, 10]]
    assert ora.digest(y) != whole


def test_digest_int32_equals_int64_of_same_values(ora):
    # Non-negative labels digest the same whether stored in 32 or 64 bits,
    # so int32 GPU arrays compare with the oracle's int64 ones.
    x = np.arange(0, 5000, 3, dtype=np.int64)
    assert ora.digest(x) == ora.digest(x.astype(np.int32))


def test_sum_r_is_pagerank_sum_and_near_exact(ora):
    rng = np.random.default_rng(9)
    r = rng.random(100_000) * np.exp(rng.normal(0, 8, 100_000))
    s = ora.sum_r(r)
    exact = math.fsum(r)
    assert abs(s - exact) <= np.spacing(exact)
    # ppo_pagerank's sums[0] is sum(r_0) formed the same way.
    n = 64
    rp = np.zeros(n + 1, np.int64)
    _, sums = ora.pagerank(n, rp, np.zeros(0, np.int32), np.zeros(0), r[:n], 1)
    assert sums[0] == ora.sum_r(r[:n])


def kron_edges(ora, scale, seed=workloads.BASE_SEED):
    p = ora.Kron(**workloads.pipeline(scale, seed).as_dict())
    u, v = ora.generate(p)
    return ora.sort(scale, u, v)


@pytest.mark.parametrize("scale,nblocks,threads", [(6, 1, 1), (10, 3, 1), (12, 7, 4),
                                                    (12, 64, 3)])
def test_filter_blocks_equals_filter(ora, scale, nblocks, threads):
    us, vs = kron_edges(ora, scale)
    f = ora.filter(scale, us, vs)
    rp, col, val, d_in, d_out, mx, nnz = ora.filter_blocks(scale, us, vs, nblocks, threads)
    assert nnz == f.nnz
    assert np.array_equal(rp, f.AT_rp)
    assert np.array_equal(col, f.AT_col)
    assert np.array_equal(val, f.AT_val)
    assert np.array_equal(d_in, f.d_in) and np.array_equal(d_out, f.d_out)
    assert mx == f.d_in.max()


@pytest.mark.parametrize("scale,threads,nblocks", [(8, 1, None), (12, 4, None), (12, 3, 17)])
def test_pagerank_rows_equals_pagerank(ora, scale, threads, nblocks):
    us, vs = kron_edges(ora, scale, seed=11)
    f = ora.filter(scale, us, vs)
    r0 = ora.init_r(f.n, 1603)
    want, wsums = ora.pagerank(f.n, f.A_rp, f.A_col, f.A_val, r0, 20, workloads.DAMPING)
    got, gsums = ora.pagerank_rows(f.n, f.AT_rp, f.AT_col, f.AT_val, r0, 20, workloads.DAMPING,
                                   threads=threads, nblocks=nblocks)
    assert np.array_equal(got, want)
    assert np.array_equal(gsums, wsums)


def test_pagerank_rows_zero_iterations_and_empty_matrix(ora):
    n = 33
    r0 = ora.init_r(n, 4)
    rp = np.zeros(n + 1, np.int64)
    r, s = ora.pagerank_rows(n, rp, np.zeros(0, np.int32), np.zeros(0), r0, 0)
    assert np.array_equal(r, r0) and s[0] == ora.sum_r(r0)
    r, s = ora.pagerank_rows(n, rp, np.zeros(0, np.int32), np.zeros(0), r0, 3, threads=2)
    want, ws = ora.pagerank(n, rp, np.zeros(0, np.int32), np.zeros(0), r0, 3)
    assert np.array_equal(r, want) and np.array_equal(s, ws)


@pytest.mark.parametrize("chunk,threads", [(1000, 3), (1 << 22, 1)])
def test_generate_parallel_equals_generate(ora, chunk, threads):
    p = ora.Kron(**workloads.pipeline(11, 77).as_dict())
    u, v = ora.generate(p)
    pu, pv = ora.generate_parallel(p, threads=threads, chunk=chunk)
    assert np.array_equal(u, pu) and np.array_equal(v, pv)
