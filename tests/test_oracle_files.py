"""Pins for the oracle's edge-file codec (Sec. IV.A-C: one edge per line,
the two labels as decimal strings separated by a tab, a newline after each
edge).  Formatting is checked against Python's own decimal formatting,
parsing against Python's int() on each field and by round trip; malformed
text of every kind the grammar excludes is rejected.
"""
import numpy as np
import pytest

from paper_1603_01876_amd import workloads


def py_format(u, v) -> bytes:
    return "".join(f"{a}\t{b}\n" for a, b in zip(u.tolist(), v.tolist())).encode()


def py_parse(text: bytes):
    lines = text.decode().split("\n")
    if lines and lines[-1] == "":
        lines = lines[:-1]
    pairs = [ln.split("\t") for ln in lines]
    return (np.array([int(a) for a, _ in pairs], np.int64),
            np.array([int(b) for _, b in pairs], np.int64))


@pytest.mark.parametrize("scale,m", [(1, 0), (1, 1), (4, 100), (30, 1000), (12, 5000)])
def test_format_matches_python(ora, scale, m):
    rng = np.random.default_rng(scale + m)
    n = 1 << scale
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    if m:
        u[0], v[0] = n - 1, 0          # longest and shortest labels
    text = ora.tsv_format(u, v)
    assert text == py_format(u, v)
    pu, pv = py_parse(text)
    assert np.array_equal(pu, u) and np.array_equal(pv, v)


def test_parse_round_trip_generated_graph(ora):
    p = ora.Kron(**workloads.pipeline(10).as_dict())
    u, v = ora.generate(p)
    text = ora.tsv_format(u, v)
    pu, pv = ora.tsv_parse(10, text)
    assert np.array_equal(pu, u) and np.array_equal(pv, v)
    # the last newline may be missing; an empty text has no edges
    pu, pv = ora.tsv_parse(10, text[:-1])
    assert np.array_equal(pu, u) and np.array_equal(pv, v)
    pu, pv = ora.tsv_parse(10, b"")
    assert pu.size == 0 and pv.size == 0


def test_parse_matches_python_int(ora):
    text = b"007\t0\n1023\t99\n0\t0"
    pu, pv = ora.tsv_parse(10, text)
    wu, wv = py_parse(text)
    assert np.array_equal(pu, wu) and np.array_equal(pv, wv)


@pytest.mark.parametrize("bad", [b"1\t2\n\n", b"\n", b"1 2\n", b"1\t2\t3\n", b"1\n", b"1\t\n",
                                 b"\t2\n", b"-1\t2\n", b"+1\t2\n", b"1\t2\r\n", b"1\t1024\n",
                                 b"1024\t1\n", b"1\t2\nx", b"12345678901234567890\t1\n"])
def test_parse_rejects_malformed(ora, bad):
    with pytest.raises(RuntimeError):
        ora.tsv_parse(10, bad)


def test_parse_respects_capacity(ora):
    text = b"1\t2\n3\t4\n"
    with pytest.raises(RuntimeError):
        ora.tsv_parse(10, text, cap=1)
    pu, _ = ora.tsv_parse(10, text, cap=2)
    assert pu.tolist() == [1, 3]
