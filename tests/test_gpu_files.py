"""GPU parity of the edge-file path (Sec. IV.A-C): text lines "u<TAB>v<LF>"
formatted and parsed on the GPU, files written and read through pinned
staging buffers, and the file-backed pipeline K0 -> files -> K1 -> files ->
K2.  Bytes and edges must equal the oracle's (pinned in test_oracle_files.py)
exactly; malformed text is rejected like the oracle rejects it.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1603_01876_amd import native as pp
from test_gpu_parity import dev, host, okron, spec

pytestmark = pytest.mark.gpu

MALFORMED = [b"1\t2\n\n", b"\n", b"1 2\n", b"1\t2\t3\n", b"1\n", b"1\t\n", b"\t2\n", b"-1\t2\n",
             b"+1\t2\n", b"1\t2\r\n", b"1\t1024\n", b"1024\t1\n", b"1\t2\nx",
             b"12345678901234567890\t1\n", b"1\t2\n" * 3 + b"1" * 40 + b"\t1\n"]


@pytest.fixture(autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def to_dev_text(b: bytes):
    t = torch.zeros(max(len(b), 16), dtype=torch.uint8)
    t[:len(b)] = torch.frombuffer(bytearray(b), dtype=torch.uint8) if b else t[:0]
    return t.cuda()


@pytest.mark.parametrize("scale", [1, 4, 10, 16])
@pytest.mark.parametrize("nsplit", [1, 3, 16])
def test_format_matches_oracle(scale, nsplit):
    s = spec(scale)
    u, v = pp.generate(s)
    text, split = pp.tsv_format(scale, u, v, nsplit=nsplit)
    ou, ov = oracle.generate(okron(s))
    want = oracle.tsv_format(ou, ov)
    got = bytes(host(text[:split[-1]]))
    assert got == want
    m = ou.size
    for k in range(nsplit + 1):
        L = m * k // nsplit
        assert split[k] == len(oracle.tsv_format(ou[:L], ov[:L])), k


def test_format_extremes_and_empty():
    n = 1 << 30
    u = np.array([n - 1, 0, 9, 10, 99, 100, 999999999, 1000000000], np.int64)
    v = u[::-1].copy()
    text, split = pp.tsv_format(30, dev(u), dev(v), nsplit=2)
    assert bytes(host(text[:split[-1]])) == oracle.tsv_format(u, v)
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    text, split = pp.tsv_format(10, empty, empty, nsplit=4)
    assert split == [0] * 5
    with pytest.raises(pp.PPError):                       # label outside [0, 2^10)
        pp.tsv_format(10, dev(np.array([1024])), dev(np.array([0])))
    with pytest.raises(pp.PPError):                       # text longer than the buffer
        pp.tsv_format(10, dev(np.arange(100)), dev(np.arange(100)),
                      text=torch.empty(64, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("scale", [8, 14])
def test_parse_matches_oracle(scale):
    s = spec(scale)
    ou, ov = oracle.generate(okron(s))
    text = oracle.tsv_format(ou, ov)
    for t in (text, text[:-1]):                           # last newline optional
        gu, gv = pp.tsv_parse(scale, to_dev_text(t), len(t), cap=ou.size)
        assert np.array_equal(host(gu), ou) and np.array_equal(host(gv), ov)


def test_parse_edge_cases():
    gu, gv = pp.tsv_parse(10, to_dev_text(b""), 0, cap=4)
    assert gu.numel() == 0
    t = b"007\t0\n1023\t99\n0\t0"
    gu, gv = pp.tsv_parse(10, to_dev_text(t), len(t), cap=3)
    wu, wv = oracle.tsv_parse(10, t)
    assert np.array_equal(host(gu), wu) and np.array_equal(host(gv), wv)
    with pytest.raises(pp.PPError):                       # more lines than capacity
        pp.tsv_parse(10, to_dev_text(t), len(t), cap=2)
    # lines crossing the 64-byte thread windows and 16 KiB blocks
    rng = np.random.default_rng(3)
    u = rng.integers(0, 1 << 30, 5000)
    v = rng.integers(0, 1 << 30, 5000)
    t = oracle.tsv_format(u, v)
    gu, gv = pp.tsv_parse(30, to_dev_text(t), len(t), cap=5000)
    assert np.array_equal(host(gu), u) and np.array_equal(host(gv), v)


@pytest.mark.parametrize("bad", MALFORMED)
def test_parse_rejects_malformed(bad):
    with pytest.raises(RuntimeError):
        oracle.tsv_parse(10, bad)
    with pytest.raises(pp.PPError) as e:
        pp.tsv_parse(10, to_dev_text(bad), len(bad), cap=100)
    assert e.value.status == pp.PP_EINVAL


def test_files_round_trip(tmp_path):
    s = spec(14)
    u, v = pp.generate(s)
    text, split = pp.tsv_format(14, u, v, nsplit=5)
    prefix = str(tmp_path / "edges")
    pp.write_text_files(prefix, text, split)
    ou, ov = oracle.generate(okron(s))
    want = oracle.tsv_format(ou, ov)
    for k in range(5):
        with open(f"{prefix}.{k:05d}", "rb") as f:
            assert f.read() == want[split[k]:split[k + 1]]
    back = torch.empty(split[-1] + 16, dtype=torch.uint8, device="cuda")
    nb = pp.read_text_files(prefix, 5, back)
    assert nb == split[-1]
    gu, gv = pp.tsv_parse(14, back, nb, cap=u.numel())
    assert torch.equal(gu, u) and torch.equal(gv, v)
    with pytest.raises(pp.PPError):                       # a file that is not there
        pp.read_text_files(prefix, 6, back)
    with pytest.raises(pp.PPError):                       # capacity too small
        pp.read_text_files(prefix, 5, back[:100])


def test_file_backed_pipeline(tmp_path):
    # K0 writes files; K1 reads them, sorts, writes; K2 reads those.
    scale = 12
    s = spec(scale)
    u, v = pp.generate(s)
    text, split = pp.tsv_format(scale, u, v, nsplit=3)
    pp.write_text_files(str(tmp_path / "k0"), text, split)
    nb = pp.read_text_files(str(tmp_path / "k0"), 3, text)
    u1, v1 = pp.tsv_parse(scale, text, nb, cap=u.numel())
    us, vs = pp.sort(scale, u1, v1)
    text2, split2 = pp.tsv_format(scale, us, vs, nsplit=4)
    pp.write_text_files(str(tmp_path / "k1"), text2, split2)
    nb2 = pp.read_text_files(str(tmp_path / "k1"), 4, text2)
    u2, v2 = pp.tsv_parse(scale, text2, nb2, cap=u.numel())
    AT, d_in, d_out = pp.filter(scale, u2, v2, "f64")
    ou, ov = oracle.generate(okron(s))
    f = oracle.filter(scale, *oracle.sort(scale, ou, ov))
    z = AT.nnz
    assert z == f.nnz
    assert np.array_equal(host(AT.row_ptr), f.AT_rp)
    assert np.array_equal(host(AT.col[:z]), f.AT_col)
    assert np.array_equal(host(AT.val[:z]), f.AT_val)
    assert np.array_equal(host(d_out), f.d_out)


def test_files_many_chunks_per_worker(tmp_path):
    # About 0.5 GB of text in 17 files: every reader thread handles several
    # files of more than one staging chunk each, so its two staging buffers
    # are reused across chunks and files; the bytes read back must be exact.
    scale = 21
    s = spec(scale)
    u, v = pp.generate(s)
    text, split = pp.tsv_format(scale, u, v, nsplit=17)
    assert split[-1] > 17 * (24 << 20)
    prefix = str(tmp_path / "big")
    pp.write_text_files(prefix, text, split, sync=False)
    back = torch.empty_like(text)
    for _ in range(2):                                    # the pooled workers again
        back.zero_()
        nb = pp.read_text_files(prefix, 17, back)
        assert nb == split[-1]
        assert torch.equal(back[:nb], text[:nb])
        gu, gv = pp.tsv_parse(scale, back, nb, cap=u.numel())
        assert torch.equal(gu, u) and torch.equal(gv, v)


def test_codec_round_trip_beyond_4gib():
    # S = 24: 2^28 edges, about 4.4 GB of text, so byte offsets pass 2^32
    # (64-bit block offsets in both directions).
    scale = 24
    s = spec(scale)
    u, v = pp.generate(s)
    text, split = pp.tsv_format(scale, u, v, nsplit=7)
    nb = split[-1]
    assert nb > (1 << 32)
    # each part starts with the oracle's line of its first edge
    m = u.numel()
    for k in range(7):
        e = m * k // 7
        line = oracle.tsv_format(host(u[e:e + 1]), host(v[e:e + 1]))
        assert bytes(host(text[split[k]:split[k] + len(line)])) == line
    last = oracle.tsv_format(host(u[-1:]), host(v[-1:]))
    assert bytes(host(text[nb - len(last):nb])) == last
    gu, gv = pp.tsv_parse(scale, text, nb, cap=u.numel())
    assert torch.equal(gu, u) and torch.equal(gv, v)
