"""Host-side logic of bench.py (no GPU needed): the algorithmic bytes the
roofline is priced with, the gating of the measured HBM traffic by the
committed counter summary, and the one-GPU contract of the command line.
"""
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SUMMARY = os.path.join(ROOT, "profiles", "k3_spmv_kron_s26_f32_counters.md")
SOURCE = os.path.join(ROOT, "paper_1603_01876_amd", "csrc", "k3_pagerank.hip")


def summary_fields(dtype="f32"):
    out = {}
    for line in open(os.path.join(ROOT, "profiles", f"k3_spmv_kron_s26_{dtype}_counters.md")):
        if ":" in line:
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def test_spmv_bytes_match_the_pull_form_counts():
    # FP32: 8Z + 12N + 4; FP64: 12Z + 20N + 4 (row pointers, columns, values,
    # x read once, y written once).
    for n, z in [(1, 0), (1024, 11614), (1 << 26, 1051749331)]:
        assert bench.spmv_bytes(n, z, "f32") == 8 * z + 12 * n + 4
        assert bench.spmv_bytes(n, z, "f64") == 12 * z + 20 * n + 4


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_measured_traffic_follows_the_committed_summary(dtype):
    f = summary_fields(dtype)
    other_dt = "f64" if dtype == "f32" else "f32"
    cfg = tuple(int(x) for x in f["k3_config"].split(","))
    relabel = f["relabel"] == "1"
    got = bench.measured_traffic(26, dtype, cfg, relabel)
    src_sha = hashlib.sha256(open(SOURCE, "rb").read()).hexdigest()
    if f["kernel_source_sha256"] != src_sha:
        assert got is None          # stale summary: no traffic is reported
        return
    want = (float(f["fetch_bytes_per_launch"]) + float(f["write_bytes_per_launch"])) / 1e9
    assert got["traffic"] == pytest.approx(want, rel=1e-12)
    l2 = got["l2"]
    assert l2["requests_per_s"] == pytest.approx(
        float(f["spmv_l2_read_requests_per_launch"]) / (float(f["spmv_launch_us"]) * 1e-6))
    # another launch configuration, relabelling choice, scale or dtype: none
    other = (cfg[0], cfg[1], cfg[2] + 1) + cfg[3:]
    assert bench.measured_traffic(26, dtype, other, relabel) is None
    assert bench.measured_traffic(26, dtype, cfg, not relabel) is None
    assert bench.measured_traffic(25, dtype, cfg, relabel) is None
    assert bench.measured_traffic(26, other_dt, cfg, relabel) is None
    scaled_off = cfg[:3] + (0,) + cfg[4:]
    assert bench.measured_traffic(26, dtype, scaled_off, relabel) is None


def test_measured_traffic_ignores_a_summary_of_other_source(tmp_path, monkeypatch):
    # A copy of the tree whose kernel source differs from the one profiled.
    root = tmp_path / "tree"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_1603_01876_amd" / "csrc").mkdir(parents=True)
    shutil.copy(SUMMARY, root / "profiles")
    (root / "paper_1603_01876_amd" / "csrc" / "k3_pagerank.hip").write_text("// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    f = summary_fields()
    cfg = tuple(int(x) for x in f["k3_config"].split(","))
    assert bench.measured_traffic(26, "f32", cfg, f["relabel"] == "1") is None


def test_spmv_label_names_the_timed_launches():
    assert bench.spmv_label((16, 0, 19), "f32") == (
        "segmented SpMV iteration, slabs of 2^19 columns: k_spmv<float,16,raw> + "
        "k_fix_raw<float> + k_seg_combine<float> + k_sum_blocks")
    assert bench.spmv_label((8, 0, 0), "f64") == "k_spmv<double,8> + k_finish<double>"


def test_scaled_form_bytes_and_label():
    # Degree-scaled form: row pointers, columns, one count byte per entry,
    # the gathered vector read and the next one written, the out-degrees.
    lay = {"relabelled": True, "segmented": True, "scaled": True, "packed": False}
    n, z = 1 << 26, 1051749331
    assert bench.form_bytes(n, z, "f64", lay) == 4 * (n + 1) + 5 * z + 16 * n + 4 * n
    assert bench.form_bytes(n, z, "f32", lay) == 4 * (n + 1) + 5 * z + 8 * n + 4 * n
    assert bench.form_bytes(n, z, "f64", dict(lay, scaled=False)) is None
    assert bench.form_bytes(n, z, "f64", None) is None
    assert bench.spmv_label((16, 0, 18, 1), "f64", lay) == (
        "segmented SpMV iteration, slabs of 2^18 columns (degree-scaled form: entries stored as "
        "counts): k_spmv<double,16,raw,uint8> + k_fix_raw<double> + k_seg_combine<double> + "
        "k_sum_blocks")
    # Packed with the column inside the slab: 4 bytes per entry.
    pk = dict(lay, packed=True)
    assert bench.form_bytes(n, z, "f64", pk) == 4 * (n + 1) + 4 * z + 16 * n + 4 * n
    assert bench.spmv_label((16, 0, 18, 1), "f64", pk) == (
        "segmented SpMV iteration, slabs of 2^18 columns (degree-scaled form: each entry one "
        "4-byte word, column inside the slab and count): k_spmv<double,16,raw,packed> + "
        "k_fix_raw<double> + k_seg_combine<double> + k_sum_blocks")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert not any(line.startswith("{") for line in r.stdout.splitlines())   # no result line
