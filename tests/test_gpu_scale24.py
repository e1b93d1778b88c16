"""Precision form at S = 24 (N = 2^24, M = 2^28): the whole GPU pipeline in
FP64 and FP32 against the FP64 oracle on the same seed.

K0, K1 and K2 must match the oracle bit for bit over their full arrays
(edges, sorted edges, d_in, d_out, nnz, CSR(A^T) with FP64 and FP32 values,
the row form CSR(A)), compared as digests against the values the oracle
wrote into tests/golden/kron_s24_pipeline.json; the initial vectors must
match bit for bit; K3's r_20 must reach the oracle's within 1e-12 relative
L1 in FP64 and 1e-5 in FP32, in every launch configuration the library
offers (default, one pass, column slabs, with and without relabelling).
"""
import numpy as np
import pytest
import torch

import pipeline_golden as pg
from paper_1603_01876_amd import native as pp
from paper_1603_01876_amd import workloads

pytestmark = pytest.mark.gpu

S = 24
TAG = "scale24"


@pytest.fixture(scope="module")
def run():
    assert torch.cuda.is_available()
    g = pg.load(S)
    spec = workloads.pipeline(S)
    assert (spec.n, spec.m, spec.seed) == (g["vertices"], g["edges"], g["seed"])
    pg.say(TAG, "GPU K0-K2")
    u, v = pp.generate(spec)
    us, vs = pp.sort(S, u, v)
    AT64, d_in, d_out = pp.filter(S, us, vs, "f64")
    AT32, _, _ = pp.filter(S, us, vs, "f32", degrees=False)
    torch.cuda.synchronize()
    state = dict(g=g, spec=spec, u=u, v=v, us=us, vs=vs, AT64=AT64, AT32=AT32, d_in=d_in,
                 d_out=d_out)
    yield state
    state.clear()
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_edges_and_sorted_edges(run):
    d = run["g"]["digest"]
    assert pg.gpu_digest(run["u"]) == d["u"]
    assert pg.gpu_digest(run["v"]) == d["v"]
    assert pg.gpu_digest(run["us"]) == d["u_sorted"]
    assert pg.gpu_digest(run["vs"]) == d["v_sorted"]


@pytest.mark.timeout(600)
def test_filter_full_arrays(run):
    g, d = run["g"], run["g"]["digest"]
    AT64, AT32 = run["AT64"], run["AT32"]
    assert AT64.nnz == g["nnz"] and AT32.nnz == g["nnz"]
    assert int(run["d_in"].max()) == g["max_in_degree"]
    assert pg.gpu_digest(run["d_in"]) == d["d_in"]
    assert pg.gpu_digest(run["d_out"]) == d["d_out"]
    assert pg.gpu_digest(AT64.row_ptr) == d["AT_row_ptr"]
    assert pg.gpu_digest(AT32.row_ptr) == d["AT_row_ptr"]
    assert pg.gpu_digest(AT64.col, AT64.nnz) == d["AT_col"]
    assert pg.gpu_digest(AT32.col, AT32.nnz) == d["AT_col"]
    assert pg.gpu_digest(AT64.val, AT64.nnz) == d["AT_val_f64"]
    assert pg.gpu_digest(AT32.val, AT32.nnz) == d["AT_val_f32"]


@pytest.mark.timeout(600)
def test_row_form_full_arrays(run):
    d = run["g"]["digest"]
    A = pp.transpose(run["AT64"])
    assert A.nnz == run["g"]["nnz"]
    assert pg.gpu_digest(A.row_ptr) == d["A_row_ptr"]
    assert pg.gpu_digest(A.col, A.nnz) == d["A_col"]
    assert pg.gpu_digest(A.val, A.nnz) == d["A_val_f64"]
    del A
    torch.cuda.empty_cache()


def test_initial_vectors(run):
    d, n = run["g"]["digest"], run["spec"].n
    assert pg.gpu_digest(pp.init_r(n, run["g"]["r0_seed"], "f64")) == d["r0_f64"]
    assert pg.gpu_digest(pp.init_r(n, run["g"]["r0_seed"], "f32")) == d["r0_f32"]


@pytest.fixture(scope="module")
def oracle_r20(run):
    # Only a matrix equal to the oracle's (all three digests) may feed the
    # oracle's K3.
    d, AT64 = run["g"]["digest"], run["AT64"]
    assert pg.gpu_digest(AT64.row_ptr) == d["AT_row_ptr"]
    assert pg.gpu_digest(AT64.col, AT64.nnz) == d["AT_col"]
    assert pg.gpu_digest(AT64.val, AT64.nnz) == d["AT_val_f64"]
    r, sums = pg.oracle_k3(AT64, run["g"], TAG)
    assert f"0x{pg.oracle.digest(r):016x}" == d["r20_f64"]
    assert [float(x).hex() for x in sums] == run["g"]["sums"]
    return r, sums


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pagerank_every_config(run, oracle_r20, dtype):
    want_r, want_sums = oracle_r20
    AT = run["AT64"] if dtype == "f64" else run["AT32"]
    ws = torch.empty(pp.workspace_bytes(pp.K3, AT.n, AT.nnz, dtype), dtype=torch.uint8,
                     device="cuda")
    errs = pg.check_k3_configs(AT, dtype, run["d_out"], want_r, want_sums, run["g"], ws, TAG)
    assert max(errs.values()) <= pg.TOL[dtype]
