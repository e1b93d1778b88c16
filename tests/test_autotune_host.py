"""Host-side logic of the K3 autotuner (no GPU needed): the candidate set,
the cache key, and a cache hit applying the stored configuration without
measuring anything.  The measuring path runs in the GPU tests.
"""
import json
from types import SimpleNamespace

from paper_1603_01876_amd import autotune
from paper_1603_01876_amd import native


def test_single_vector_candidates():
    plain = autotune.candidates(1)
    assert plain == [(8, 0, 0, False), (16, 0, 0, False), (16, 0, 18, False),
                     (16, 0, 19, False), (16, 0, 20, False)]
    both = autotune.candidates(1, (False, True))
    assert both[:5] == plain and [c[:3] for c in both[5:]] == [c[:3] for c in plain]
    assert all(c[3] for c in both[5:])


def test_spmm_lane_and_tile_candidates():
    # One pass with lanes = nextpow2(nrhs) or 64, then column tiles of 16 and
    # 8 right-hand sides where they are narrower than nrhs.
    assert autotune.candidates(32) == [(8, 32, 0, False, 0), (8, 64, 0, False, 0),
                                       (8, 0, 0, False, 16), (8, 0, 0, False, 8)]
    assert [c[1] for c in autotune.candidates(3)] == [4, 64]
    assert [c[4] for c in autotune.candidates(12)] == [0, 0, 8]
    assert autotune.candidates(64) == [(8, 64, 0, False, 0), (8, 0, 0, False, 16),
                                       (8, 0, 0, False, 8)]
    assert [c[1] for c in autotune.candidates(2, (False, True))] == [2, 2, 64, 64]
    for c in autotune.candidates(17, (False, True)) + autotune.candidates(1, (False, True)):
        native.set_k3_config(*autotune.config_of(c))   # every candidate is a valid configuration
    assert autotune.config_of((8, 0, 0, True, 16)) == [8, 0, 0, 1, 16]
    assert autotune.config_of((16, 0, 19, True)) == [16, 0, 19, 1, 0]
    native.set_k3_config()


def test_name_and_key():
    assert autotune.name((16, 0, 19, True)) == "16,0,19,1"
    AT = SimpleNamespace(n=1 << 26, nnz=1051749331)
    k = autotune.key(AT, "f32", 1, True, 20)
    assert k.endswith("|n2^26|nnz2^29|f32|k1|it20|weights1")
    assert autotune.key(AT, "f32", 1, False, 20) != k
    assert autotune.key(SimpleNamespace(n=0, nnz=0), "f64", 8, False, 5).endswith(
        "|n2^0|nnz2^0|f64|k8|it5|weights0")


def test_cache_hit_applies_the_stored_choice(tmp_path):
    AT = SimpleNamespace(n=1 << 20, nnz=15_900_000)
    cache = tmp_path / "tuning.json"
    entry = {"config": [16, 0, 19], "relabel": True, "ms": {"16,0,19,1": 1.0}}
    cache.write_text(json.dumps({autotune.key(AT, "f32", 1, True, 20): entry}))
    native.set_k3_config()
    got = autotune.tune(AT, "f32", 1, weights=object(), iters=20, cache=str(cache))
    assert got == entry
    assert native.get_k3_config()[:3] == (16, 0, 19)
    native.set_k3_config()


def test_unreadable_cache_is_empty(tmp_path):
    assert autotune._load(str(tmp_path / "missing.json")) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{ not json")
    assert autotune._load(str(bad)) == {}
