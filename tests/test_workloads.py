"""The seeded workload recipes (no GPU needed): sizes follow the paper's
benchmark definition (N = 2^S, M = 16 N, Graph500 initiator), and the
many-small-graphs batch is reproducible, in range and as large as its
distribution says."""
import numpy as np

from paper_1603_01876_amd import workloads


def test_pipeline_sizes_and_initiator():
    s = workloads.pipeline(26)
    assert (s.n, s.m) == (1 << 26, 1 << 30)
    assert (s.a, s.b, s.c, s.d) == (0.57, 0.19, 0.19, 0.05)
    assert abs(s.a + s.b + s.c + s.d - 1.0) < 1e-12
    assert s.with_seed(5).seed == 5 and s.with_seed(5).scale == 26
    assert s.as_dict()["edge_factor"] == 16


def test_batch_is_reproducible_and_in_range():
    a = workloads.batch(512, 8, 14)
    b = workloads.batch(512, 8, 14)
    assert a == b
    scales = np.array([g.scale for g in a])
    assert scales.min() >= 8 and scales.max() <= 14
    assert set(scales.tolist()) == set(range(8, 15))       # every scale drawn at 512 graphs
    assert len({g.seed for g in a}) == 512                 # graphs have their own seeds
    assert workloads.batch(512, 8, 14, seed=7) != a


def test_batch_edge_total_matches_its_distribution():
    # S uniform on 8..14: E[M] = 16 * mean(2^8..2^14) per graph; the sum of
    # 512 draws lies well within 4 standard deviations of 512 * E[M].
    g = workloads.batch(512, 8, 14)
    total = sum(x.m for x in g)
    m = 16 * (2.0 ** np.arange(8, 15))
    mean, sd = m.mean(), m.std()
    assert abs(total - 512 * mean) < 4 * sd * np.sqrt(512)
