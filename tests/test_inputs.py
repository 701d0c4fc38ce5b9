"""Seeded workload generators: determinism, bijectivity of the relabelling,
RMAT quadrant statistics, ranges, and the source picker's contract."""
import numpy as np


def test_splitmix64_published_vector(inputs_mod):
    # First outputs of SplitMix64 seeded with 0 (reference values of the
    # published algorithm, as used by e.g. xoshiro's seeding code).
    assert inputs_mod.splitmix64_at(0, 0) == 0xE220A8397B1DCDAF
    assert inputs_mod.splitmix64_at(0, 1) == 0x6E789E6AA1B965F4
    assert inputs_mod.splitmix64_at(0, 2) == 0x06C45D188009454F


def test_permutation_is_bijective(inputs_mod):
    for bits in (1, 2, 5, 10, 12):
        vals = {inputs_mod.perm_value(bits, 1234, x) for x in range(1 << bits)}
        assert vals == set(range(1 << bits))


def test_rmat_deterministic_and_in_range(inputs_mod):
    s1, d1 = inputs_mod.rmat_edges(12)
    s2, d2 = inputs_mod.rmat_edges(12, nthreads=3)
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    assert len(s1) == 16 << 12
    assert s1.min() >= 0 and s1.max() < 4096 and d1.min() >= 0 and d1.max() < 4096
    s3, _ = inputs_mod.rmat_edges(12, seed=99)
    assert not np.array_equal(s1, s3)


def test_rmat_quadrant_frequencies(inputs_mod):
    """Top bit of (src, dst) before relabelling follows the quadrant
    probabilities a, b, c, d = .57, .19, .19, .05."""
    src, dst = inputs_mod.rmat_edges(16, permute=False)
    top_s, top_d = src >> 15, dst >> 15
    g = len(src)
    freq = [np.mean((top_s == r) & (top_d == c)) for r, c in ((0, 0), (0, 1), (1, 0), (1, 1))]
    for f, p in zip(freq, (0.57, 0.19, 0.19, 0.05)):
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / g)


def test_er_range(inputs_mod):
    s, d = inputs_mod.er_edges(1000, 50000, seed=5)
    assert s.min() >= 0 and s.max() < 1000 and d.min() >= 0 and d.max() < 1000
    assert abs(np.mean(s) - 499.5) < 10


def test_pick_sources(inputs_mod):
    src = np.array([0, 1, 2, 5, 5], np.int32)
    dst = np.array([1, 2, 2, 5, 6], np.int32)     # 2-2 and 5-5 are loops
    out = inputs_mod.pick_sources(src, dst, 10, 10, seed=3)
    assert sorted(out.tolist()) == [0, 1, 2, 5, 6]
    s, d = inputs_mod.rmat_edges(10)
    out = inputs_mod.pick_sources(s, d, 1024, 64, seed=1001)
    assert len(set(out.tolist())) == 64
    ok = np.zeros(1024, bool)
    m = s != d
    ok[s[m]] = True
    ok[d[m]] = True
    assert ok[out].all()
    assert np.array_equal(out, inputs_mod.pick_sources(s, d, 1024, 64, seed=1001))


def test_pick_sources_from_degrees_equals_edge_list_picker(inputs_mod, oracle_mod):
    """The degree-array picker returns the edge-list picker's sources (a vertex
    has degree > 0 in the simple graph iff it ends a non-loop pair)."""
    for scale, k, seed in ((10, 64, 1), (12, 300, 7), (8, 10 ** 4, 3)):
        n = 1 << scale
        src, dst = inputs_mod.rmat_edges(scale)
        deg = oracle_mod.Graph(src, dst, n).degrees()
        np.testing.assert_array_equal(inputs_mod.pick_sources_deg(deg, k, seed),
                                      inputs_mod.pick_sources(src, dst, n, k, seed))
