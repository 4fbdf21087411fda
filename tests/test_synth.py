"""The seeded input generators: determinism, exact sizes, clustering."""
import numpy as np

from paper_1810_02916_amd.synth import (WORKLOADS, batched_specs, clustered_box, make_box,
                                        occupancy_stats, uniform_box)


def test_uniform_deterministic_and_in_box():
    a = uniform_box(1000, 2.0, 7)
    b = uniform_box(1000, 2.0, 7)
    assert a.shape == (1000, 3) and a.dtype == np.float64
    assert np.array_equal(a, b)
    assert not np.array_equal(a, uniform_box(1000, 2.0, 8))
    assert a.min() >= 0 and a.max() < 2.0


def test_clustered_exact_n_and_clustered():
    pos = clustered_box(20000, 24, 12, 1.0, 1.5, 0.5, seed=3)
    assert pos.shape == (20000, 3)
    assert np.array_equal(pos, clustered_box(20000, 24, 12, 1.0, 1.5, 0.5, seed=3))
    st = occupancy_stats(pos, 12, 1.0)
    # lognormal re-weighting gives a spread of log-counts well above Poisson
    assert st["std_ln_count"] > 0.8
    assert st["max_cell"] > 10 * 20000 / 12 ** 3
    assert st["interactions_per_particle"] > 125 * 20000 / 12 ** 3


def test_input_not_sorted():
    pos = clustered_box(5000, 16, 8, 1.0, 1.5, 0.5, seed=1)
    c = np.floor(pos * 8).astype(int)
    lin = (c[:, 0] * 8 + c[:, 1]) * 8 + c[:, 2]
    assert (np.diff(lin) < 0).sum() > 1000


def test_registry_shapes():
    sp = WORKLOADS["uniform32k"]
    assert (sp.n, sp.K) == (32768, 16)
    np.testing.assert_allclose(sp.eps_s, 2.16 * 0.04 / 32)
    sp = WORKLOADS["clustered2m"]
    assert (sp.n, sp.K, sp.side) == (128 ** 3, 64, 128)
    sp = WORKLOADS["clustered134m"]
    assert (sp.n, sp.K, sp.L) == (512 ** 3, 256, 125.0)
    specs = batched_specs(64)
    assert len(specs) == 64
    assert all(32 ** 3 <= s.n <= 96 ** 3 for s in specs)
    assert all(s.K >= 5 for s in specs)
    pos = make_box(specs[0])
    assert pos.shape == (specs[0].n, 3)
