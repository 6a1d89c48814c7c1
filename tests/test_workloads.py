"""Seeded synthetic workloads: shapes, ranges, determinism (CPU only)."""
import numpy as np
import pytest

from paper_1310_3322_amd import workloads


@pytest.mark.parametrize("cfg", ["brute", "c1", "paper", "c2"])
def test_shapes_and_ranges(cfg):
    w = workloads.make_workload(cfg)
    assert w.pi.dtype == np.float32 and w.A.dtype == np.float32 and w.B.dtype == np.float32
    assert w.pi.shape == (w.K, w.N) and w.A.shape == (w.K, w.N, w.N) and w.B.shape == (w.K, w.N, w.M)
    assert w.symbols.dtype == np.int32 and w.offsets.dtype == np.int64 and w.lengths.dtype == np.int32
    assert w.symbols.min() >= 0 and w.symbols.max() < w.M
    assert w.offsets[0] == 0 and np.all(np.diff(w.offsets) == w.lengths[:-1])
    assert w.total_symbols == int(w.lengths.sum())
    np.testing.assert_allclose(w.A.sum(axis=-1), 1.0, atol=1e-6)
    np.testing.assert_allclose(w.B.sum(axis=-1), 1.0, atol=1e-6)


def test_length_ranges():
    assert workloads.make_workload("c2").lengths.min() >= 50
    assert workloads.make_workload("c2").lengths.max() <= 400
    w4 = workloads.make_workload("c4", scale=0.05)
    assert w4.lengths.min() >= 100 and w4.lengths.max() <= 1000 and w4.logits is not None
    w3 = workloads.make_workload("c3", scale=0.01)
    assert w3.lengths.min() >= 16 and w3.lengths.max() <= 2048 and w3.all_pairs


def test_deterministic():
    a = workloads.make_workload("c2", scale=0.05)
    b = workloads.make_workload("c2", scale=0.05)
    np.testing.assert_array_equal(a.symbols, b.symbols)
    np.testing.assert_array_equal(a.A, b.A)


def test_sampler_frequencies():
    rng = np.random.default_rng(0)
    rows = np.array([[0.1, 0.0, 0.6, 0.3], [0.0, 0.0, 0.0, 1.0]])
    s = workloads._RowSampler(rows)
    for r in range(2):
        d = s.draw(np.full(100000, r), rng.random(100000))
        f = np.bincount(d, minlength=4) / 1e5
        np.testing.assert_allclose(f, rows[r], atol=0.01)
        assert f[1] == 0.0


def test_subset_repacks():
    w = workloads.make_workload("paper")
    sub = w.subset(np.array([5, 2, 9]))
    assert sub.S == 3
    for d, s in enumerate([5, 2, 9]):
        np.testing.assert_array_equal(sub.symbols[sub.offsets[d]:sub.offsets[d] + sub.lengths[d]],
                                      w.symbols[w.offsets[s]:w.offsets[s] + w.lengths[s]])
