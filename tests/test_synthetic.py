"""The seeded input generators: determinism, shapes, and the drift rule."""
import numpy as np

from synthetic import DriftingGaussians, system_sizes_batched


def test_deterministic_and_shapes():
    a = DriftingGaussians((64, 48), 3, 0.05, seed=1000)
    b = DriftingGaussians((64, 48), 3, 0.05, seed=1000)
    assert a.field(0).shape == (64, 48)
    assert np.array_equal(a.field(7), b.field(7))
    assert not np.array_equal(a.field(0), DriftingGaussians((64, 48), 3, 0.05, seed=1001).field(0))
    g3 = DriftingGaussians((10, 12, 14), 2, 0.1, seed=3)
    assert g3.field(0).shape == (10, 12, 14)


def test_drift_speed_and_reflection():
    g = DriftingGaussians((32, 32), 4, 0.05, seed=5)
    prev = g.centres(0)
    for t in range(1, 400):
        c = g.centres(t)
        assert np.all(c >= 0.2 - 1e-15) and np.all(c <= 0.8 + 1e-15)
        step = np.linalg.norm(c - prev, axis=1)
        assert np.all(step <= 0.01 + 1e-12)          # reflection can only shorten a step
        prev = c
    assert np.all(g.amps >= 0.5) and np.all(g.amps <= 2.0)


def test_field_is_sum_of_gaussians():
    g = DriftingGaussians((16, 20), 2, 0.07, seed=8)
    f = g.field(3)
    c = g.centres(3)
    x = np.arange(1, 21) / 21.0
    y = np.arange(1, 17) / 17.0
    X, Y = np.meshgrid(x, y)
    ref = sum(a * np.exp(-((X - cc[0]) ** 2 + (Y - cc[1]) ** 2) / (2 * 0.07 ** 2)) for a, cc in zip(g.amps, c))
    assert np.allclose(f, ref, rtol=1e-13, atol=0)


def test_batched_sizes():
    s2, s3 = system_sizes_batched(5000)
    assert len(s2) == 64 and len(s3) == 8
    assert set(s2) <= {128, 192, 256, 384, 512, 768, 1024}
    assert all(64 <= s <= 128 for s in s3)
