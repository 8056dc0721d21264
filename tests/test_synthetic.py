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


def test_dipoles_independent_steps_and_shape():
    """Every step is drawn from its own (seed, t) generator: the same field
    whatever order the steps are asked for, a new dipole at every step."""
    from synthetic import RandomDipoles
    a, b = RandomDipoles((48, 64), seed=7), RandomDipoles((48, 64), seed=7)
    f5 = a.field(5)
    assert f5.shape == (48, 64)
    for t in (9, 0, 3):
        b.field(t)
    assert np.array_equal(b.field(5), f5)
    assert not np.array_equal(a.field(6), f5)
    assert RandomDipoles((8, 10, 12), seed=1).field(0).shape == (8, 10, 12)


def test_dipole_is_two_asymmetric_two_scale_poles():
    """The field equals the stated sum written out pointwise; it has a
    positive and a negative extremum near the two poles, at the drawn
    separation; and the poles differ (widths, strength)."""
    from synthetic import RandomDipoles
    n = 96
    g = RandomDipoles((n, n), seed=11)
    for t in range(6):
        d = g.draw(t)
        f = g.field(t)
        x = np.arange(1, n + 1) / (n + 1.0)
        X, Y = np.meshgrid(x, x)

        def pole(p, widths):
            r2 = (X - p[0]) ** 2 + (Y - p[1]) ** 2
            return np.exp(-r2 / (2 * widths[0] ** 2)) + 0.5 * np.exp(-r2 / (2 * widths[1] ** 2))
        ref = d["scale"] * (pole(d["pos"], d["widths_pos"]) - d["ratio"] * pole(d["neg"], d["widths_neg"]))
        assert np.allclose(f, ref, rtol=1e-12, atol=1e-14)
        assert np.isclose(np.linalg.norm(d["pos"] - d["neg"]), d["sep"])
        assert 0.08 <= d["sep"] <= 0.3 and 0.5 <= d["scale"] <= 2.0 and 0.4 <= d["ratio"] <= 1.0
        for (a, b), base in ((d["widths_pos"], (0.015, 0.06)), (d["widths_neg"], (0.025, 0.10))):
            k = a / base[0]
            assert 0.75 <= k <= 1.5 and np.isclose(b / base[1], k)
        ip, jp = np.unravel_index(np.argmax(f), f.shape)
        im, jm = np.unravel_index(np.argmin(f), f.shape)
        assert f[ip, jp] > 0 > f[im, jm]
        assert np.hypot(x[jp] - d["pos"][0], x[ip] - d["pos"][1]) < 0.03
        assert np.hypot(x[jm] - d["neg"][0], x[im] - d["neg"][1]) < 0.06


def test_random_blob():
    from synthetic import RandomBlob
    g = RandomBlob((30, 30), 0.03, seed=3)
    f = g.field(4)
    c = g.centre(4)
    x = np.arange(1, 31) / 31.0
    X, Y = np.meshgrid(x, x)
    assert np.allclose(f, np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * 0.03 ** 2)), rtol=1e-13)
    assert np.array_equal(RandomBlob((30, 30), 0.03, seed=3).field(4), f)
    cs = np.array([g.centre(t) for t in range(200)])
    assert cs.min() >= 0.05 and cs.max() <= 0.95 and cs.std(axis=0).min() > 0.2
