"""Drifting-Gaussian right-hand-side streams.

The paper's benchmark (Section 3, "Benchmarking an Accelerated Poisson
Solver") solves a time series of zero-Dirichlet Poisson problems whose sources
are localized blobs that move randomly from step to step.  This module is the
seeded stand-in for that workload:

    f_t(x) = sum_s a_s * exp(-|x - c_s(t)|^2 / (2 sigma^2))

evaluated at the interior points x = (i h_x, j h_y[, k h_z]), h = 1/(N+1), of
the unit square / cube.  Per source, in this order, one ``default_rng(seed)``
draws the amplitude a_s ~ U[0.5, 2], the start centre c_s(0) ~ U[0.2, 0.8]^d
and a direction (2D: angle ~ U[0, 2pi); 3D: normalised N(0, I_3)).  Each step
moves every centre by ``drift`` along its direction, reflecting off the faces
of [0.2, 0.8]^d.

Layout of every field: row-major with x fastest, numpy shape (ny, nx) in 2D and
(nz, ny, nx) in 3D, float64.
"""
from __future__ import annotations

import numpy as np


def grid_coords(n: int) -> np.ndarray:
    """Interior coordinates i/(n+1), i = 1..n, of one axis of the unit interval."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


class DriftingGaussians:
    """A seeded stream of source fields f_t on a ``dim``-dimensional grid."""

    LO, HI = 0.2, 0.8

    def __init__(self, shape, n_sources: int, sigma: float, seed: int,
                 drift: float = 0.01):
        self.shape = tuple(int(s) for s in shape)          # (ny, nx) or (nz, ny, nx)
        self.dim = len(self.shape)
        if self.dim not in (2, 3):
            raise ValueError("shape must have 2 or 3 axes")
        self.sigma = float(sigma)
        self.drift = float(drift)
        rng = np.random.default_rng(seed)
        amps, centres, dirs = [], [], []
        for _ in range(n_sources):
            amps.append(rng.uniform(0.5, 2.0))
            centres.append(rng.uniform(self.LO, self.HI, size=self.dim))
            if self.dim == 2:
                th = rng.uniform(0.0, 2.0 * np.pi)
                dirs.append(np.array([np.cos(th), np.sin(th)]))
            else:
                v = rng.standard_normal(3)
                dirs.append(v / np.linalg.norm(v))
        self.amps = np.array(amps)
        # centres and directions are stored in (x, y[, z]) order
        self.c0 = np.array(centres).reshape(n_sources, self.dim)
        self.dirs = np.array(dirs).reshape(n_sources, self.dim)

    def centres(self, t: int) -> np.ndarray:
        """Centres after t drift steps, with reflection at the box faces."""
        width = self.HI - self.LO
        raw = self.c0 - self.LO + t * self.drift * self.dirs
        # reflect onto [0, width]: fold with period 2*width
        folded = np.mod(raw, 2.0 * width)
        folded = np.where(folded > width, 2.0 * width - folded, folded)
        return folded + self.LO

    def field(self, t: int) -> np.ndarray:
        """f_t on the grid, float64, shape ``self.shape``."""
        axes = [grid_coords(n) for n in reversed(self.shape)]   # x, y[, z]
        out = np.zeros(self.shape, dtype=np.float64)
        inv = 1.0 / (2.0 * self.sigma ** 2)
        for a, c in zip(self.amps, self.centres(t)):
            factors = [np.exp(-(ax - cc) ** 2 * inv) for ax, cc in zip(axes, c)]
            if self.dim == 2:
                out += a * np.outer(factors[1], factors[0])
            else:
                out += a * (factors[2][:, None, None] * factors[1][None, :, None]
                            * factors[0][None, None, :])
        return out


class RandomDipoles:
    """The multi-scale workload of Section 3 ("Neural Network Designed for
    Multiple Scales"): every step's source is one asymmetric dipole whose two
    poles each have two scales, placed, separated and scaled at random anew at
    every step (steps are independent, so u_{t-1} is a poor guess).

    Step t draws from ``default_rng([seed, t])`` (any step can be generated on
    its own), in this order: the dipole centre c ~ U[0.3, 0.7]^d; the pole
    separation l ~ U[0.08, 0.3] along a uniformly random direction e (2D: angle;
    3D: normalised N(0, I_3)); the overall amplitude s ~ U[0.5, 2]; the negative
    pole's strength ratio q ~ U[0.4, 1]; one width factor per pole k+, k- ~
    U[0.75, 1.5].  Then

        f_t = s * (P(x; c + l e / 2, k+ (0.015, 0.06))
                   - q * P(x; c - l e / 2, k- (0.025, 0.10)))

    with P(x; p, (a, b)) = G(x; p, a) + 0.5 G(x; p, b) and G the unit-height
    Gaussian exp(-|x - p|^2 / (2 sigma^2)): a narrow core and a wide skirt per
    pole, the two poles different in widths and strength.  Layout as
    ``DriftingGaussians``."""

    WIDTHS_POS = (0.015, 0.06)
    WIDTHS_NEG = (0.025, 0.10)
    SKIRT = 0.5

    def __init__(self, shape, seed: int):
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        if self.dim not in (2, 3):
            raise ValueError("shape must have 2 or 3 axes")
        self.seed = int(seed)

    def draw(self, t: int) -> dict:
        """The random parameters of step t."""
        rng = np.random.default_rng([self.seed, int(t)])
        c = rng.uniform(0.3, 0.7, size=self.dim)
        sep = rng.uniform(0.08, 0.3)
        if self.dim == 2:
            th = rng.uniform(0.0, 2.0 * np.pi)
            e = np.array([np.cos(th), np.sin(th)])
        else:
            v = rng.standard_normal(3)
            e = v / np.linalg.norm(v)
        s = rng.uniform(0.5, 2.0)
        q = rng.uniform(0.4, 1.0)
        kp, kn = rng.uniform(0.75, 1.5, size=2)
        return {"centre": c, "sep": sep, "dir": e, "scale": s, "ratio": q,
                "pos": c + 0.5 * sep * e, "neg": c - 0.5 * sep * e,
                "widths_pos": tuple(kp * w for w in self.WIDTHS_POS),
                "widths_neg": tuple(kn * w for w in self.WIDTHS_NEG)}

    def _gauss(self, axes, p, sigma):
        inv = 1.0 / (2.0 * sigma ** 2)
        f = [np.exp(-(ax - pc) ** 2 * inv) for ax, pc in zip(axes, p)]
        if self.dim == 2:
            return np.outer(f[1], f[0])
        return f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]

    def field(self, t: int) -> np.ndarray:
        """f_t on the grid, float64, shape ``self.shape``."""
        d = self.draw(t)
        axes = [grid_coords(n) for n in reversed(self.shape)]   # x, y[, z]
        out = np.zeros(self.shape, dtype=np.float64)
        for w, k in zip(d["widths_pos"], (1.0, self.SKIRT)):
            out += k * self._gauss(axes, d["pos"], w)
        for w, k in zip(d["widths_neg"], (1.0, self.SKIRT)):
            out -= d["ratio"] * k * self._gauss(axes, d["neg"], w)
        return d["scale"] * out


class RandomBlob:
    """The linear-model workload of Section 3: one localized source moved at
    random.  Step t draws its centre c ~ U[0.05, 0.95]^d from
    ``default_rng([seed, t])`` (any step can be generated on its own), and
    f_t = exp(-|x - c|^2 / (2 sigma^2)).  Layout as ``DriftingGaussians``."""

    def __init__(self, shape, sigma: float, seed: int):
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        if self.dim not in (2, 3):
            raise ValueError("shape must have 2 or 3 axes")
        self.sigma, self.seed = float(sigma), int(seed)

    def centre(self, t: int) -> np.ndarray:
        return np.random.default_rng([self.seed, int(t)]).uniform(0.05, 0.95, size=self.dim)

    def field(self, t: int) -> np.ndarray:
        c = self.centre(t)
        axes = [grid_coords(n) for n in reversed(self.shape)]
        inv = 1.0 / (2.0 * self.sigma ** 2)
        f = [np.exp(-(ax - cc) ** 2 * inv) for ax, cc in zip(axes, c)]
        if self.dim == 2:
            return np.outer(f[1], f[0])
        return f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]


def system_sizes_batched(seed: int, n2d: int = 64, n3d: int = 8):
    """Grid sides of the uneven batched workload: 2D sides drawn uniformly from
    {128, 192, 256, 384, 512, 768, 1024}, 3D sides uniformly from 64..128."""
    rng = np.random.default_rng(seed)
    sides2 = rng.choice([128, 192, 256, 384, 512, 768, 1024], size=n2d)
    sides3 = rng.integers(64, 129, size=n3d)
    return [int(s) for s in sides2], [int(s) for s in sides3]
