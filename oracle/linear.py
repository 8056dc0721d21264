"""NumPy FP64 oracle for the single-layer linear model (test infrastructure only).

Section 3 of the paper studies a network that is one fully connected layer
without bias, so the initial guess is a matrix product x0 = T b, trained on the
solver's (b, x) pairs.  Its residual is r0 = b - A T b = (I - A T) b, bounded
by |I - A T|_2 |b|_2 (the paper prints this as an equality), so training
drives the spectrum of A T towards the unit circle, where the paper observes
it over the course of a run.

Loss (Section 2.3): L = (1/B) sum_i |T b_i - x_i|_2^2, gradient
dL/dT = (2/B) sum_i (T b_i - x_i) b_i^T.  The paper does not name the
optimiser of this model; it is read as plain gradient descent, T <- T - lr dL/dT.
"""
from __future__ import annotations

import numpy as np

from . import gmres as _gmres


def forward(T: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b [B, n] -> x0 [B, n], x0_i = T b_i."""
    return b @ T.T


def loss_and_grad(T: np.ndarray, b: np.ndarray, x: np.ndarray):
    B = b.shape[0]
    e = forward(T, b) - x
    return float(np.sum(e ** 2) / B), (2.0 / B) * e.T @ b


def sgd_step(T: np.ndarray, b: np.ndarray, x: np.ndarray, lr: float):
    """One gradient-descent step; returns (new T, loss before the step, gradient)."""
    L, g = loss_and_grad(T, b, x)
    return T - lr * g, L, g


def dense_operator(shape) -> np.ndarray:
    """The solver's discrete Laplacian A as a dense n x n matrix (column j is
    A applied to the j-th unit vector of the row-major grid)."""
    n = int(np.prod(shape))
    cols = [_gmres.apply(e.reshape(shape)).ravel() for e in np.eye(n)]
    return np.stack(cols, axis=1)


def spectrum(T: np.ndarray, shape) -> np.ndarray:
    """Eigenvalues of A T."""
    return np.linalg.eigvals(dense_operator(shape) @ T)
