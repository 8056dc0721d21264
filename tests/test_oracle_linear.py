"""Pins of the linear-model oracle: finite differences and torch autograd for
the gradient, the exact inverse (zero loss, every eigenvalue of A T at 1),
the residual bound |r0| <= |I - A T|_2 |b|, and the dense operator against
the oracle's stencil and its known extreme eigenvalues."""
import numpy as np
import torch

from oracle import gmres as og
from oracle import linear as lin


def test_dense_operator_matches_stencil_and_eigenvalues():
    shape = (5, 7)
    A = lin.dense_operator(shape)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(shape)
    assert np.allclose(A @ u.ravel(), og.apply(u).ravel(), rtol=1e-14, atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(A))
    lam = lambda k, n: 4 * (n + 1) ** 2 * np.sin(k * np.pi / (2 * (n + 1))) ** 2  # noqa: E731
    assert np.isclose(ev[0], lam(1, 5) + lam(1, 7), rtol=1e-12)
    assert np.isclose(ev[-1], lam(5, 5) + lam(7, 7), rtol=1e-12)


def test_gradient_fd_and_torch():
    rng = np.random.default_rng(1)
    n, B = 12, 3
    T = rng.standard_normal((n, n)) * 0.1
    b = rng.standard_normal((B, n))
    x = rng.standard_normal((B, n))
    L, g = lin.loss_and_grad(T, b, x)
    D = rng.standard_normal((n, n))
    eps = 1e-6
    fd = (lin.loss_and_grad(T + eps * D, b, x)[0] - lin.loss_and_grad(T - eps * D, b, x)[0]) / (2 * eps)
    assert abs(fd - np.sum(g * D)) <= 1e-7 * abs(fd)
    Tt = torch.tensor(T, requires_grad=True)
    lt = torch.sum((torch.tensor(b) @ Tt.T - torch.tensor(x)) ** 2) / B
    lt.backward()
    assert np.isclose(float(lt.detach()), L, rtol=1e-14)
    assert np.allclose(Tt.grad.numpy(), g, rtol=1e-12, atol=1e-14)


def test_exact_inverse_and_residual_bound():
    shape = (6, 6)
    A = lin.dense_operator(shape)
    Ainv = np.linalg.inv(A)
    rng = np.random.default_rng(2)
    b = rng.standard_normal((4, 36))
    x = b @ Ainv.T
    L, g = lin.loss_and_grad(Ainv, b, x)
    assert L <= 1e-20 and np.abs(g).max() <= 1e-12
    assert np.allclose(lin.spectrum(Ainv, shape), 1.0, atol=1e-10)
    T = Ainv + 1e-4 * rng.standard_normal((36, 36))
    r0 = b - lin.forward(T, b) @ A.T
    bound = np.linalg.norm(np.eye(36) - A @ T, 2) * np.linalg.norm(b, axis=1)
    assert np.all(np.linalg.norm(r0, axis=1) <= bound * (1 + 1e-12))


def test_gradient_descent_fits_the_pairs_it_sees():
    """Gradient descent on pairs from the true inverse: the loss falls and the
    eigenvalues of A T stay in the unit disk while some move to 1."""
    shape = (6, 6)
    A = lin.dense_operator(shape)
    Ainv = np.linalg.inv(A)
    rng = np.random.default_rng(3)
    T = np.zeros((36, 36))
    b = rng.standard_normal((8, 36))
    x = b @ Ainv.T
    losses = []
    for _ in range(200):
        T, L, _ = lin.sgd_step(T, b, x, lr=0.05)
        losses.append(L)
    assert losses[-1] < 1e-3 * losses[0]
    ev = lin.spectrum(T, shape)
    assert np.abs(ev).max() <= 1 + 1e-6
    assert np.sum(np.abs(ev - 1) < 0.05) >= 6
