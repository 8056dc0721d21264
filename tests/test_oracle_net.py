"""Pins for the NumPy FP64 guess-network oracle.

Checked against: a brute-force direct sum for the convolution and torch's CPU
conv2d in float64, SciPy's DST-I for the sine basis, the closed-form inverse
of the Dirichlet Laplacian on the retained modes, central finite differences
for every gradient, the Adam closed form after one step and torch's CPU Adam;
the band's least-squares fit against the closed-form eigenvalues of A (one
consistent pair from a dense solve) and against brute-force perturbation of
the loss it minimises.
"""
import numpy as np
import pytest
import scipy.fft
import torch

from oracle import gmres as og
from oracle import net
from synthetic import DriftingGaussians, guess_net_params


def laplacian_modes(H, W, K):
    """lambda[k, l] of the zero-Dirichlet 5-point Laplacian (h = 1/(n+1)) on
    the mode sin((k+1) pi y) sin((l+1) pi x), k, l < K (closed form)."""
    k = np.arange(1, K + 1, dtype=np.float64)
    ly = 4.0 * (H + 1) ** 2 * np.sin(k * np.pi / (2 * (H + 1))) ** 2
    lx = 4.0 * (W + 1) ** 2 * np.sin(k * np.pi / (2 * (W + 1))) ** 2
    return ly[:, None] + lx[None, :]


def small_params(C=4, M=3, seed=0, K=None):
    return guess_net_params(seed, channels=C, modes=M, zero_last=False, random_bias=True,
                            skip_modes=K)


def test_conv_direct_sum_and_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = net.conv3x3(x, w, b)
    ref = np.zeros_like(y)
    for bi in range(2):
        for d in range(4):
            for i in range(5):
                for j in range(6):
                    s = b[d]
                    for c in range(3):
                        for p in range(3):
                            for q in range(3):
                                ii, jj = i + p - 1, j + q - 1
                                if 0 <= ii < 5 and 0 <= jj < 6:
                                    s += w[d, c, p, q] * x[bi, c, ii, jj]
                    ref[bi, d, i, j] = s
    assert np.max(np.abs(y - ref)) < 1e-12
    t = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                   padding=1).numpy()
    assert np.max(np.abs(y - t)) < 1e-12


def test_sine_basis_is_dst1():
    n, M = 37, 16
    S = net.sine_basis(n, M)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n)
    assert np.allclose(S @ x, scipy.fft.dst(x, type=1)[:M] / 2.0, atol=1e-12)
    Sf = net.sine_basis(n, n)
    assert np.allclose(Sf @ Sf.T, (n + 1) / 2.0 * np.eye(n), atol=1e-11)


def test_spectral_layer_inverts_laplacian_on_retained_modes():
    N, M, C = 40, 16, 1
    h = 1.0 / (N + 1)
    k = np.arange(1, M + 1)
    lam1 = (4.0 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2
    lam = lam1[:, None] + lam1[None, :]                       # [ky, kx]
    wk = (1.0 / lam)[:, :, None, None]
    rng = np.random.default_rng(2)
    coef = rng.standard_normal((M, M))
    S = net.sine_basis(N, M)
    f = S.T @ coef @ S                                         # f in the span of the retained modes
    _, cache = net.spectral_forward(f[None, None], np.zeros((C, C)), np.zeros(C), wk)
    z = cache[2][0, 0]                                         # pre-activation
    assert np.max(np.abs(og.apply(z) - f)) <= 1e-11 * np.abs(f).max()


def test_untrained_output_layer_returns_previous_solution():
    p = guess_net_params(3, channels=8, modes=4, zero_last=True)
    g = DriftingGaussians((20, 20), 2, 0.05, seed=9)
    f = np.stack([g.field(1), g.field(2)])
    u = np.stack([og.gmres(g.field(0), m=10, rtol=1e-6)[0], g.field(0) * 0.01])
    guess, out, s = net.forward(p, f, u)
    assert np.array_equal(guess, u) and np.all(out == 0)


def test_forward_is_homogeneous_in_the_inputs():
    """Scaling (f, u_prev) by a > 0 scales the guess by a (input normalisation)."""
    p = small_params()
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2, 9, 11))
    u = rng.standard_normal((2, 9, 11)) * 0.01
    g1, _, _ = net.forward(p, f, u)
    g2, _, _ = net.forward(p, 7.5 * f, 7.5 * u)
    assert np.allclose(g2, 7.5 * g1, rtol=1e-12, atol=1e-14)


def test_zero_source_and_exact_previous_solution():
    p = small_params()
    u = np.random.default_rng(5).standard_normal((1, 6, 6))
    g, out, s = net.forward(p, np.zeros((1, 6, 6)), u)
    assert np.all(np.isfinite(g))
    # a previous solution that already solves A u = f leaves nothing to correct
    f = og.apply(u[0])[None]
    g2, out2, s2 = net.forward(p, f, u)
    assert s2[0] == 1.0 and np.array_equal(g2, u)


def test_input_is_residual_of_previous_solution():
    """Channel 0 is (f - A u_prev)/RMS, channel 1 is f/RMS: checked against the
    sparse Kronecker-sum Laplacian."""
    from test_oracle_gmres import sparse_laplacian
    rng = np.random.default_rng(8)
    f = rng.standard_normal((2, 9, 7))
    u = rng.standard_normal((2, 9, 7))
    x, s_r, s_in = net.normalise(f, u)
    A = sparse_laplacian((9, 7))
    for b in range(2):
        r = f[b].ravel() - A @ u[b].ravel()
        assert np.allclose(x[b, 0].ravel(), r / np.sqrt(np.mean(r ** 2)), rtol=1e-12, atol=1e-12)
        assert np.allclose(x[b, 1], f[b] / np.sqrt(np.mean(f[b] ** 2)), rtol=1e-13)
        assert abs(s_r[b] - np.sqrt(np.mean(r ** 2))) <= 1e-12 * s_r[b]


def test_band_path_is_the_truncated_inverse():
    """With the convolutional output switched off and the band weights at
    c_u / lambda_kl, the correction d = guess - u_prev solves A d = P r exactly, P the
    projection on the retained sine modes and r = f - A u_prev (checked
    against the sparse Kronecker-sum Laplacian and an explicit projection)."""
    from test_oracle_gmres import sparse_laplacian
    H, W, M = 21, 17, 6
    p = guess_net_params(7, channels=4, modes=M, zero_last=True)
    p["band.w"] = net.C_U / laplacian_modes(H, W, M)
    rng = np.random.default_rng(11)
    f = rng.standard_normal((2, H, W))
    u = rng.standard_normal((2, H, W))
    g, _, _ = net.forward(p, f, u)
    A = sparse_laplacian((H, W))
    # projection on the first M modes per axis: orthonormal sine rows
    Qy = net.sine_basis(H, M) * np.sqrt(2.0 / (H + 1))
    Qx = net.sine_basis(W, M) * np.sqrt(2.0 / (W + 1))
    for b in range(2):
        r = f[b] - (A @ u[b].ravel()).reshape(H, W)
        Pr = Qy.T @ (Qy @ r @ Qx.T) @ Qx
        d = (g[b] - u[b]).ravel()
        assert np.allclose(A @ d, Pr.ravel(), rtol=0, atol=1e-9 * np.abs(Pr).max())
    # the eigenvalues used are those of A
    lam = laplacian_modes(H, W, M)
    phi = np.outer(np.sin(3 * np.pi * np.arange(1, H + 1) / (H + 1)),
                   np.sin(5 * np.pi * np.arange(1, W + 1) / (W + 1)))
    assert np.allclose((A @ phi.ravel()).reshape(H, W), lam[2, 4] * phi, atol=1e-9 * lam[2, 4])


def test_guess_is_exact_on_the_band_whatever_the_convolutions():
    """With the band weights at c_u / lambda_kl and random (nonzero) convolutions, the
    correction d = guess - u_prev agrees with the exact correction A^-1 r
    (dense LU solve) on the K x K skip band, and the convolutional branch
    still acts off the band."""
    from test_oracle_gmres import sparse_laplacian
    H, W, M, K = 13, 11, 3, 5
    p = guess_net_params(9, channels=4, modes=M, skip_modes=K)
    p["band.w"] = net.C_U / laplacian_modes(H, W, K)
    rng = np.random.default_rng(21)
    f = rng.standard_normal((2, H, W))
    u = rng.standard_normal((2, H, W))
    g, _, _ = net.forward(p, f, u)
    A = sparse_laplacian((H, W)).toarray()
    Qy = net.sine_basis(H, K) * np.sqrt(2.0 / (H + 1))
    Qx = net.sine_basis(W, K) * np.sqrt(2.0 / (W + 1))
    for b in range(2):
        r = f[b] - (A @ u[b].ravel()).reshape(H, W)
        d_exact = np.linalg.solve(A, r.ravel()).reshape(H, W)
        d = g[b] - u[b]
        on_band = Qy @ d @ Qx.T
        assert np.allclose(on_band, Qy @ d_exact @ Qx.T, rtol=0,
                           atol=1e-10 * np.abs(Qy @ d_exact @ Qx.T).max())
        off_band = d - Qy.T @ on_band @ Qx
        assert np.linalg.norm(off_band) > 1e-3 * np.linalg.norm(d)


def test_loss_closed_form():
    p = small_params()
    rng = np.random.default_rng(6)
    f = rng.standard_normal((3, 7, 8))
    u = rng.standard_normal((3, 7, 8)) * 0.1
    _, out, s = net.forward(p, f, u)
    delta = rng.standard_normal(out.shape)
    # choose the target so that out - t = delta
    u_t = u + (out - delta) * s[:, None, None] / net.C_U
    L, _ = net.loss_and_grads(p, f, u, u_t)
    assert abs(L - np.sum(delta ** 2) / 3) <= 1e-10 * L


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    p = small_params(C=4, M=3, seed=seed, K=4)
    rng = np.random.default_rng(10 + seed)
    B, H, W = 2, 7, 6
    f = rng.standard_normal((B, H, W))
    u = rng.standard_normal((B, H, W)) * 0.05
    ut = u + rng.standard_normal((B, H, W)) * 0.05
    L, g = net.loss_and_grads(p, f, u, ut)
    assert set(g) == set(p) - {"band.w"}
    eps = 1e-6
    for name in g:
        d = rng.standard_normal(p[name].shape)
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        pp[name] = p[name] + eps * d
        pm[name] = p[name] - eps * d
        fd = (net.loss_and_grads(pp, f, u, ut)[0] - net.loss_and_grads(pm, f, u, ut)[0]) / (2 * eps)
        an = float(np.sum(g[name] * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(L)), name


def test_gradients_match_torch_autograd():
    """Same network written with torch CPU float64 ops and autograd."""
    p = small_params(C=4, M=3, seed=2, K=5)
    rng = np.random.default_rng(12)
    B, H, W = 2, 8, 9
    f = rng.standard_normal((B, H, W))
    u = rng.standard_normal((B, H, W)) * 0.05
    ut = u + rng.standard_normal((B, H, W)) * 0.05
    L, g = net.loss_and_grads(p, f, u, ut)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    F = torch.nn.functional
    x0, _, s = net.normalise(f, u)
    x = torch.tensor(x0)
    a = F.relu(F.conv2d(x, T["conv1.w"], T["conv1.b"], padding=1))
    a = F.relu(F.conv2d(a, T["conv2.w"], T["conv2.b"], padding=1))
    M = 3
    Sy = torch.tensor(np.sin(np.arange(1, M + 1)[:, None] * np.pi * np.arange(1, H + 1)[None] / (H + 1)))
    Sx = torch.tensor(np.sin(np.arange(1, M + 1)[:, None] * np.pi * np.arange(1, W + 1)[None] / (W + 1)))
    X = Sy @ a @ Sx.T                                          # [B, C, M, M]
    Y = torch.einsum("kldc,bckl->bdkl", T["spec.wk"], X)
    ys = (2.0 / (H + 1)) * (2.0 / (W + 1)) * (Sy.T @ Y @ Sx)
    a = F.relu(F.conv2d(a, T["spec.w1"][:, :, None, None], T["spec.b"]) + ys)
    a = F.relu(F.conv2d(a, T["conv4.w"], T["conv4.b"], padding=1))
    a = F.relu(F.conv2d(a, T["conv5.w"], T["conv5.b"], padding=1))
    c6 = F.conv2d(a, T["conv6.w"], T["conv6.b"], padding=1)[:, 0]
    K = 5
    Ky = torch.tensor(np.sin(np.arange(1, K + 1)[:, None] * np.pi * np.arange(1, H + 1)[None] / (H + 1)))
    Kx = torch.tensor(np.sin(np.arange(1, K + 1)[:, None] * np.pi * np.arange(1, W + 1)[None] / (W + 1)))
    nrm = (2.0 / (H + 1)) * (2.0 / (W + 1))
    Xr = Ky @ x[:, 0] @ Kx.T
    out = c6 - nrm * (Ky.T @ (Ky @ c6 @ Kx.T) @ Kx) + nrm * (Ky.T @ (T["band.w"] * Xr) @ Kx)
    t = torch.tensor(net.target(ut, u, s))
    Lt = ((out - t) ** 2).sum() / B
    Lt.backward()
    assert abs(Lt.item() - L) <= 1e-12 * L
    for k in g:
        assert np.allclose(T[k].grad.numpy(), g[k], rtol=1e-9, atol=1e-12 * np.abs(g[k]).max()), k


def test_without_band_the_output_is_the_last_convolution():
    """K = 0 (no band path): out is the L6 convolution itself, so the guess is
    u_prev + (s_r / c_u) L6(a5) with nothing projected."""
    p = guess_net_params(13, channels=4, modes=3, zero_last=False, skip_modes=0)
    assert "band.w" not in p
    rng = np.random.default_rng(23)
    f = rng.standard_normal((2, 8, 10))
    u = rng.standard_normal((2, 8, 10)) * 0.1
    guess, out, s, c = net.forward(p, f, u, keep=True)
    c6 = net.conv3x3(c["a5"], p["conv6.w"], p["conv6.b"])[:, 0]
    assert np.array_equal(out, c6)
    s_r = np.sqrt(np.mean((f - np.stack([og.apply(ub) for ub in u])) ** 2, axis=(1, 2)))
    assert np.allclose(guess, u + (s_r / net.C_U)[:, None, None] * c6, rtol=1e-13, atol=1e-15)


def test_band_fit_recovers_the_inverse_eigenvalues():
    """One pair from a loose solve (GMRES to 1e-4 only): since the fit pairs
    the correction with the right-hand side it solves exactly, the
    least-squares band weights equal c_u / lambda_kl of the closed form on
    every band mode to rounding, on a non-square grid (a transposed basis, a
    scale taken from s_f instead of s_r, or a fit on the residual input
    instead -- 1e-4 off here -- would fail)."""
    H, W, K = 19, 14, 6
    g = DriftingGaussians((H, W), 3, 0.08, seed=3)
    f = g.field(2)[None]
    u_prev = og.gmres(g.field(1), m=10, rtol=1e-4)[0][None]
    u_t = og.gmres(f[0], u_prev[0], m=10, rtol=1e-4)[0][None]
    sxt, sxx = net.band_stats(f, u_prev, u_t, K)
    w = net.band_weights(sxt, sxx)
    expect = net.C_U / laplacian_modes(H, W, K)
    assert np.all(sxx > 0)
    assert np.allclose(w, expect, rtol=1e-10, atol=0)
    # the same fit on the network's own input (the residual of u_prev) is off
    # by the loose solve's error
    x0, _, s = net.normalise(f, u_prev)
    Sy, Sx = net.sine_basis(H, K), net.sine_basis(W, K)
    Xr = Sy @ x0[0, 0] @ Sx.T
    Tt = Sy @ net.target(u_t, u_prev, s)[0] @ Sx.T
    assert np.max(np.abs(Tt / Xr / expect - 1.0)) > 1e-6
    # with the fitted weights and no convolutional output, the guess solves
    # A d = r exactly on the band (dense LU)
    from test_oracle_gmres import sparse_laplacian
    A = sparse_laplacian((H, W)).toarray()
    p = guess_net_params(4, channels=4, modes=3, zero_last=True, skip_modes=K)
    p["band.w"] = w
    guess, _, _ = net.forward(p, f, u_prev)
    r = f[0] - (A @ u_prev[0].ravel()).reshape(H, W)
    d_exact = np.linalg.solve(A, r.ravel()).reshape(H, W)
    Qy = net.sine_basis(H, K) * np.sqrt(2.0 / (H + 1))
    Qx = net.sine_basis(W, K) * np.sqrt(2.0 / (W + 1))
    on = Qy @ (guess[0] - u_prev[0] - d_exact) @ Qx.T
    assert np.abs(on).max() <= 1e-10 * np.abs(Qy @ d_exact @ Qx.T).max()


def test_band_fit_is_the_least_squares_minimiser():
    """Random (inconsistent) pairs: the fitted weights minimise the band's
    loss on the exact pairs -- the network loss with f = A u_t (so that the
    residual input is A d exactly) and the convolutional output off: every
    perturbation raises it and the central difference along random
    directions vanishes."""
    H, W, K, B = 9, 12, 4, 3
    rng = np.random.default_rng(17)
    u = rng.standard_normal((B, H, W)) * 0.05
    ut = u + rng.standard_normal((B, H, W)) * 0.05
    fe = np.stack([og.apply(ub) for ub in ut])            # r_fin = 0: the exact pair
    sxt, sxx = net.band_stats(fe, u, ut, K)
    p = guess_net_params(5, channels=4, modes=3, zero_last=True, skip_modes=K)
    p["band.w"] = net.band_weights(sxt, sxx)
    # with one sample the fit does not depend on f (only on the pair A d, d)
    f1 = fe[:1] + 1e-3 * rng.standard_normal((1, H, W))
    w1 = net.band_weights(*net.band_stats(f1, u[:1], ut[:1], K))
    assert np.allclose(w1, net.band_weights(*net.band_stats(fe[:1], u[:1], ut[:1], K)),
                       rtol=1e-12, atol=0)
    L0, _ = net.loss_and_grads(p, fe, u, ut)
    L_zero, _ = net.loss_and_grads({**p, "band.w": np.zeros((K, K))}, fe, u, ut)
    assert L0 < L_zero
    eps = 1e-4
    for _ in range(5):
        d = rng.standard_normal((K, K))
        Lp, _ = net.loss_and_grads({**p, "band.w": p["band.w"] + eps * d}, fe, u, ut)
        Lm, _ = net.loss_and_grads({**p, "band.w": p["band.w"] - eps * d}, fe, u, ut)
        assert Lp > L0 and Lm > L0
        Lz, _ = net.loss_and_grads({**p, "band.w": eps * d}, fe, u, ut)
        assert abs(Lp - Lm) <= 1e-6 * abs(Lz - L_zero)


def test_output_gain_is_the_least_squares_scale_of_the_branch():
    """gate_stats: gamma = <c, t> / |c|^2 minimises |gamma c - t|^2 over the
    off-band part (brute force over a scan of gammas), and with that gamma
    the network's loss off the band is the minimum over gains; gamma = 0
    gives the band-only guess, gamma = 1 the raw network."""
    H, W, K, B = 10, 9, 3, 2
    rng = np.random.default_rng(29)
    p = guess_net_params(31, channels=4, modes=3, zero_last=False, skip_modes=K)
    f = rng.standard_normal((B, H, W))
    u = rng.standard_normal((B, H, W)) * 0.05
    ut = u + rng.standard_normal((B, H, W)) * 0.05
    sct, scc = net.gate_stats(p, f, u, ut)
    g = sct / scc
    losses = [net.loss_and_grads({**p, "band.w": p["band.w"]}, f, u, ut)[0]]
    _, out1, s = net.forward({**p, "gate": 1.0}, f, u)
    t = net.target(ut, u, s)

    def off_loss(gamma):
        _, out, _ = net.forward({**p, "gate": gamma}, f, u)
        d = out - t
        return float(np.sum((d - net.band_project(d, K)) ** 2))
    scan = np.linspace(g - 1.0, g + 1.0, 41)
    assert min(off_loss(x) for x in scan) >= off_loss(g) - 1e-12 * off_loss(g)
    assert off_loss(g) <= off_loss(1.0) and off_loss(g) <= off_loss(0.0)
    # the training loss does not see the gain
    assert net.loss_and_grads({**p, "gate": 0.3}, f, u, ut)[0] == losses[0]
    g0, _, _ = net.forward({**p, "gate": 0.0}, f, u)
    pb = {**p, "conv6.w": np.zeros_like(p["conv6.w"]), "conv6.b": np.zeros_like(p["conv6.b"])}
    gb, _, _ = net.forward(pb, f, u)
    assert np.allclose(g0, gb, rtol=1e-13, atol=1e-15)


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(3)
    p = {"a": rng.standard_normal((4, 5)), "b": rng.standard_normal(3)}
    grads = [{k: rng.standard_normal(v.shape) for k, v in p.items()} for _ in range(10)]
    q = {k: v.copy() for k, v in p.items()}
    st = {}
    net.adam_step(q, grads[0], st, lr=1e-3)
    for k in p:
        step = p[k] - q[k]
        assert np.allclose(step, 1e-3 * grads[0][k] / (np.abs(grads[0][k]) + 1e-8), rtol=1e-12, atol=0)
    for gk in grads[1:]:
        net.adam_step(q, gk, st, lr=1e-3)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(T.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for gk in grads:
        for k, t in T.items():
            t.grad = torch.tensor(gk[k])
        opt.step()
    for k in p:
        assert np.allclose(T[k].detach().numpy(), q[k], rtol=1e-12, atol=1e-15)
