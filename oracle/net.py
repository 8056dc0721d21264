"""NumPy FP64 oracle for the learned initial guess (test infrastructure only).

The paper (Section 2, "A Real-Time AI-Based Acceleration Algorithm") feeds the
network's output to GMRES(k) as the initial guess x0 = N(b), trains it on the
(RHS, solution) pairs GMRES produces with the squared 2-norm loss
L = |x_tilde - x|_2^2 (Section 2.3), by back-propagation and an adaptive
gradient method such as ADAM.  Its Section 2.1 asks for a network that can
represent non-local relations (the inverse of the discrete Laplacian is
dense) without compressing resolution.

The network built here (readings where the paper is silent are listed in the
design notes of the repository):
  inputs   (r / s_r, f / s_f): r = f - A u_prev, the residual of the previous
           solution formed in FP64 by the discrete Laplacian A (a fixed first
           layer), s_r = RMS(r), s_f = RMS(f) (a zero scale is replaced by 1
           for the division)
  L1 conv3x3 2->C + ReLU;  L2 conv3x3 C->C + ReLU
  L3 spectral: ReLU(W1 x + b + S^-1[W_kl . S[x]_kl]) on the M x M slowest
     sine modes (S = the DST-I basis sin(k pi i/(N+1)), k = 1..M), per-mode
     C x C channel mixing
  L4, L5 conv3x3 C->C + ReLU;  L6 conv3x3 C->1
  band     S^-1[w_kl S[r / s_r]_kl] on the K x K slowest sine modes (the
           band; K = 0 switches it off): a linear spectral path whose
           per-mode weights w are learned from the solver's pairs, as the
           least-squares minimiser of the loss over those weights,
           w_kl = sum X T / sum X^2 over the training samples seen (X, T the
           band coefficients of the right-hand side the correction
           u_t - u_prev solves exactly and of the target; see band_stats)
  out = gamma (L6 - P_K L6) + band, P_K the orthogonal projection on the
        K x K modes: the band path alone sets the output there, the
        convolutional branch the rest, scaled by its output gain gamma (the
        least-squares gain of that branch against the off-band targets of
        recent training batches, see gate_stats; 1 while training and while
        no batch has been seen)
  guess = u_prev + (s_r / c_u) * out, c_u = 2 pi^2
Convolutions are cross-correlations with zero padding (the Dirichlet zero),
weights in [out, in, ky, kx] layout.  Everything is float64, NCHW, written
from the definitions (numpy tensordot is the only library primitive).
"""
from __future__ import annotations

import numpy as np

from . import gmres as _gmres

C_U = 2.0 * np.pi ** 2


# ---------------------------------------------------------------- pieces
def _rms(a: np.ndarray) -> np.ndarray:
    return np.sqrt(np.mean(a.reshape(a.shape[0], -1) ** 2, axis=1))


def normalise(f: np.ndarray, u_prev: np.ndarray):
    """Network input.  f, u_prev: [B, H, W] -> x [B, 2, H, W], s_r [B] (output
    scale: RMS of the residual of u_prev) and s_in [B] (its input scale)."""
    r = np.stack([f[b] - _gmres.apply(u_prev[b]) for b in range(f.shape[0])])
    s_r = _rms(r)
    s_in = np.where(s_r > 0.0, s_r, 1.0)
    s_f = _rms(f)
    s_f = np.where(s_f > 0.0, s_f, 1.0)
    x = np.stack([r / s_in[:, None, None], f / s_f[:, None, None]], axis=1)
    return x, s_r, s_in


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b,d,i,j] = b[d] + sum_{c,p,q} w[d,c,p,q] x[b,c,i+p-1,j+q-1], x = 0 outside."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, w.shape[0], H, W)) + b[None, :, None, None]
    for p in range(3):
        for q in range(3):
            # [B, Ci, H, W] x [Co, Ci] -> [B, H, W, Co]
            y += np.moveaxis(np.tensordot(xp[:, :, p:p + H, q:q + W], w[:, :, p, q],
                                          axes=([1], [1])), 3, 1)
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for p in range(3):
        for q in range(3):
            # dx[b,c,i+p-1,j+q-1] += sum_d w[d,c,p,q] dy[b,d,i,j]
            dxp[:, :, p:p + H, q:q + W] += np.moveaxis(
                np.tensordot(dy, w[:, :, p, q], axes=([1], [0])), 3, 1)
            # dw[d,c,p,q] = sum_{b,i,j} dy[b,d,i,j] x[b,c,i+p-1,j+q-1]
            dw[:, :, p, q] = np.tensordot(dy, xp[:, :, p:p + H, q:q + W],
                                          axes=([0, 2, 3], [0, 2, 3]))
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dw, db


def sine_basis(n: int, modes: int) -> np.ndarray:
    """S[k, i] = sin((k+1) pi (i+1) / (n+1)), k < modes, i < n: the first
    eigenvectors of the 1D zero-Dirichlet second difference."""
    k = np.arange(1, modes + 1, dtype=np.float64)[:, None]
    i = np.arange(1, n + 1, dtype=np.float64)[None, :]
    return np.sin(k * np.pi * i / (n + 1))


def spectral_forward(x, w1, b, wk):
    """Returns (y, cache).  x [B, C, H, W]; wk [M, M, C, C] = [ky, kx, out, in]."""
    B, C, H, W = x.shape
    M = wk.shape[0]
    Sy, Sx = sine_basis(H, M), sine_basis(W, M)
    norm = (2.0 / (H + 1)) * (2.0 / (W + 1))
    # forward transform X[b,c,k,l] = sum_{i,j} Sy[k,i] Sx[l,j] x[b,c,i,j]
    X = np.einsum("ki,bcij,lj->bckl", Sy, x, Sx, optimize=True)
    # per-mode channel mixing Y[b,d,k,l] = sum_c wk[k,l,d,c] X[b,c,k,l]
    Y = np.einsum("kldc,bckl->bdkl", wk, X, optimize=True)
    # inverse on the retained modes, scaled so a full basis would invert exactly
    ys = norm * np.einsum("ki,bdkl,lj->bdij", Sy, Y, Sx, optimize=True)
    z = np.einsum("dc,bcij->bdij", w1, x, optimize=True) + b[None, :, None, None] + ys
    return np.maximum(z, 0.0), (x, X, z, Sy, Sx, norm)


def spectral_backward(w1, wk, cache, dy):
    x, X, z, Sy, Sx, norm = cache
    dz = dy * (z > 0.0)
    dw1 = np.einsum("bdij,bcij->dc", dz, x, optimize=True)
    db = dz.sum(axis=(0, 2, 3))
    dx = np.einsum("dc,bdij->bcij", w1, dz, optimize=True)
    dY = norm * np.einsum("ki,bdij,lj->bdkl", Sy, dz, Sx, optimize=True)
    dwk = np.einsum("bdkl,bckl->kldc", dY, X, optimize=True)
    dX = np.einsum("kldc,bdkl->bckl", wk, dY, optimize=True)
    dx += np.einsum("ki,bckl,lj->bcij", Sy, dX, Sx, optimize=True)
    return dx, dw1, db, dwk


def band_weights(sxt: np.ndarray, sxx: np.ndarray) -> np.ndarray:
    """Per-mode band weights from the running sums: sxt / sxx, 0 where no
    sample has touched the mode (sxx = 0)."""
    safe = np.where(sxx > 0.0, sxx, 1.0)
    return np.where(sxx > 0.0, sxt / safe, 0.0)


def skip_forward(x_r: np.ndarray, w: np.ndarray):
    """Band path.  x_r [B, H, W] (residual channel), w [K, K] -> (out [B, H, W], X)
    with X [B, K, K] the band coefficients of x_r."""
    B, H, W = x_r.shape
    K = w.shape[0]
    Sy, Sx = sine_basis(H, K), sine_basis(W, K)
    norm = (2.0 / (H + 1)) * (2.0 / (W + 1))
    X = np.einsum("ki,bij,lj->bkl", Sy, x_r, Sx, optimize=True)
    out = norm * np.einsum("ki,bkl,lj->bij", Sy, w[None] * X, Sx, optimize=True)
    return out, X


def band_project(y: np.ndarray, K: int) -> np.ndarray:
    """P_K y: the orthogonal projection of y [B, H, W] on the K x K slowest
    sine modes (orthonormal rows sqrt(2/(n+1)) S)."""
    B, H, W = y.shape
    Sy, Sx = sine_basis(H, K), sine_basis(W, K)
    norm = (2.0 / (H + 1)) * (2.0 / (W + 1))
    Y = np.einsum("ki,bij,lj->bkl", Sy, y, Sx, optimize=True)
    return norm * np.einsum("ki,bkl,lj->bij", Sy, Y, Sx, optimize=True)


def band_stats(f: np.ndarray, u_prev: np.ndarray, u_target: np.ndarray, K: int):
    """The per-mode sums a training batch adds to the band's least-squares
    state: (sum_b X_b T_b, sum_b X_b^2) [K, K].  The pair is made exact: the
    solver's u_t solves A u_t = f_t - r_fin exactly (r_fin its final
    residual), so the correction d = u_t - u_prev solves A d = r - r_fin,
    r = f_t - A u_prev; X_b = S[A d_b / s_b] and T_b = S[t_b] are the band
    coefficients of that right-hand side and of the target t_b = c_u d_b / s_b
    (unnormalised sine basis, s_b the input scale of the sample).  The band's
    share of the loss on these pairs, norm * sum_b sum_kl (w_kl X_b - T_b)^2,
    is minimal at w = sum X T / sum X^2, mode by mode, since the orthonormal
    sine modes decouple."""
    _, _, s = normalise(f, u_prev)
    d = u_target - u_prev
    t = target(u_target, u_prev, s)
    ad = np.stack([_gmres.apply(db) for db in d]) / s[:, None, None]
    H, W = f.shape[1:]
    Sy, Sx = sine_basis(H, K), sine_basis(W, K)
    X = np.einsum("ki,bij,lj->bkl", Sy, ad, Sx, optimize=True)
    T = np.einsum("ki,bij,lj->bkl", Sy, t, Sx, optimize=True)
    return np.sum(X * T, axis=0), np.sum(X * X, axis=0)


def gate_stats(params: dict, f, u_prev, u_target):
    """The sums a training batch adds to the output gain's least-squares
    state: (sum_b <c_b, t_b>, sum_b |c_b|^2) with c_b the convolutional
    branch's output off the band (L6 - P_K L6) and t_b the target off the
    band; gamma = their ratio minimises sum_b |gamma c_b - t_b|^2.  Requires
    a band path (K > 0)."""
    K = band_modes(params)
    _, _, s, c = forward({**params, "gate": 1.0}, f, u_prev, keep=True)
    c6 = conv3x3(c["a5"], params["conv6.w"], params["conv6.b"])[:, 0]
    co = c6 - band_project(c6, K)
    t = target(u_target, u_prev, s)
    to = t - band_project(t, K)
    return float(np.sum(co * to)), float(np.sum(co * co))


# ---------------------------------------------------------------- network
def band_modes(params: dict) -> int:
    """K of the band path (0: no band path)."""
    w = params.get("band.w")
    return 0 if w is None else int(w.shape[0])


def forward(params: dict, f: np.ndarray, u_prev: np.ndarray, keep: bool = False):
    """f, u_prev: [B, H, W] float64.  Returns (guess [B, H, W], out [B, H, W]
    in normalised units, s_in [B][, cache])."""
    x0, s_r, s = normalise(f, u_prev)
    c = {"x0": x0}
    a1 = np.maximum(conv3x3(x0, params["conv1.w"], params["conv1.b"]), 0.0)
    a2 = np.maximum(conv3x3(a1, params["conv2.w"], params["conv2.b"]), 0.0)
    a3, sc = spectral_forward(a2, params["spec.w1"], params["spec.b"], params["spec.wk"])
    a4 = np.maximum(conv3x3(a3, params["conv4.w"], params["conv4.b"]), 0.0)
    a5 = np.maximum(conv3x3(a4, params["conv5.w"], params["conv5.b"]), 0.0)
    c6 = conv3x3(a5, params["conv6.w"], params["conv6.b"])[:, 0]
    K = band_modes(params)
    out = c6
    if K > 0:
        band, _ = skip_forward(x0[:, 0], params["band.w"])
        out = params.get("gate", 1.0) * (c6 - band_project(c6, K)) + band
    guess = u_prev + (s_r / C_U)[:, None, None] * out
    if keep:
        c.update(a1=a1, a2=a2, a3=a3, a4=a4, a5=a5, spec=sc)
        return guess, out, s, c
    return guess, out, s


def target(u_target: np.ndarray, u_prev: np.ndarray, s: np.ndarray) -> np.ndarray:
    """The GMRES solution expressed in the network's output units."""
    return C_U * (u_target - u_prev) / s[:, None, None]


def loss_and_grads(params: dict, f, u_prev, u_target):
    """L = (1/B) sum_b |out_b - t_b|_2^2 and its gradient for every parameter
    trained by gradient (all but the band weights and the output gain; the
    convolutional branch trains on its raw output, gain 1)."""
    B = f.shape[0]
    _, out, s, c = forward({**params, "gate": 1.0}, f, u_prev, keep=True)
    t = target(u_target, u_prev, s)
    diff = out - t
    loss = float(np.sum(diff ** 2) / B)
    g = {}
    d6 = (2.0 / B) * diff[:, None]
    K = band_modes(params)
    if K > 0:
        # the projection is symmetric: the conv branch sees the gradient off
        # the band (the band weights are fitted by band_stats, not by gradient)
        d6 = d6 - band_project(d6[:, 0], K)[:, None]
    d5, g["conv6.w"], g["conv6.b"] = conv3x3_backward(c["a5"], params["conv6.w"], d6)
    d5 = d5 * (c["a5"] > 0.0)
    d4, g["conv5.w"], g["conv5.b"] = conv3x3_backward(c["a4"], params["conv5.w"], d5)
    d4 = d4 * (c["a4"] > 0.0)
    d3, g["conv4.w"], g["conv4.b"] = conv3x3_backward(c["a3"], params["conv4.w"], d4)
    d2, g["spec.w1"], g["spec.b"], g["spec.wk"] = spectral_backward(
        params["spec.w1"], params["spec.wk"], c["spec"], d3)
    d2 = d2 * (c["a2"] > 0.0)
    d1, g["conv2.w"], g["conv2.b"] = conv3x3_backward(c["a1"], params["conv2.w"], d2)
    d1 = d1 * (c["a1"] > 0.0)
    _, g["conv1.w"], g["conv1.b"] = conv3x3_backward(c["x0"], params["conv1.w"], d1)
    return loss, g


def adam_step(params: dict, grads: dict, state: dict, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, with bias correction), in place.
    state holds 't' and per-parameter 'm.<name>', 'v.<name>'."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k, gk in grads.items():
        m = state.get("m." + k, np.zeros_like(gk))
        v = state.get("v." + k, np.zeros_like(gk))
        m = beta1 * m + (1.0 - beta1) * gk
        v = beta2 * v + (1.0 - beta2) * gk * gk
        state["m." + k], state["v." + k] = m, v
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params
