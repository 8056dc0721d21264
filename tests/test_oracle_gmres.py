"""Pins for the FP64 GMRES oracle, independent of the oracle itself.

Each check is fixed by mathematics rather than by re-running the oracle's own
formulas: closed-form eigenpairs of the Dirichlet Laplacian, a dense direct
solve, finite termination on invariant subspaces, the Arnoldi relations, an
explicit Krylov least-squares solve, and SciPy's GMRES.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import gmres as og
from synthetic import DriftingGaussians


def dense_operator(shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = og.apply(e.reshape(shape)).ravel()
    return A


def lam_1d(k, n):
    h = 1.0 / (n + 1)
    return (4.0 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2


def mode(shape, ks):
    """sin(k pi x) sin(l pi y) [sin(m pi z)] on the interior grid; ks in (x, y[, z])."""
    axes = [np.sin(k * np.pi * np.arange(1, n + 1) / (n + 1))
            for k, n in zip(ks, reversed(shape))]
    if len(shape) == 2:
        return np.outer(axes[1], axes[0])
    return axes[2][:, None, None] * axes[1][None, :, None] * axes[0][None, None, :]


def mode_eig(shape, ks):
    return sum(lam_1d(k, n) for k, n in zip(ks, reversed(shape)))


def sparse_laplacian(shape):
    mats = []
    for n in reversed(shape):                     # x, y[, z]
        h = 1.0 / (n + 1)
        mats.append(sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / h ** 2)
    eyes = [sp.identity(n) for n in reversed(shape)]
    if len(shape) == 2:
        return (sp.kron(eyes[1], mats[0]) + sp.kron(mats[1], eyes[0])).tocsr()
    return (sp.kron(sp.kron(eyes[2], eyes[1]), mats[0]) + sp.kron(sp.kron(eyes[2], mats[1]), eyes[0])
            + sp.kron(sp.kron(mats[2], eyes[1]), eyes[0])).tocsr()


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("shape", [(8, 8), (5, 7), (4, 4, 4), (3, 4, 5)])
def test_operator_dense_spd_and_spectrum(shape):
    A = dense_operator(shape)
    assert np.array_equal(A, A.T)
    ev = np.sort(np.linalg.eigvalsh(A))
    grids = np.meshgrid(*[np.arange(1, n + 1) for n in reversed(shape)], indexing="ij")
    closed = np.sort(sum(lam_1d(g.ravel(), n) for g, n in zip(grids, reversed(shape))))
    assert np.max(np.abs(ev - closed)) <= 1e-12 * closed.max()
    assert ev.min() > 0


@pytest.mark.parametrize("shape,ks", [((64, 64), (3, 5)), ((33, 20), (1, 7)), ((16, 16, 16), (2, 1, 3))])
def test_operator_eigenvectors(shape, ks):
    phi = mode(shape, ks)
    lam = mode_eig(shape, ks)
    assert np.max(np.abs(og.apply(phi) - lam * phi)) <= 1e-13 * lam


def test_operator_matches_kronecker_sum():
    rng = np.random.default_rng(3)
    for shape in [(9, 13), (6, 5, 7)]:
        u = rng.standard_normal(shape)
        ref = sparse_laplacian(shape) @ u.ravel()
        assert np.allclose(og.apply(u).ravel(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------- GMRES
@pytest.mark.parametrize("shape,m", [((8, 8), 20), ((6, 8), 5), ((4, 4, 4), 10), ((3, 5, 4), 3)])
@pytest.mark.parametrize("ortho", ["cgs2", "mgs"])
def test_gmres_matches_dense_solve(shape, m, ortho):
    rng = np.random.default_rng(11)
    b = rng.standard_normal(shape)
    x, st = og.gmres(b, m=m, rtol=1e-13, ortho=ortho)
    ref = np.linalg.solve(dense_operator(shape), b.ravel())
    assert st.status == 0
    assert np.linalg.norm(x.ravel() - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,ks", [((64, 64), (3, 5)), ((128, 96), (1, 1)), ((20, 20, 20), (2, 3, 1))])
def test_eigenvector_rhs_one_iteration(shape, ks):
    phi = mode(shape, ks)
    x, st = og.gmres(mode_eig(shape, ks) * phi, m=20, rtol=1e-8)
    assert st.iters == 1 and st.status == 0
    assert np.max(np.abs(x - phi)) <= 1e-14 * 10


def test_finite_termination_distinct_eigenvalues():
    # Modes from the top of the spectrum: A then amplifies the signal at least as
    # much as the rounding noise in every other eigendirection, so the Krylov
    # space stays numerically 5-dimensional.
    shape = (48, 48)
    modes_ = [(48, 48), (47, 45), (40, 44), (46, 30), (44, 44)]   # 5 distinct eigenvalues
    lams = [mode_eig(shape, k) for k in modes_]
    assert len(set(np.round(lams, 6))) == 5
    rng = np.random.default_rng(5)
    coef = rng.uniform(0.5, 2.0, size=5)
    u = sum(c * mode(shape, k) for c, k in zip(coef, modes_))
    x, st = og.gmres(og.apply(u), m=10, rtol=1e-12)
    assert st.iters <= 5 and st.status == 0
    assert np.max(np.abs(x - u)) <= 1e-11 * np.abs(u).max()


@pytest.mark.parametrize("shape,k", [((24, 24), 20), ((10, 10, 10), 12)])
@pytest.mark.parametrize("ortho", ["cgs2", "mgs"])
def test_arnoldi_relations(shape, k, ortho):
    rng = np.random.default_rng(7)
    r0 = rng.standard_normal(shape)
    V, H, steps = og.arnoldi(r0, k, ortho)
    assert steps == k
    assert np.max(np.abs(V @ V.T - np.eye(k + 1))) < 1e-12
    AV = np.stack([og.apply(V[i].reshape(shape)).ravel() for i in range(k)])   # rows = A v_i
    lam_max = mode_eig(shape, tuple(n for n in reversed(shape)))
    rel = np.linalg.norm(AV.T - V.T @ H) / (lam_max * np.linalg.norm(V[:k]))
    assert rel < 1e-12
    assert np.allclose(np.triu(H, -1), H)                      # Hessenberg
    # A symmetric: the Hessenberg is tridiagonal up to rounding
    assert np.max(np.abs(np.triu(H[:k], 2))) < 1e-8 * lam_max


def test_first_cycle_equals_krylov_least_squares():
    shape = (8, 8)
    A = dense_operator(shape)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    r0 = b.ravel() - A @ x0.ravel()
    for k in range(1, 9):
        K = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, r0, rcond=None)
        ref = x0.ravel() + Q @ y
        x, st = og.gmres(b, x0, m=8, fixed_iters=k)
        assert st.iters == k
        assert np.linalg.norm(x.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_residual_monotone_and_estimate_tracks_true():
    g = DriftingGaussians((48, 48), 3, 0.05, seed=1000)
    b = g.field(0)
    m = 20
    x, st, hist = og.gmres(b, m=m, rtol=1e-10, history=True)
    assert st.status == 0
    # within every cycle the Givens estimate never increases
    for c0 in range(0, len(hist) - 1, m):
        seg = hist[c0: c0 + m + 1]
        assert np.all(np.diff(seg) <= 1e-15 * seg[0])
    # restarts: estimates continue from the true residual and keep decreasing
    assert np.all(np.diff(hist[::m]) <= 0)
    rn, bn = og.residual_norm(b, x)
    assert abs(rn / bn - st.relres_true) <= 1e-8 * st.relres_true
    assert abs(st.relres_est - st.relres_true) <= 1e-6 * st.relres_true + 1e-14


def test_matches_scipy_gmres_and_error_bound():
    shape = (40, 40)
    b = DriftingGaussians(shape, 3, 0.05, seed=1000).field(2)
    A = sparse_laplacian(shape)
    tol, m = 1e-10, 20
    x, st = og.gmres(b, m=m, rtol=tol)
    xs, info = spla.gmres(A, b.ravel(), rtol=tol, atol=0.0, restart=m, maxiter=10 ** 5)
    assert info == 0
    exact = spla.spsolve(A.tocsc(), b.ravel())
    kappa = mode_eig(shape, (40, 40)) / mode_eig(shape, (1, 1))
    for sol in (x.ravel(), xs):
        assert np.linalg.norm(sol - exact) <= kappa * tol * np.linalg.norm(exact)
    assert np.linalg.norm(x.ravel() - xs) <= 2 * kappa * tol * np.linalg.norm(exact)


def test_cgs2_and_mgs_same_trajectory():
    b = DriftingGaussians((64, 64), 3, 0.05, seed=1000).field(0)
    x1, s1 = og.gmres(b, m=20, rtol=1e-8, ortho="cgs2")
    x2, s2 = og.gmres(b, m=20, rtol=1e-8, ortho="mgs")
    assert abs(s1.iters - s2.iters) <= 1
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)


def test_edge_cases():
    z = np.zeros((6, 6))
    x, st = og.gmres(z, np.ones((6, 6)), m=5)
    assert st.iters == 0 and np.all(x == 0)
    b = DriftingGaussians((16, 16), 2, 0.1, seed=3).field(0)
    x, st = og.gmres(b, m=5, rtol=1e-12, max_iters=7)
    assert st.status == 1 and st.iters == 7
    xs, _ = og.gmres(b, m=5, rtol=1e-12)
    x2, st2 = og.gmres(b, xs, m=5, rtol=1e-8)                # already converged guess
    assert st2.iters == 0 and np.array_equal(x2, xs)
    # restart length 1 still converges (steepest-descent-like GMRES(1) on SPD)
    x1, st1 = og.gmres(DriftingGaussians((6, 6), 1, 0.2, seed=4).field(0), m=1, rtol=1e-8)
    assert st1.status == 0


def test_thread_count_does_not_change_results():
    """The oracle's OpenMP loops and fixed-chunk dot products give bitwise the
    same GMRES trajectory with 1 and with several threads (2D and 3D)."""
    from synthetic import DriftingGaussians
    for shape in [(70, 90), (20, 24, 18)]:
        b = DriftingGaussians(shape, 3, 0.05, seed=12).field(0)
        out = []
        for nt in (1, 4):
            og.set_threads(nt)
            x, st = og.gmres(b, m=20, fixed_iters=95)
            out.append((x, st))
        og.set_threads(1)
        assert np.array_equal(out[0][0], out[1][0])
        assert out[0][1] == out[1][1]
