"""Batched solves over systems of uneven size and dimension (one graph-replayed
launch sequence for all of them) against the FP64 oracle and against the
one-system solve."""
import numpy as np
import pytest
import torch

from oracle import gmres as og
from synthetic import DriftingGaussians

pytestmark = pytest.mark.gpu

SHAPES = [(40, 56), (64, 64), (23, 31), (12, 14, 10), (16, 16, 16)]


@pytest.fixture(scope="module")
def mlg():
    import paper_2103_10975_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def streams(nrhs, seed):
    out = []
    for i, sh in enumerate(SHAPES):
        g = DriftingGaussians(sh, 3, 0.08, seed=seed + i)
        out.append(np.stack([g.field(t) for t in range(nrhs)]))
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_matches_oracle(mlg, precision):
    print("batched vs oracle", precision, flush=True)
    nrhs, m, tol = 3, 15, 1e-9
    rhs = streams(nrhs, 500)
    guesses = [0, 1, 1, 0, 1]
    bs = [torch.from_numpy(r).cuda() for r in rhs]
    xs = [torch.zeros_like(b) for b in bs]
    systems = [mlg.make_system(b, x, gs) for b, x, gs in zip(bs, xs, guesses)]
    opts = mlg.Opts(restart_m=m, rtol=tol, precision=precision)
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    stats = mlg.gmres_solve_batched(systems, opts, ws)
    torch.cuda.synchronize()
    assert len(stats) == nrhs * len(SHAPES)
    k = 0
    for s_i, (r, x, gs) in enumerate(zip(rhs, xs, guesses)):
        xo_prev = np.zeros(r.shape[1:])
        for t in range(nrhs):
            st = stats[k]
            k += 1
            x0 = xo_prev if (gs == 1 and t > 0) else np.zeros(r.shape[1:])
            xo, so = og.gmres(r[t], x0, m=m, rtol=tol)
            xo_prev = xo
            xg = x[t].cpu().numpy()
            rn, bn = og.residual_norm(r[t], xg)
            assert st.status == 0 and rn <= tol * bn, (s_i, t)
            assert rel(xg, xo) <= (1e-8 if precision == 0 else 1e-5), (s_i, t)
            if precision == 0:
                assert abs(st.iters - so.iters) <= 2, (s_i, t, st.iters, so.iters)


def test_batched_equals_single(mlg):
    print("batched vs single", flush=True)
    nrhs, m, tol = 2, 12, 1e-11
    rhs = streams(nrhs, 900)
    bs = [torch.from_numpy(r).cuda() for r in rhs]
    xs = [torch.zeros_like(b) for b in bs]
    systems = [mlg.make_system(b, x, 1) for b, x in zip(bs, xs)]
    opts = mlg.Opts(restart_m=m, rtol=tol)
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    stats = mlg.gmres_solve_batched(systems, opts, ws)
    k = 0
    for b, x in zip(bs, xs):
        grid = mlg.grid_of(b.shape[1:])
        ws1 = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
        prev = torch.zeros_like(b[0])
        for t in range(nrhs):
            x1 = prev.clone()
            st1 = mlg.gmres_solve(grid, b[t].contiguous(), x1, opts, ws1)
            assert abs(st1.iters - stats[k].iters) <= 2
            assert rel(x[t].cpu().numpy(), x1.cpu().numpy()) <= 1e-9
            prev = x1
            k += 1


def test_batched_split_form_matches_fused(mlg):
    """A batch of 2D and 3D systems with the split form: the 2D group sums its
    partials over workgroups while the 3D group keeps one coef launch per
    system; every solution matches the fused form bitwise."""
    print("batched split", flush=True)
    nrhs, m, tol = 2, 12, 1e-10
    rhs = streams(nrhs, 700)
    out = []
    for schedule in (2, 3):
        bs = [torch.from_numpy(r).cuda() for r in rhs]
        xs = [torch.zeros_like(b) for b in bs]
        systems = [mlg.make_system(b, x, 1) for b, x in zip(bs, xs)]
        opts = mlg.Opts(restart_m=m, rtol=tol, schedule=schedule)
        ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
        stats = mlg.gmres_solve_batched(systems, opts, ws)
        out.append(([x.cpu().numpy() for x in xs], [(s.iters, s.status) for s in stats]))
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("schedule", [0, 3])
def test_batched_edge_cases(mlg, schedule):
    print("batched edges", schedule, flush=True)
    # a zero right-hand side, an exactly solvable one and a NaN guess in one batch
    sh = (20, 24)
    g = DriftingGaussians(sh, 2, 0.1, seed=1)
    b = torch.from_numpy(np.stack([np.zeros(sh), g.field(1), g.field(2)])).cuda()
    x = torch.zeros_like(b)
    x[0] = 1.0
    b2 = torch.from_numpy(g.field(3)[None]).cuda()
    x2 = torch.zeros_like(b2)
    x2[0, 3, 3] = float("nan")
    systems = [mlg.make_system(b, x, 0), mlg.make_system(b2, x2, 0)]
    opts = mlg.Opts(restart_m=10, rtol=1e-8, schedule=schedule)
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    with pytest.raises(mlg.MlgError) as e:
        mlg.gmres_solve_batched(systems, opts, ws)
    assert e.value.code == mlg.MLG_ERR_NONFINITE
    # the healthy system still finished every right-hand side
    assert torch.all(x[0] == 0)
    for t in (1, 2):
        rn, bn = og.residual_norm(b[t].cpu().numpy(), x[t].cpu().numpy())
        assert rn <= 1e-8 * bn


LARGE = [(256, 256), (200, 136), (97, 161), (36, 40, 70), (64, 64, 64)]


def dirichlet_eigs(shape):
    """Eigenvalues of -lap_h on each axis with zero Dirichlet boundary and
    h = 1/(n+1): (4/h^2) sin^2(j pi h / 2), j = 1..n."""
    out = []
    for n in shape:
        h = 1.0 / (n + 1)
        j = np.arange(1, n + 1)
        out.append(4.0 / h ** 2 * np.sin(j * np.pi * h / 2) ** 2)
    return out


def spectral_solve(b):
    """Exact solution of -lap_h x = b: the orthonormal DST-I diagonalises the
    operator on every axis."""
    from scipy.fft import dstn, idstn
    eig = dirichlet_eigs(b.shape)
    lam = eig[0].reshape((-1,) + (1,) * (b.ndim - 1))
    for a in range(1, b.ndim):
        shp = [1] * b.ndim
        shp[a] = -1
        lam = lam + eig[a].reshape(shp)
    return idstn(dstn(b, type=1, norm="ortho") / lam, type=1, norm="ortho"), float(lam.max() / lam.min())


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_large_systems_to_tolerance(mlg, precision):
    """Systems of up to 256^2 and 64^3 with ragged tails on every tiled axis,
    solved together over two right-hand sides (some from the previous
    solution): every solution meets the FP64 residual bound, lies within
    cond(A) * relres of the exact DST solution, and matches the one-system
    solve from the same guess within the bound that both solutions imply."""
    print("batched large", precision, flush=True)
    nrhs, m, tol = 2, 30, 1e-8
    rhs = []
    for i, sh in enumerate(LARGE):
        g = DriftingGaussians(sh, 3, 0.08, seed=1200 + i)
        rhs.append(np.stack([g.field(t) for t in range(nrhs)]))
    guesses = [1, 0, 1, 0, 1]
    bs = [torch.from_numpy(r).cuda() for r in rhs]
    xs = [torch.zeros_like(b) for b in bs]
    systems = [mlg.make_system(b, x, gs) for b, x, gs in zip(bs, xs, guesses)]
    opts = mlg.Opts(restart_m=m, rtol=tol, precision=precision)
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    stats = mlg.gmres_solve_batched(systems, opts, ws)
    torch.cuda.synchronize()
    assert len(stats) == nrhs * len(LARGE)
    k = 0
    for s_i, (r, b, x, gs) in enumerate(zip(rhs, bs, xs, guesses)):
        grid = mlg.grid_of(b.shape[1:])
        ws1 = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
        prev = torch.zeros_like(b[0])
        for t in range(nrhs):
            st = stats[k]
            k += 1
            xg = x[t].cpu().numpy()
            rn, bn = og.residual_norm(r[t], xg)
            assert st.status == 0 and rn <= tol * bn, (s_i, t, rn / bn)
            xe, cond = spectral_solve(r[t])
            assert rel(xg, xe) <= cond * rn / bn * (1 + 1e-6) + 1e-12, (s_i, t)
            x1 = prev.clone() if (gs == 1 and t > 0) else torch.zeros_like(b[0])
            st1 = mlg.gmres_solve(grid, b[t].contiguous(), x1, opts, ws1)
            x1n = x1.cpu().numpy()
            rn1, _ = og.residual_norm(r[t], x1n)
            assert st1.status == 0 and rn1 <= tol * bn
            assert rel(xg, x1n) <= cond * (rn + rn1) / bn * 1.01, (s_i, t)
            # the same arithmetic in another order: within a few restart cycles
            assert abs(st1.iters - st.iters) <= max(2 * m, st.iters // 20), (s_i, t, st.iters, st1.iters)
            prev = x[t].clone()
