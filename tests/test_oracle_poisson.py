"""Pins of the oracle's Dirichlet Poisson solve and finite differences
(Sec. III.B: fast Poisson solver by a type-I DST plus finite-difference
operators) against a dense direct solve, analytic sine eigenmodes, the
continuum limit and exact polynomial differentiation."""
import numpy as np
import pytest

import workloads as W
from oracle import qsp_oracle as O


def box(nx, ny, lx=3.0, ly=2.0):
    return W.BoxConfig(nx=nx, ny=ny, x_lo=-lx, x_hi=lx, y_lo=-ly, y_hi=ly,
                       nzeta=4, zeta_hi=0.0, dzeta=0.1)


def dense_laplacian(cfg, shift=0.0):
    """5-point Laplacian on the (ny-1)x(nx-1) interior, zero Dirichlet
    neighbours, assembled entry by entry."""
    mx, my = cfg.nx - 1, cfg.ny - 1
    n = mx * my
    A = np.zeros((n, n))
    for j in range(my):
        for i in range(mx):
            r = j * mx + i
            A[r, r] = -2.0 / cfg.hx ** 2 - 2.0 / cfg.hy ** 2 - shift
            if i > 0:
                A[r, r - 1] = 1.0 / cfg.hx ** 2
            if i < mx - 1:
                A[r, r + 1] = 1.0 / cfg.hx ** 2
            if j > 0:
                A[r, r - mx] = 1.0 / cfg.hy ** 2
            if j < my - 1:
                A[r, r + mx] = 1.0 / cfg.hy ** 2
    return A


@pytest.mark.parametrize("nx,ny,shift", [(8, 8, 0.0), (16, 8, 0.0),
                                         (24, 16, 0.0), (16, 16, 1.32)])
def test_poisson_matches_dense_solve(nx, ny, shift):
    cfg = box(nx, ny)
    rng = np.random.default_rng(1)
    src = np.zeros((ny + 1, nx + 1))
    src[1:-1, 1:-1] = rng.normal(size=(ny - 1, nx - 1))
    u = O.poisson_solve(cfg, src, shift)
    ref = np.linalg.solve(dense_laplacian(cfg, shift), src[1:-1, 1:-1].ravel())
    assert np.all(u[0] == 0) and np.all(u[-1] == 0)
    assert np.all(u[:, 0] == 0) and np.all(u[:, -1] == 0)
    err = np.linalg.norm(u[1:-1, 1:-1].ravel() - ref) / np.linalg.norm(ref)
    assert err < 1e-12


def test_sine_modes_are_eigenfunctions():
    cfg = box(32, 16)
    i = np.arange(cfg.nx + 1)
    j = np.arange(cfg.ny + 1)
    for p, q in [(1, 1), (3, 2), (31, 15), (7, 9)]:
        mode = np.sin(np.pi * q * j / cfg.ny)[:, None] * \
            np.sin(np.pi * p * i / cfg.nx)[None, :]
        # apply the 5-point stencil explicitly
        lap = np.zeros_like(mode)
        lap[1:-1, 1:-1] = ((mode[1:-1, 2:] - 2 * mode[1:-1, 1:-1] + mode[1:-1, :-2]) / cfg.hx ** 2 +
                           (mode[2:, 1:-1] - 2 * mode[1:-1, 1:-1] + mode[:-2, 1:-1]) / cfg.hy ** 2)
        lam = O.laplacian_eigenvalues(cfg)[q - 1, p - 1]
        assert np.allclose(lap[1:-1, 1:-1], lam * mode[1:-1, 1:-1], rtol=0,
                           atol=1e-10 * abs(lam))
        u = O.poisson_solve(cfg, mode)
        assert np.abs(u - mode / lam).max() < 1e-13 * np.abs(mode / lam).max()


def test_eigenvalues_continuum_limit():
    # lambda_pq -> -pi^2 (p^2/Lx^2 + q^2/Ly^2) with relative error ~ (pi p h / L)^2 / 12
    for n in (32, 64, 128, 256):
        cfg = box(n, n)
        lam = O.laplacian_eigenvalues(cfg)[1, 2]            # p = 3, q = 2
        Lx, Ly = cfg.x_hi - cfg.x_lo, cfg.y_hi - cfg.y_lo
        cont = -np.pi ** 2 * (3 ** 2 / Lx ** 2 + 2 ** 2 / Ly ** 2)
        bound = max((np.pi * 3 / n) ** 2, (np.pi * 2 / n) ** 2) / 12 * 1.01
        assert abs(lam / cont - 1) < bound


def test_poisson_self_adjoint():
    cfg = box(32, 16)
    rng = np.random.default_rng(2)
    a = O.zero_boundary(rng.normal(size=(cfg.ny + 1, cfg.nx + 1)))
    b = O.zero_boundary(rng.normal(size=(cfg.ny + 1, cfg.nx + 1)))
    l, r = np.sum(a * O.poisson_solve(cfg, b)), np.sum(O.poisson_solve(cfg, a) * b)
    assert abs(l - r) < 1e-12 * abs(l)


def test_dst_matches_brute_force_sine_sum():
    import scipy.fft
    n = 12
    x = np.random.default_rng(3).normal(size=n - 1)
    jj = np.arange(1, n)
    brute = np.array([np.sum(x * np.sin(np.pi * jj * p / n)) for p in range(1, n)])
    assert np.allclose(scipy.fft.dst(x, type=1), 2.0 * brute, atol=1e-12)


def test_fd_exact_on_quadratics_and_antisymmetric():
    cfg = box(16, 12)
    x, y = O.node_coords(cfg)
    X, Y = np.meshgrid(x, y)
    f = 1.5 + 0.3 * X - 0.7 * Y + 0.25 * X * X - 0.4 * X * Y + 0.9 * Y * Y
    dfx = 0.3 + 0.5 * X - 0.4 * Y
    dfy = -0.7 - 0.4 * X + 1.8 * Y
    assert np.allclose(O.ddx(cfg, f)[1:-1, 1:-1], dfx[1:-1, 1:-1], atol=1e-12)
    assert np.allclose(O.ddy(cfg, f)[1:-1, 1:-1], dfy[1:-1, 1:-1], atol=1e-12)
    rng = np.random.default_rng(4)
    a = O.zero_boundary(rng.normal(size=X.shape))
    b = O.zero_boundary(rng.normal(size=X.shape))
    for d in (O.ddx, O.ddy):
        assert abs(np.sum(a * d(cfg, b)) + np.sum(d(cfg, a) * b)) < 1e-12
