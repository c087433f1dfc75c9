"""Pins of the oracle's geometric multigrid (not gpu)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import grid, multigrid


@pytest.mark.parametrize("n", [6, 7, 32, 33])
def test_interpolation_is_piecewise_linear(n):
    h = 1.0 / (n + 1)
    xf = (np.arange(n) + 1) * h
    nc = multigrid.coarse_size(n)
    xc = xf[1::2][:nc]
    g = np.sin(3.0 * xc) + xc ** 2
    P = multigrid.interpolation_1d(n)
    ref = np.interp(xf, np.concatenate([[0.0], xc, [1.0]]), np.concatenate([[0.0], g, [0.0]]))
    assert np.allclose(P @ g, ref, atol=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 64), (2, 53), (3, 16)])
def test_galerkin_levels_are_kronecker_sums(dim, n):
    """Constant coefficients: A_l = kron(M..) + a sum kron(..T..M..) with 1D Galerkin factors."""
    a = 0.37
    K = grid.stiffness(n, dim)
    H = multigrid.Hierarchy(K, n, dim, a)
    h = 1.0 / (n + 1)
    M1 = sp.identity(n, format="csr")
    T1 = grid.stiffness(n, 1)
    assert H.levels >= 3
    assert H.sizes[-1] ** dim <= 256 < H.sizes[-2] ** dim
    for lev in range(1, min(3, H.levels)):
        P1 = multigrid.interpolation_1d(H.sizes[lev - 1])
        M1 = (P1.T @ M1 @ P1) / 2.0
        T1 = (P1.T @ T1 @ P1) / 2.0
        if dim == 2:
            ref = sp.kron(M1, M1) + a * (sp.kron(M1, T1) + sp.kron(T1, M1))
        else:
            ref = (sp.kron(sp.kron(M1, M1), M1)
                   + a * (sp.kron(sp.kron(T1, M1), M1) + sp.kron(sp.kron(M1, T1), M1)
                          + sp.kron(sp.kron(M1, M1), T1)))
        assert abs(ref - H.ops[lev]).max() <= 1e-12 * abs(ref).max()
    assert h > 0


@pytest.mark.parametrize("dim,n,a", [(2, 32, 0.004), (2, 24, 0.3), (3, 12, 0.01)])
def test_cycles_converge_to_direct_solve(dim, n, a):
    K = grid.stiffness(n, dim)
    H = multigrid.Hierarchy(K, n, dim, a)
    b = np.random.default_rng(5).standard_normal(n ** dim)
    xd = spla.spsolve(H.ops[0].tocsc(), b)
    x = multigrid.solve(H, b, cycles=40, omega=0.8 if dim == 2 else 6 / 7)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("dim,n,a", [(2, 64, 1 / 64 * 0.2), (3, 16, 1 / 32 * 0.2)])
def test_contraction_factor(dim, n, a):
    K = grid.stiffness(n, dim)
    H = multigrid.Hierarchy(K, n, dim, a)
    b = np.random.default_rng(6).standard_normal(n ** dim)
    xd = spla.spsolve(H.ops[0].tocsc(), b)
    omega = 0.8 if dim == 2 else 6 / 7
    e1 = np.linalg.norm(multigrid.solve(H, b, 4, omega) - xd)
    e2 = np.linalg.norm(multigrid.solve(H, b, 5, omega) - xd)
    assert e2 / e1 < 0.5


@pytest.mark.parametrize("n,coarse_max", [(64, 1024), (70, 1024), (33, 64)])
def test_coarse_max_sets_the_exact_level_and_cycles_still_converge(n, coarse_max):
    K = grid.stiffness(n, 2)
    H = multigrid.Hierarchy(K, n, 2, 0.05, coarse_max=coarse_max)
    assert H.sizes[-1] ** 2 <= coarse_max < H.sizes[-2] ** 2
    b = np.random.default_rng(9).standard_normal(n * n)
    xd = spla.spsolve(H.ops[0].tocsc(), b)
    x = multigrid.solve(H, b, cycles=40, omega=0.8)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # one level only: the cycle is the exact solve
    H1 = multigrid.Hierarchy(grid.stiffness(16, 2), 16, 2, 0.3, coarse_max=256)
    b1 = np.random.default_rng(10).standard_normal(256)
    assert H1.levels == 1
    assert np.allclose(multigrid.vcycle(H1, b1), spla.spsolve(H1.ops[0].tocsc(), b1), rtol=1e-12, atol=1e-12)
