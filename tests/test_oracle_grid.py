"""Pins of the oracle's finite-difference stiffness matrix (not gpu)."""
import itertools

import numpy as np
import pytest

from oracle import grid


def _hand_apply(n, dim, kappa, u):
    """(K u)_p by looping over nodes and their 2*dim neighbours (pure Python)."""
    h = 1.0 / (n + 1)
    shape = (n,) * dim
    U = u.reshape(shape)
    Kp = kappa.reshape(shape)
    out = np.zeros(shape)
    for p in itertools.product(range(n), repeat=dim):
        acc = 0.0
        for ax in range(dim):
            for d in (-1, 1):
                q = list(p)
                q[ax] += d
                if 0 <= q[ax] < n:
                    kf = 2 * Kp[p] * Kp[tuple(q)] / (Kp[p] + Kp[tuple(q)])
                    acc += kf * (U[p] - U[tuple(q)])
                else:
                    acc += Kp[p] * U[p]
        out[p] = acc / h ** 2
    return out.ravel()


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 4)])
def test_variable_kappa_matches_hand_sum(dim, n):
    rng = np.random.default_rng(7)
    kappa = np.exp(rng.standard_normal(n ** dim))
    u = rng.standard_normal(n ** dim)
    K = grid.stiffness(n, dim, kappa)
    assert np.allclose(K @ u, _hand_apply(n, dim, kappa, u), rtol=1e-13, atol=1e-10)
    assert abs(K - K.T).max() < 1e-9


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 5)])
def test_dst_eigenpairs(dim, n):
    K = grid.stiffness(n, dim)
    lam = grid.dst_eigenvalues(n, dim)
    X = grid.node_coordinates(n, dim)
    rng = np.random.default_rng(1)
    for _ in range(4):
        k = rng.integers(1, n + 1, size=dim)
        phi = np.ones((n,) * dim)
        for ax in range(dim):
            phi = phi * np.sin(k[ax] * np.pi * X[ax])
        Kphi = K @ phi.ravel()
        # lam is indexed [k_z, k_y, k_x] (axis 0 slowest)
        assert np.allclose(Kphi, lam[tuple(k[::-1] - 1)] * phi.ravel(), rtol=1e-12, atol=1e-9)


def test_constant_row_sums_are_boundary_terms():
    n, dim = 6, 2
    h = 1.0 / (n + 1)
    K = grid.stiffness(n, dim)
    rs = (K @ np.ones(n * n)).reshape(n, n)
    nb = np.zeros((n, n))
    nb[0, :] += 1
    nb[-1, :] += 1
    nb[:, 0] += 1
    nb[:, -1] += 1
    assert np.allclose(rs, nb / h ** 2)
