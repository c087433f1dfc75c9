"""Pins of the oracle's all-at-once operator and layout (not gpu)."""
import math
import os

import numpy as np
import pytest

from oracle import allatonce, stepping

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_q1_dof.txt")


def test_layout_reproduces_table1_dof():
    """U = N (nt (s+1) + 1) gives every Q1 DoF entry of Table 1 (Sec. 5.1)."""
    rows = [list(map(int, line.split())) for line in open(GOLDEN)
            if line.strip() and not line.startswith("#")]
    assert len(rows) == 20
    for s, l, dof in rows:
        h = 2.0 ** (1 - l)
        N = (round(2.0 / h) - 1) ** 2                 # interior Q1 nodes of [-1,1]^2
        nt = math.ceil(2.0 / h ** (2.0 / (2 * s - 1)) - 1e-12)
        assert allatonce.unknowns(N, nt, s) == dof


def _random_problem(dim, n, s, nt, var_kappa, seed):
    rng = np.random.default_rng(seed)
    kappa = np.exp(rng.standard_normal(n ** dim)) if var_kappa else None
    p = allatonce.Problem(n, dim, s, nt, T=0.7, kappa=kappa)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    return p, f, u0


CASES = [(2, 3, 1, 3, False), (2, 3, 2, 4, True), (2, 4, 3, 2, False),
         (3, 2, 2, 3, False), (3, 3, 3, 2, True)]


@pytest.mark.parametrize("dim,n,s,nt,vk", CASES)
def test_stepping_equals_dense_solve(dim, n, s, nt, vk):
    p, f, u0 = _random_problem(dim, n, s, nt, vk, 11)
    Ad = allatonce.operator(p, sparse=False)
    assert Ad.shape == (p.U, p.U)
    rhs = allatonce.rhs(p, f, u0)
    x_dense = np.linalg.solve(Ad, rhs)
    x_step = stepping.solve(p, f, u0, method="lu")
    assert np.linalg.norm(x_step - x_dense) <= 1e-12 * np.linalg.norm(x_dense)
    assert np.linalg.norm(Ad @ x_step - rhs) <= 1e-12 * np.linalg.norm(rhs) * np.linalg.cond(Ad)


@pytest.mark.parametrize("dim,n,s,nt,vk", CASES)
def test_blockwise_apply_equals_dense(dim, n, s, nt, vk):
    p, _, _ = _random_problem(dim, n, s, nt, vk, 12)
    Ad = allatonce.operator(p, sparse=False)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(p.U)
    y = rng.standard_normal(p.U)
    Ax = allatonce.apply_blockwise(p, x)
    ATy = allatonce.apply_blockwise(p, y, transpose=True)
    assert np.allclose(Ax, Ad @ x, rtol=1e-13, atol=1e-13 * np.abs(Ad).max())
    assert np.allclose(ATy, Ad.T @ y, rtol=1e-13, atol=1e-13 * np.abs(Ad).max())
    assert abs(Ax @ y - x @ ATy) <= 1e-13 * np.abs(Ad).max() * np.linalg.norm(x) * np.linalg.norm(y)


@pytest.mark.parametrize("dim,n,s,nt,vk", CASES)
def test_row_apply_equals_blockwise(dim, n, s, nt, vk):
    p, _, _ = _random_problem(dim, n, s, nt, vk, 13)
    x = np.random.default_rng(4).standard_normal(p.U)
    rows = np.arange(p.U)
    assert np.allclose(allatonce.apply_rows(p, x, rows), allatonce.apply_blockwise(p, x),
                       rtol=1e-13, atol=1e-12 * np.abs(x).max() / p.h ** 2)


def test_first_rows_are_initial_condition():
    p, f, u0 = _random_problem(2, 3, 2, 3, False, 5)
    Ad = allatonce.operator(p, sparse=False)
    assert np.array_equal(Ad[: p.N, : p.N], np.eye(p.N))
    assert np.count_nonzero(Ad[: p.N]) == p.N
