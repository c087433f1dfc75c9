"""Pins of the oracle's preconditioners and FGMRES (not gpu)."""
import numpy as np
import pytest

from oracle import allatonce, precond, stepping


def _prob(dim=2, n=3, s=2, nt=3, seed=31):
    rng = np.random.default_rng(seed)
    p = allatonce.Problem(n, dim, s, nt, 0.8)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    return p, f, u0, rng


@pytest.mark.parametrize("dim,n,s,nt", [(2, 3, 2, 3), (2, 3, 3, 2), (3, 2, 2, 2)])
def test_ideal_preconditioner_minimal_polynomial(dim, n, s, nt):
    """Sec. 3: sigma(P^{-1} A) = {1} with minimal polynomial of degree two."""
    p, *_ = _prob(dim, n, s, nt)
    Ad = allatonce.operator(p, sparse=False)
    Pd = precond.dense_ideal_preconditioner(p)
    E = Ad @ np.linalg.inv(Pd) - np.eye(p.U)
    assert np.abs(E @ E).max() <= 1e-10 * np.abs(Ad).max()
    assert np.abs(E).max() > 1e-6          # degree two, not one


def test_block_back_substitution_equals_dense_ideal():
    p, _, _, rng = _prob(2, 3, 2, 3)
    ops = precond.StageOps(p)
    r = rng.standard_normal(p.U)
    z = precond.apply_preconditioner(ops, r, exact=True)
    zd = np.linalg.solve(precond.dense_ideal_preconditioner(p), r)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)


def test_fgmres_with_ideal_preconditioner_two_steps():
    p, f, u0, _ = _prob(2, 4, 3, 4)
    ops = precond.StageOps(p)
    K = p.K()
    rhs = allatonce.rhs(p, f, u0)
    x, its, _ = precond.fgmres(lambda y: allatonce.apply_blockwise(p, y, K),
                               lambda r: precond.apply_preconditioner(ops, r, exact=True),
                               rhs, restart=10, tol=1e-11)
    assert its <= 2
    xs = stepping.solve(p, f, u0, method="lu")
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_inner_gmres_is_krylov_minimiser():
    """GMRES(k) from zero minimises ||b - A M^{-1} y|| over K_k(A M^{-1}, b)."""
    rng = np.random.default_rng(8)
    m, k = 30, 4
    A = np.eye(m) * 3 + rng.standard_normal((m, m)) * 0.3
    Mi = np.eye(m) + rng.standard_normal((m, m)) * 0.05
    b = rng.standard_normal(m)
    x, its = precond.gmres(lambda v: A @ v, lambda v: Mi @ v, b, k)
    assert its == k
    B = A @ Mi
    Kr = np.column_stack([np.linalg.matrix_power(B, j) @ b for j in range(k)])
    y, *_ = np.linalg.lstsq(B @ Kr, b, rcond=None)
    assert np.linalg.norm(x - Mi @ Kr @ y) <= 1e-10 * np.linalg.norm(x)


def test_rana_exact_for_one_stage():
    """s = 1: L = A_RK, so Rana with exact blocks is Theta_hat^{-1}."""
    p, _, _, rng = _prob(2, 5, 1, 2)
    ops = precond.StageOps(p, inner_k=1, exact_blocks=True)
    r = rng.standard_normal((1, p.N))
    assert np.allclose(ops.theta_tilde_inv(r), ops.theta_inv(r), rtol=1e-12, atol=1e-12)


def test_rana_is_block_lower_triangular_solve():
    p, _, _, rng = _prob(2, 4, 3, 2)
    ops = precond.StageOps(p, exact_blocks=True)
    r = rng.standard_normal((3, p.N))
    z = ops.rana(r)
    import scipy.sparse as sp
    Pint = sp.kron(np.eye(3), sp.identity(p.N)) + p.tau * sp.kron(ops.L, ops.K)
    assert np.allclose(Pint @ z.ravel(), r.ravel(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_fgmres_practical_preconditioner_converges_to_stepping(s):
    rng = np.random.default_rng(40 + s)
    p = allatonce.Problem(16, 2, s, 6, 1.0)
    f = rng.standard_normal((6, s, p.N))
    u0 = rng.standard_normal(p.N)
    ops = precond.StageOps(p, inner_k=3, cycles=3)
    K = p.K()
    rhs = allatonce.rhs(p, f, u0)
    x, its, _ = precond.fgmres(lambda y: allatonce.apply_blockwise(p, y, K),
                               lambda r: precond.apply_preconditioner(ops, r),
                               rhs, restart=30, tol=1e-10)
    xs = stepping.solve(p, f, u0)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # Sec. 5.1: at most 10 outer iterations to 1e-8 with 3 multigrid cycles (here 1e-10)
    assert its <= 14
