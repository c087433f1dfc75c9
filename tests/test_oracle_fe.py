"""Pins of the Q1 finite-element pieces of the oracle (not gpu): element
matrices, assembly, eigenpairs, the Chebyshev mass solve, and the
all-at-once system with a mass matrix (Sec. 2, Sec. 5)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import allatonce, fe, precond, stepping, tableau


def test_element_matrices_are_the_textbook_bilinear_ones():
    h = 0.3
    Me, Ke = fe.element_matrices(h)
    # corners (0,0), (1,0), (0,1), (1,1)
    Mt = h * h / 36.0 * np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]])
    Kt = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(Me, Mt, atol=1e-15) and np.allclose(Ke, Kt, atol=1e-14)


@pytest.mark.parametrize("n,length", [(3, 1.0), (7, 2.0), (10, 1.5)])
def test_assembly_is_the_tensor_form(n, length):
    h = fe.spacing(n, length)
    M, K = fe.q1_matrices(n, length)
    e = np.ones(n)
    M1 = sp.diags([e[:-1] / 6, 2 * e / 3, e[:-1] / 6], [-1, 0, 1]) * h
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]) / h
    assert abs(M - sp.kron(M1, M1)).max() <= 1e-15
    assert abs(K - (sp.kron(T, M1) + sp.kron(M1, T))).max() <= 1e-13


def test_sine_modes_are_eigenpairs():
    n, length = 9, 2.0
    h = fe.spacing(n, length)
    M, K = fe.q1_matrices(n, length)
    X, Y = fe.node_coordinates(n, length)
    for k, l in [(1, 1), (2, 5), (9, 3)]:
        v = (np.sin(k * np.pi * X / length) * np.sin(l * np.pi * Y / length)).ravel()
        mu = lambda q: h * (2.0 / 3.0 + np.cos(q * np.pi * h / length) / 3.0)
        lam = lambda q: 2.0 / h * (1.0 - np.cos(q * np.pi * h / length))
        assert np.allclose(M @ v, mu(k) * mu(l) * v, atol=1e-14)
        assert np.allclose(K @ v, (lam(k) * mu(l) + mu(k) * lam(l)) * v, atol=1e-12)


def test_jacobi_spectrum_inside_the_bounds():
    M, _ = fe.q1_matrices(12, 2.0)
    ev = np.linalg.eigvalsh((M / M.diagonal()[:, None]).toarray())
    lo, hi = fe.Q1_JACOBI_BOUNDS
    assert lo < ev.min() and ev.max() < hi


@pytest.mark.parametrize("steps", [1, 2, 7, 20])
def test_chebyshev_error_is_the_chebyshev_polynomial(steps):
    """On an eigenvector of D^{-1} M (sine modes, D constant), k steps scale
    the error by T_k(g / rho) / T_k(1 / rho)."""
    n, length = 9, 2.0
    M, _ = fe.q1_matrices(n, length)
    X, Y = fe.node_coordinates(n, length)
    lo, hi = fe.Q1_JACOBI_BOUNDS
    theta, rho = (lo + hi) / 2, (hi - lo) / (hi + lo)
    for k, l in [(1, 1), (4, 7), (9, 9)]:
        v = (np.sin(k * np.pi * X / length) * np.sin(l * np.pi * Y / length)).ravel()
        lj = (v @ (M @ v)) / (v @ v) / M.diagonal()[0]
        y = fe.chebyshev_mass(M, M @ v, steps=steps)
        factor = fe.chebyshev_error_factor(1.0 - lj / theta, rho, steps)
        assert np.allclose(y - v, -factor * v, atol=1e-13 * np.abs(v).max())


def test_twenty_chebyshev_steps_meet_the_bound():
    n = 15
    M, _ = fe.q1_matrices(n, 2.0)
    t = np.random.default_rng(4).standard_normal((3, n * n))
    x = np.linalg.solve(M.toarray(), t.T).T
    y = fe.chebyshev_mass(M, t)
    bound = 1.0 / np.cosh(20 * np.arccosh(1.25))
    assert np.linalg.norm(y - x) <= bound * np.linalg.norm(x)
    assert bound < 2e-6


def _q1_problem(n=4, s=2, nt=3, T=0.6, length=2.0, seed=3):
    p = allatonce.Problem(n, 2, s, nt, T, disc="q1", length=length)
    rng = np.random.default_rng(seed)
    return p, rng.standard_normal((nt, s, p.N)), rng.standard_normal(p.N)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_q1_all_at_once_equals_stepping(s):
    p, f, u0 = _q1_problem(s=s)
    A = allatonce.operator(p, sparse=False)
    x = np.linalg.solve(A, allatonce.rhs(p, f, u0))
    xs = stepping.solve(p, f, u0)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    # the blockwise apply is the dense operator, forward and transposed
    y = np.random.default_rng(1).standard_normal(p.U)
    assert np.allclose(allatonce.apply_blockwise(p, y), A @ y, atol=1e-12)
    assert np.allclose(allatonce.apply_blockwise(p, y, transpose=True), A.T @ y, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2])
def test_q1_temporal_order(s):
    """On a fixed mesh the Radau IIA error in time falls like tau^(2s-1)."""
    n, T = 5, 0.5
    X, Y = fe.node_coordinates(n, 2.0)
    u0 = (np.sin(np.pi * X / 2) * np.sin(np.pi * Y / 2)).ravel()

    def final(nt):
        p = allatonce.Problem(n, 2, s, nt, T, disc="q1", length=2.0)
        v, _ = allatonce.split(p, stepping.solve(p, np.zeros((nt, s, p.N)), u0))
        return v[-1]

    ref = final(512)
    e1, e2 = np.linalg.norm(final(8) - ref), np.linalg.norm(final(16) - ref)
    assert 2 ** (2 * s - 1) * 0.8 <= e1 / e2 <= 2 ** (2 * s - 1) * 1.25


def test_q1_ideal_preconditioner_minimal_polynomial():
    p, _, _ = _q1_problem(n=3, s=2, nt=3)
    Ad = allatonce.operator(p, sparse=False)
    Pd = precond.dense_ideal_preconditioner(p)
    E = Ad @ np.linalg.inv(Pd) - np.eye(p.U)
    assert np.abs(E @ E).max() <= 1e-9 * np.abs(Ad).max()
    assert np.abs(E).max() > 1e-6


def test_q1_exact_block_back_substitution_is_the_ideal_preconditioner():
    p, _, _ = _q1_problem(n=3, s=2, nt=3)
    ops = precond.StageOps(p)
    r = np.random.default_rng(2).standard_normal(p.U)
    z = precond.apply_preconditioner(ops, r, exact=True)
    zd = np.linalg.solve(precond.dense_ideal_preconditioner(p), r)
    assert np.linalg.norm(z - zd) <= 1e-11 * np.linalg.norm(zd)


def test_q1_fgmres_with_the_practical_preconditioner_reaches_stepping():
    p, f, u0 = _q1_problem(n=15, s=2, nt=6, T=2.0)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2)
    K = p.K()
    x, its, _ = precond.fgmres(lambda y: allatonce.apply_blockwise(p, y, K),
                               lambda r: precond.apply_preconditioner(ops, r),
                               allatonce.rhs(p, f, u0), restart=20, tol=1e-12)
    xs = stepping.solve(p, f, u0)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert its <= 15


def paper_problem_error(s, l):
    """v_error of Sec. 5.1's problem (v = exp(t_f - t) times a cosine bump
    plus 1 on [-1, 1]^2, t_f = 2; here on [0, 2]^2 as a sine bump), Q1 with
    h = 2^(1-l) and the paper's rule for nt, by exact load vectors."""
    tf, length = 2.0, 2.0
    h = 2.0 ** (1 - l)
    n = 2 ** l - 1
    nt = int(np.ceil(tf / h ** (2.0 / (2 * s - 1)) - 1e-12))
    p = allatonce.Problem(n, 2, s, nt, tf, disc="q1", length=length)
    X, Y = fe.node_coordinates(n, length)
    k = np.pi / 2
    phi = (np.sin(k * X) * np.sin(k * Y)).ravel()
    load = fe.load_sine(n, length, k)
    Mm, K = p.M(), p.K()
    # right-hand side with the exact load vectors (not M times nodal values)
    v = np.zeros((nt + 1, p.N))
    v[0] = Mm @ (np.exp(tf) * phi)
    F = np.array([[(k * k * 2 - 1) * np.exp(tf - t) * load for t in row] for row in p.stage_times()])
    x = np.linalg.solve(allatonce.operator(p, sparse=False), allatonce.join(v, F)) if p.U < 3000 else None
    if x is None:
        import scipy.sparse.linalg as spla
        x = spla.spsolve(allatonce.operator(p).tocsc(), allatonce.join(v, F))
    vn, _ = allatonce.split(p, x)
    err = 0.0
    for m in range(1, nt + 1):
        vs = np.exp(tf - m * p.tau) * phi + 1.0
        j = np.argmax(np.abs(vn[m] + 1.0 - vs))
        err = max(err, abs(vn[m][j] + 1.0 - vs[j]) / abs(vs[j]))
    return p.U, err


def test_paper_problem_dof_and_error_trend():
    """Sec. 5.1, Table 1 (Q1): the DoF match exactly; the discretisation
    error falls by about 4 per level (second order in h, with tau tied to h)
    and sits within a factor 1.5 of the printed v_error (the paper's load
    vector and boundary treatment are not given, so the errors are a trend,
    not a pin)."""
    printed = {(2, 3): (931, 5.09e-3), (2, 4): (5625, 1.35e-3), (3, 3): (833, 5.71e-3), (3, 4): (4725, 1.46e-3)}
    errs = {}
    for (s, l), (dof, verr) in printed.items():
        U, e = paper_problem_error(s, l)
        assert U == dof
        assert verr / 1.5 <= e <= verr * 1.5, (s, l, e, verr)
        errs[s, l] = e
    for s in (2, 3):
        assert 3.0 <= errs[s, 3] / errs[s, 4] <= 5.0
