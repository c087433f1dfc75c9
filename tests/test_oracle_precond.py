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


def test_schur_steps_take_their_own_inner_count():
    """S-tilde's steps use schur_k inner iterations: one iteration from zero
    is the minimal-residual multiple of Rana's step, x = alpha z with
    z = Rana(r), w = Theta_hat z, alpha = <r, w> / <w, w>; the propagator of
    a schur_k = 1 problem applies exactly that."""
    p, _, _, rng = _prob(2, 6, 3, 3)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2, schur_k=1)
    assert ops.schur_k == 1 and ops.inner_k == 3
    r = rng.standard_normal((3, p.N))
    z = ops.rana(r).ravel()
    w = ops.Th @ z
    alpha = (r.ravel() @ w) / (w @ w)
    assert np.allclose(ops.theta_tilde_inv(r, 1).ravel(), alpha * z, rtol=1e-12, atol=1e-13)
    v = rng.standard_normal(p.N)
    phi = precond.schur_propagator(ops)
    rhs = np.tile(ops.K @ v, (3, 1))
    zr = ops.rana(rhs).ravel()
    wr = ops.Th @ zr
    y = ((rhs.ravel() @ wr) / (wr @ wr) * zr).reshape(3, p.N)
    assert np.allclose(phi(v), v - p.tau * np.tensordot(p.b, y, axes=(0, 0)), rtol=1e-12, atol=1e-12)
    # the default takes inner_k, which differs
    assert not np.allclose(precond.schur_propagator(precond.StageOps(p, inner_k=3, nu1=2, nu2=2))(v), phi(v))


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


# ---- Algorithm 1 (split preconditioning, four precisions) ------------------
def test_algorithm1_without_preconditioners_is_gmres_minimiser():
    """P_L = P_R = I, one cycle of k steps: x_k minimises ||b - A x|| over the
    Krylov space K_k(A, b) (brute-force least squares over its power basis)."""
    rng = np.random.default_rng(12)
    m, k = 25, 5
    A = np.eye(m) * 2 + rng.standard_normal((m, m)) * 0.3
    b = rng.standard_normal(m)
    x, its, _ = precond.fgmres_split(lambda v: A @ v, None, None, b, restart=k, tol=0.0, maxit=k)
    assert its == k
    Kr = np.column_stack([np.linalg.matrix_power(A, j) @ b for j in range(k)])
    y, *_ = np.linalg.lstsq(A @ Kr, b, rcond=None)
    assert np.linalg.norm(x - Kr @ y) <= 1e-9 * np.linalg.norm(x)


def test_algorithm1_left_ideal_preconditioner_two_steps():
    """P_L = the ideal P of eq. (3.1): (P^{-1} A - I)^2 = 0, so the
    left-preconditioned iteration ends in at most two steps (Sec. 3)."""
    p, f, u0, _ = _prob(2, 4, 3, 4)
    ops = precond.StageOps(p)
    K = p.K()
    rhs = allatonce.rhs(p, f, u0)
    x, its, _ = precond.fgmres_split(lambda y: allatonce.apply_blockwise(p, y, K),
                                     lambda r: precond.apply_preconditioner(ops, r, exact=True), None,
                                     rhs, restart=10, tol=1e-12)
    assert its <= 2
    xs = stepping.solve(p, f, u0, method="lu")
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_algorithm1_right_equals_fgmres():
    """Algorithm 1 with P_L = I is the right-preconditioned FGMRES."""
    p, f, u0, _ = _prob(2, 6, 3, 4)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2)
    K = p.K()
    A = lambda y: allatonce.apply_blockwise(p, y, K)
    P = lambda r: precond.apply_preconditioner(ops, r)
    rhs = allatonce.rhs(p, f, u0)
    x1, its1, _ = precond.fgmres_split(A, None, P, rhs, restart=30, tol=1e-10)
    x2, its2, _ = precond.fgmres(A, P, rhs, restart=30, tol=1e-10)
    assert its1 == its2
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x2)


@pytest.mark.parametrize("side,k", [("right", 3), ("split", 3), ("left", 10)])
def test_algorithm1_sides_reach_the_solution(side, k):
    """With P-tilde on either side (or both), tightly converged Algorithm 1
    reaches x* = sequential stepping; on the left the inner solves must be
    tight, since the test is then on P-tilde^{-1}(A x) - P-tilde^{-1} b for
    a nonlinear P-tilde (next test)."""
    p, f, u0, _ = _prob(2, 6, 2, 4)
    ops = precond.StageOps(p, inner_k=k, nu1=2, nu2=2)
    K = p.K()
    P = lambda r: precond.apply_preconditioner(ops, r)
    PL = P if side in ("left", "split") else None
    PR = P if side in ("right", "split") else None
    rhs = allatonce.rhs(p, f, u0)
    x, its, hist = precond.fgmres_split(lambda y: allatonce.apply_blockwise(p, y, K), PL, PR, rhs,
                                        restart=30, tol=1e-12, maxit=200)
    xs = stepping.solve(p, f, u0, method="lu")
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs), (its, hist[-1])


def test_algorithm1_left_accuracy_follows_inner_accuracy():
    """Left preconditioning with the nonlinear P-tilde (inner GMRES from zero,
    Sec. 3): once the preconditioned residual is tiny, the true residual is
    bounded by how far P-tilde is from a fixed linear map, which shrinks as
    the inner iterations grow."""
    p, f, u0, _ = _prob(2, 6, 2, 4)
    K = p.K()
    A = lambda y: allatonce.apply_blockwise(p, y, K)
    rhs = allatonce.rhs(p, f, u0)
    true = []
    for k in (3, 6, 10):
        ops = precond.StageOps(p, inner_k=k, nu1=2, nu2=2)
        _, _, hist = precond.fgmres_split(A, lambda r: precond.apply_preconditioner(ops, r), None, rhs,
                                          restart=30, tol=1e-12, maxit=100)
        true.append(hist[-1])
    assert true[0] > 1e-6 and true[2] < 1e-10 and true[0] > true[1] > true[2]


def test_algorithm1_single_precision_system_stagnates():
    """Approach A3 (Sec. 5): the system solved in single precision
    (u = u_A = u_PR = FP32).  The true FP64 residual cannot go far below the
    FP32 unit roundoff times the condition of the problem, unlike FP64."""
    p, f, u0, _ = _prob(2, 12, 2, 6)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2)
    K = p.K()
    A = lambda y: allatonce.apply_blockwise(p, y, K)
    P = lambda r: precond.apply_preconditioner(ops, r)
    rhs = allatonce.rhs(p, f, u0)
    r32 = precond.round_fp32
    _, _, h32 = precond.fgmres_split(A, None, P, rhs, restart=30, tol=1e-12, maxit=60, rnd=r32, rnd_A=r32,
                                     rnd_PR=r32)
    _, _, h64 = precond.fgmres_split(A, None, P, rhs, restart=30, tol=1e-12, maxit=60)
    assert min(h64) <= 1e-11
    assert min(h32) >= 1e-9


def test_round_bf16_is_nearest_even_bfloat16():
    """Against a brute-force choice between the two neighbouring bfloat16
    values of the FP32 input (ties to the even significand)."""
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, 1.0, 2.0 ** -126]])
    f = x.astype(np.float32)
    bits = f.view(np.uint32).astype(np.int64)
    lo = (bits & ~0xFFFF) & 0xFFFFFFFF
    hi = lo + 0x10000
    vlo = lo.astype(np.uint32).view(np.float32).astype(np.float64)
    vhi = hi.astype(np.uint32).view(np.float32).astype(np.float64)
    fv = f.astype(np.float64)
    dlo, dhi = np.abs(fv - vlo), np.abs(vhi - fv)
    even_lo = ((lo >> 16) & 1) == 0
    want = np.where(dlo < dhi, vlo, np.where(dhi < dlo, vhi, np.where(even_lo, vlo, vhi)))
    got = precond.round_bf16(x)
    assert np.array_equal(got, want)
    nz = x != 0
    assert np.max(np.abs(got[nz] - fv[nz]) / np.abs(fv[nz])) <= 2.0 ** -8


def _relax_problem():
    p, f, u0, _ = _prob(2, 12, 2, 6)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2)
    K = p.K()
    return (lambda y: allatonce.apply_blockwise(p, y, K)), (lambda r: precond.apply_preconditioner(ops, r)), \
        allatonce.rhs(p, f, u0)


def test_relaxed_matvec_keeps_the_target():
    """The iteration-dependent matvec tolerance (Sec. 4, after Simoncini and
    Szyld): products taken in BF16 / FP32 once the residual has fallen far
    enough still reach the target, in the same number of iterations."""
    A, P, rhs = _relax_problem()
    for tol in (1e-8, 1e-11):
        st = {}
        _, its_r, hist_r = precond.fgmres_split(A, None, P, rhs, restart=30, tol=tol, maxit=60, relax=True,
                                                stats=st)
        _, its, _ = precond.fgmres_split(A, None, P, rhs, restart=30, tol=tol, maxit=60)
        assert hist_r[-1] <= tol
        assert abs(its_r - its) <= 1
        assert st.get("fp32", 0) >= 1 and st.get("bf16", 0) >= 1 and sum(st.values()) < its_r


def test_relaxing_every_product_loses_the_target():
    """Without the criterion (every product in BF16) the true residual stalls
    far above 1e-8: the relaxation has to follow the residual."""
    A, P, rhs = _relax_problem()
    _, _, hist = precond.fgmres_split(A, None, P, rhs, restart=30, tol=1e-8, maxit=60,
                                      rnd_A=precond.round_bf16)
    assert min(hist) > 1e-6
