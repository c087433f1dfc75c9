"""GPU parity of the preconditioner P-tilde (eqs. (3.2)-(3.3)) against the oracle.

FP64: the GPU applies the same algorithm as the oracle (inner GMRES(k) with
Rana's stage preconditioner, Galerkin V-cycles with weighted Jacobi), so the
outputs agree to rounding (the map is nonlinear but smooth: the inner
least-squares problems are well conditioned).  Tolerance 1e-10 relative:
FP64 rounding (~1e-16) amplified by the inner Krylov recurrences and the
nt-step S-tilde recursion.  Lower precisions are compared against the FP64
oracle with tolerances set by their unit roundoff (FP32 ~6e-8, BF16 ~4e-3,
FP16 ~5e-4) times the same amplification.
"""
import numpy as np
import pytest

from gpu_util import announce, rel_err, require_gpu, to_dev, to_host
from oracle import allatonce, precond

pytestmark = pytest.mark.gpu


def _pair(dim, n, s, nt, precision="fp64", k=3, cycles=1, nu=2, seed=0, transpose=False, orth="cgs2"):
    from paper_2609_16863_amd import HeatProblem
    p = allatonce.Problem(n, dim, s, nt, 1.0)
    hp = HeatProblem(dim, n, s, nt, 1.0, inner_k=k, cycles=cycles, nu1=nu, nu2=nu, precision=precision,
                     inner_orth=orth)
    ops = precond.StageOps(p, inner_k=k, cycles=cycles, nu1=nu, nu2=nu)
    return p, hp, ops, np.random.default_rng(seed)


# sizes: exact coarse solve only (16, 13), one or more grid levels plus the
# LDS tail (32, 72, 130), 3D grid levels (8, 7, 12); ragged N throughout
@pytest.mark.parametrize("dim,n,s,nt", [(2, 16, 2, 4), (2, 13, 3, 3), (2, 32, 1, 3), (2, 72, 2, 3),
                                        (2, 130, 3, 2), (3, 8, 2, 2), (3, 7, 3, 2), (3, 12, 2, 2)])
def test_apply_P_fp64_matches_oracle(dim, n, s, nt):
    require_gpu()
    p, hp, ops, rng = _pair(dim, n, s, nt, seed=n)
    r = rng.standard_normal(p.U)
    announce("apply_P fp64", dim, n, s, nt)
    z = to_host(hp.apply_P(to_dev(r)))
    ref = precond.apply_preconditioner(ops, r)
    assert rel_err(z, ref) <= 1e-10
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
@pytest.mark.parametrize("dim,n,s,nt", [(2, 72, 2, 3), (2, 130, 3, 2), (3, 12, 2, 2)])
def test_apply_P_one_pass_gram_schmidt_matches_oracle(dim, n, s, nt, precision, tol):
    """The inner GMRES with one classical Gram-Schmidt pass (h_{j+1,j} from
    <w,w> - |h|^2) is the oracle's modified Gram-Schmidt GMRES up to
    rounding."""
    require_gpu()
    p, hp, ops, rng = _pair(dim, n, s, nt, precision=precision, k=4, seed=n + 1, orth="cgs1")
    ops = precond.StageOps(p, inner_k=4, cycles=1, nu1=2, nu2=2)
    r = rng.standard_normal(p.U)
    announce("apply_P cgs1", precision, dim, n, s, nt)
    z = to_host(hp.apply_P(to_dev(r)))
    assert rel_err(z, precond.apply_preconditioner(ops, r)) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
@pytest.mark.parametrize("n,s,nt,nu", [(130, 3, 9, 2), (61, 3, 8, 1), (100, 2, 8, 3)])
def test_apply_P_row_march_equals_tiles(precision, tol, n, s, nt, nu):
    """The batched Theta-tilde solves (nt blocks per launch) run level 0 of
    the constant-coefficient operator in the row-marching down and up
    kernels once a launch has tall_min_b blocks; the down kernel also forms
    Rana's coupling terms of stages 2 and 3.  tall_min_b = 2^30 keeps every
    launch on the LDS tiles.  The kernels apply the same arithmetic to every
    node and the reductions run in a fixed order, so P-tilde is the same
    bit for bit; the FP64 oracle checks the march."""
    require_gpu()
    p, hp, ops, rng = _pair(2, n, s, nt, precision=precision, nu=nu, seed=7 * n)
    r = rng.standard_normal(p.U)
    announce("apply_P row march vs tiles", precision, n, s, nt, "nu", nu)
    hp.set_launch_shapes(1, 0)
    z_march = to_host(hp.apply_P(to_dev(r)))
    hp.set_launch_shapes(1 << 30, 0)
    z_tiles = to_host(hp.apply_P(to_dev(r)))
    assert np.array_equal(z_march, z_tiles)
    ref = precond.apply_preconditioner(ops, r)
    assert rel_err(z_march, ref) <= tol, rel_err(z_march, ref)


@pytest.mark.parametrize("dim,n,nt", [(2, 40, 12), (3, 14, 8)])
def test_solve_with_the_benchmark_settings_reaches_stepping(dim, n, nt):
    """One-pass Gram-Schmidt, one inner iteration in S-tilde and on MGRIT's
    coarse level, FP32 P-tilde: the solve reaches x* (stepping)."""
    require_gpu()
    from oracle import stepping
    from paper_2609_16863_amd import HeatProblem
    s = 3
    p = allatonce.Problem(n, dim, s, nt, 1.0)
    hp = HeatProblem(dim, n, s, nt, 1.0, tol=1e-11, maxit=200, precision="fp32", inner_k=4, schur="mgrit",
                     mgrit_cf=4, mgrit_coarse_k=1, schur_k=1, inner_orth="cgs1")
    rng = np.random.default_rng(dim * 100 + n)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    announce("solve benchmark settings", dim, n, nt)
    x, st = hp.solve(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
    assert st["converged"], st
    assert rel_err(to_host(x), stepping.solve(p, f, u0)) <= 1e-8


@pytest.mark.parametrize("n,s,nt", [(40, 2, 3), (72, 3, 2)])
def test_apply_P_variable_kappa_fp64_matches_oracle(n, s, nt):
    """Lognormal patch diffusivity: face coefficients on the fine level,
    Galerkin 9-point stencils on the coarse levels, as in the oracle."""
    require_gpu()
    import heat_inputs
    from paper_2609_16863_amd import HeatProblem
    rng = np.random.default_rng(17 + n)
    kappa = heat_inputs.lognormal_kappa(rng, n, 2)
    p = allatonce.Problem(n, 2, s, nt, 1.0, kappa=kappa)
    hp = HeatProblem(2, n, s, nt, 1.0, kappa=kappa, nu1=2, nu2=2)
    ops = precond.StageOps(p, inner_k=3, cycles=1, nu1=2, nu2=2)
    r = rng.standard_normal(p.U)
    announce("apply_P vk fp64", n, s, nt)
    z = to_host(hp.apply_P(to_dev(r)))
    ref = precond.apply_preconditioner(ops, r)
    assert rel_err(z, ref) <= 1e-10


def test_apply_P_coarse_max_1024_matches_oracle():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 72, 3, 3
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, coarse_max=1024, nu1=2, nu2=2)
    ops = precond.StageOps(p, inner_k=3, cycles=1, nu1=2, nu2=2, coarse_max=1024)
    r = np.random.default_rng(23).standard_normal(p.U)
    announce("apply_P coarse_max 1024", n, s, nt)
    z = to_host(hp.apply_P(to_dev(r)))
    assert rel_err(z, precond.apply_preconditioner(ops, r)) <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-4), ("bf16", 5e-2), ("fp16", 1e-3)])
def test_apply_P_low_precision_close_to_fp64_oracle(precision, tol):
    require_gpu()
    p, hp, ops, rng = _pair(2, 72, 3, 3, precision=precision, seed=5)
    r = rng.standard_normal(p.U)
    announce("apply_P", precision)
    z = to_host(hp.apply_P(to_dev(r)))
    ref = precond.apply_preconditioner(ops, r)
    assert np.all(np.isfinite(z))
    assert rel_err(z, ref) <= tol


def test_apply_P_tends_to_ideal_preconditioner():
    """Many inner iterations and cycles: P-tilde -> P of eq. (3.1) (Sec. 3)."""
    require_gpu()
    p, hp, _, rng = _pair(2, 12, 2, 3, k=12, cycles=6, seed=3)
    exact = precond.StageOps(p)
    r = rng.standard_normal(p.U)
    announce("apply_P ideal limit")
    z = to_host(hp.apply_P(to_dev(r)))
    ref = precond.apply_preconditioner(exact, r, exact=True)
    assert rel_err(z, ref) <= 1e-7


@pytest.mark.parametrize("dim,n,s,nt", [(2, 12, 2, 3), (2, 9, 3, 2)])
def test_adjoint_with_near_exact_transposed_preconditioner(dim, n, s, nt):
    """P-tilde^T with near-exact inner solves -> P^T: the adjoint FGMRES needs <= 2 steps (Sec. 3)."""
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    p = allatonce.Problem(n, dim, s, nt, 1.0)
    hp = HeatProblem(dim, n, s, nt, 1.0, inner_k=12, cycles=6, tol=1e-9)
    r = np.random.default_rng(11).standard_normal(p.U)
    announce("adjoint near-exact", dim, n, s, nt)
    lam, st = hp.solve_adjoint(to_dev(r))
    Ad = allatonce.operator(p, sparse=False)
    assert st["converged"] and st["outer_iterations"] <= 3
    assert rel_err(to_host(lam), np.linalg.solve(Ad.T, r)) <= 1e-7
