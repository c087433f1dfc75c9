"""GPU parity of S-tilde by two-level MGRIT (the parallel-in-time route of
Sec. 5.2) against the oracle (oracle/mgrit.py through
oracle.precond.apply_preconditioner).

* P-tilde with S-tilde by MGRIT, FP64: equal to the oracle's MGRIT
  preconditioner (same propagators, same iteration) to rounding, for one
  iteration and for K - 1 iterations (K coarse intervals), F- and
  FCF-relaxation, nt a multiple of the coarsening factor and not, constant
  and variable diffusivity (dense coarsest inverses for the coarse step);
* K - 1 iterations reproduce the forward substitution: GPU MGRIT equals the
  GPU sweep;
* a coarse propagator with fewer inner GMRES iterations (mgrit_coarse_k)
  equals the oracle's MGRIT with the same coarse propagator, and S-tilde's
  steps with their own inner count (schur_k) equal the oracle's, with the
  substitution and with MGRIT;
* a solve with the MGRIT preconditioner (one iteration) reaches the unique
  solution x* = A^{-1} [b; f] (sequential stepping), forward and adjoint.
Tolerance 1e-10 as for the substitution preconditioner (FP64 rounding
amplified by the inner Krylov recurrences and the time recursion).
"""
import numpy as np
import pytest

import heat_inputs
from gpu_util import announce, rel_err, require_gpu, to_dev, to_host
from oracle import adjoint, allatonce, precond, stepping

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,s,nt,cf,iters,fcf", [(24, 2, 8, 4, 1, False), (24, 3, 8, 4, 1, True),
                                                  (20, 2, 7, 3, 1, False), (20, 2, 7, 3, 2, False),
                                                  (32, 3, 9, 3, 1, True), (16, 1, 6, 2, 2, False)])
def test_apply_P_mgrit_fp64_matches_oracle(n, s, nt, cf, iters, fcf):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, inner_k=3, nu1=2, nu2=2, schur="mgrit", mgrit_cf=cf,
                     mgrit_iters=iters, mgrit_fcf=fcf)
    ops = precond.StageOps(p, inner_k=3, cycles=1, nu1=2, nu2=2)
    r = np.random.default_rng(n + nt).standard_normal(p.U)
    announce("apply_P mgrit", n, s, nt, cf, iters, fcf)
    z = to_host(hp.apply_P(to_dev(r)))
    ref = precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=iters, relax="FCF" if fcf else "F"))
    assert rel_err(z, ref) <= 1e-10
    # short of exactness it is an approximation of the substitution, not
    # equal to it (F: one more exact C-point per iteration, FCF: two)
    sub = precond.apply_preconditioner(ops, r)
    K = -(-nt // cf)
    exact_after = -(-(K - 1) // 2) if fcf else K - 1
    if iters < exact_after:
        assert rel_err(ref, sub) > 1e-9


@pytest.mark.parametrize("n,s,nt,cf,iters,fcf,ck", [(24, 2, 12, 4, 1, False, 1), (20, 3, 10, 3, 1, False, 2),
                                                     (20, 2, 7, 2, 2, False, 1)])
def test_apply_P_mgrit_coarse_k_matches_oracle(n, s, nt, cf, iters, fcf, ck):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, inner_k=3, nu1=2, nu2=2, schur="mgrit", mgrit_cf=cf,
                     mgrit_iters=iters, mgrit_fcf=fcf, mgrit_coarse_k=ck)
    ops = precond.StageOps(p, inner_k=3, cycles=1, nu1=2, nu2=2)
    r = np.random.default_rng(n + nt + ck).standard_normal(p.U)
    announce("apply_P mgrit coarse k", n, s, nt, cf, iters, fcf, ck)
    z = to_host(hp.apply_P(to_dev(r)))
    relax = "FCF" if fcf else "F"
    ref = precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=iters, relax=relax, coarse_k=ck))
    assert rel_err(z, ref) <= 1e-10
    # the coarse propagator's inner count changes P-tilde
    full = precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=iters, relax=relax))
    assert rel_err(ref, full) > 1e-9


@pytest.mark.parametrize("schur,sk,ck", [("sweep", 1, 0), ("mgrit", 1, 1), ("mgrit", 2, 0)])
def test_apply_P_schur_k_matches_oracle(schur, sk, ck):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt, cf = 24, 3, 10, 4
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, inner_k=4, nu1=2, nu2=2, schur=schur, mgrit_cf=cf, schur_k=sk,
                     mgrit_coarse_k=ck)
    ops = precond.StageOps(p, inner_k=4, cycles=1, nu1=2, nu2=2, schur_k=sk)
    r = np.random.default_rng(17 + sk).standard_normal(p.U)
    announce("apply_P schur k", schur, sk, ck)
    z = to_host(hp.apply_P(to_dev(r)))
    mg = None if schur == "sweep" else dict(cf=cf, iters=1, coarse_k=ck or None)
    ref = precond.apply_preconditioner(ops, r, mgrit=mg)
    assert rel_err(z, ref) <= 1e-10
    full = precond.apply_preconditioner(precond.StageOps(p, inner_k=4, cycles=1, nu1=2, nu2=2), r, mgrit=mg)
    assert rel_err(ref, full) > 1e-9


@pytest.mark.parametrize("adjoint_solve", [False, True])
def test_solve_with_cheap_coarse_propagator_reaches_oracle(adjoint_solve):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 28, 3, 12
    rng = np.random.default_rng(44)
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, tol=1e-11, precision="fp32", inner_k=4, schur="mgrit", mgrit_cf=4,
                     mgrit_coarse_k=1, schur_k=1)
    announce("solve mgrit coarse k", adjoint_solve)
    if adjoint_solve:
        g = rng.standard_normal(p.U)
        lam, st = hp.solve_adjoint(to_dev(g))
        assert st["converged"], st
        assert rel_err(to_host(lam), adjoint.solve(p, g)) <= 1e-8
    else:
        f = rng.standard_normal((nt, s, p.N))
        u0 = rng.standard_normal(p.N)
        x, st = hp.solve(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
        assert st["converged"], st
        assert rel_err(to_host(x), stepping.solve(p, f, u0)) <= 1e-8


def test_apply_P_mgrit_variable_kappa_matches_oracle():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt, cf = 40, 2, 6, 3
    rng = np.random.default_rng(71)
    kappa = heat_inputs.lognormal_kappa(rng, n, 2)
    p = allatonce.Problem(n, 2, s, nt, 1.0, kappa=kappa)
    hp = HeatProblem(2, n, s, nt, 1.0, kappa=kappa, nu1=2, nu2=2, schur="mgrit", mgrit_cf=cf)
    ops = precond.StageOps(p, inner_k=3, cycles=1, nu1=2, nu2=2)
    r = rng.standard_normal(p.U)
    announce("apply_P mgrit vk")
    z = to_host(hp.apply_P(to_dev(r)))
    assert rel_err(z, precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=1))) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nt,cf", [(12, 4), (10, 4)])
def test_converged_mgrit_equals_gpu_sweep(precision, nt, cf):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s = 48, 3
    K = -(-nt // cf)
    common = dict(inner_k=3, nu1=2, nu2=2, precision=precision)
    sweep = HeatProblem(2, n, s, nt, 1.0, **common)
    mg = HeatProblem(2, n, s, nt, 1.0, schur="mgrit", mgrit_cf=cf, mgrit_iters=K - 1, **common)
    r = to_dev(np.random.default_rng(nt).standard_normal(sweep.U))
    announce("mgrit K-1 vs sweep", precision, nt, cf)
    z1 = to_host(sweep.apply_P(r))
    z2 = to_host(mg.apply_P(r))
    assert rel_err(z2, z1) <= (1e-11 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_with_mgrit_reaches_stepping(precision):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 40, 3, 16
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, tol=1e-11, inner_k=3, precision=precision, schur="mgrit",
                     mgrit_cf=4)
    rng = np.random.default_rng(1001)
    f = heat_inputs.bump_source(rng, n, 2, hp.stage_times())
    u0 = heat_inputs.smooth_initial(rng, n, 2)
    announce("solve mgrit", precision)
    rhs = hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0))
    x, st = hp.solve(rhs)
    assert st["converged"], st
    assert rel_err(to_host(x), stepping.solve(p, f, u0)) <= 1e-8


def test_adjoint_with_mgrit_matches_oracle():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 24, 2, 9
    rng = np.random.default_rng(32)
    kappa = heat_inputs.lognormal_kappa(rng, n, 2)
    p = allatonce.Problem(n, 2, s, nt, 1.0, kappa=kappa)
    hp = HeatProblem(2, n, s, nt, 1.0, kappa=kappa, tol=1e-11, precision="fp32", schur="mgrit", mgrit_cf=3,
                     mgrit_fcf=True)
    g = rng.standard_normal(p.U)
    announce("adjoint mgrit")
    lam, st = hp.solve_adjoint(to_dev(g))
    assert st["converged"], st
    assert rel_err(to_host(lam), adjoint.solve(p, g)) <= 1e-8
