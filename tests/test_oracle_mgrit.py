"""Pins of the two-level MGRIT oracle (oracle/mgrit.py) against facts that do
not come from its own code.

* K - 1 iterations (K = ceil(nt / cf) C-points) reproduce forward
  substitution exactly, for linear and nonlinear propagators, with F- and
  FCF-relaxation, for nt both a multiple of cf and not;
* with the exact coarse propagator Phi_c = Phi^cf (linear), one iteration is
  exact (the coarse system is then the exact reduced system);
* for the scalar recurrence z_{n+1} = t_{n+1} + a z_n the C-point errors after
  one iteration follow the two-level error recursion written out in closed
  form, from any initial C-point guess;
* through the preconditioner: P-tilde with S-tilde by MGRIT iterated to
  exactness equals P-tilde with the forward substitution.
"""
import numpy as np
import pytest

import heat_inputs
from oracle import allatonce, mgrit, precond


def _rand_prop(rng, n, scale=0.9):
    M = rng.standard_normal((n, n))
    M *= scale / np.linalg.norm(M, 2)
    return M


@pytest.mark.parametrize("nt,cf", [(16, 4), (17, 4), (9, 3), (5, 8), (12, 2)])
@pytest.mark.parametrize("relax", ["F", "FCF"])
def test_exact_after_K_minus_1_iterations(nt, cf, relax):
    rng = np.random.default_rng(nt * 10 + cf)
    n = 5
    A = _rand_prop(rng, n)
    Ac = _rand_prop(rng, n, 0.5)
    t = [rng.standard_normal(n) for _ in range(nt + 1)]
    ref = mgrit.sequential(t, lambda z: A @ z)
    K = -(-nt // cf)
    z = mgrit.solve(t, lambda z: A @ z, lambda e: Ac @ e, cf, max(K - 1, 0), relax)
    for a, b in zip(z, ref):
        assert np.allclose(a, b, rtol=0, atol=1e-12 * (1 + np.abs(b).max()))


@pytest.mark.parametrize("nt,cf", [(20, 4), (27, 3), (14, 2)])
def test_fcf_makes_two_c_points_exact_per_iteration(nt, cf):
    rng = np.random.default_rng(nt + cf)
    n = 3
    A = _rand_prop(rng, n)
    t = [rng.standard_normal(n) for _ in range(nt + 1)]
    ref = mgrit.sequential(t, lambda z: A @ z)
    K = -(-nt // cf)
    for iters in range(1, K):
        z = mgrit.solve(t, lambda z: A @ z, lambda e: 0.2 * e, cf, iters, "FCF")
        exact = [k for k in range(K) if np.abs(z[k * cf] - ref[k * cf]).max() <= 1e-12]
        assert exact[: min(2 * iters, K - 1) + 1] == list(range(min(2 * iters, K - 1) + 1))
        if 2 * iters < K - 1:
            assert np.abs(z[(2 * iters + 1) * cf] - ref[(2 * iters + 1) * cf]).max() > 1e-9


def test_exact_for_nonlinear_propagator():
    rng = np.random.default_rng(3)
    n, nt, cf = 4, 14, 3
    A = _rand_prop(rng, n, 0.7)
    phi = lambda z: A @ z + 0.1 * np.tanh(z)
    t = [rng.standard_normal(n) for _ in range(nt + 1)]
    ref = mgrit.sequential(t, phi)
    z = mgrit.solve(t, phi, lambda e: 0.3 * e, cf, -(-nt // cf) - 1)
    assert max(np.abs(a - b).max() for a, b in zip(z, ref)) <= 1e-12


def test_one_iteration_exact_with_exact_coarse_propagator():
    rng = np.random.default_rng(4)
    n, nt, cf = 6, 20, 4
    A = _rand_prop(rng, n)
    Ac = np.linalg.matrix_power(A, cf)
    t = [rng.standard_normal(n) for _ in range(nt + 1)]
    ref = mgrit.sequential(t, lambda z: A @ z)
    z = mgrit.solve(t, lambda z: A @ z, lambda e: Ac @ e, cf, 1)
    assert max(np.abs(a - b).max() for a, b in zip(z, ref)) <= 1e-12
    # one iteration is not exact with an inexact coarse propagator
    z2 = mgrit.solve(t, lambda z: A @ z, lambda e: 0.5 * Ac @ e, cf, 1)
    assert max(np.abs(a - b).max() for a, b in zip(z2, ref)) > 1e-6


@pytest.mark.parametrize("a,a_c,cf", [(0.8, 0.3, 4), (0.5, 0.2, 3), (-0.7, 0.1, 2)])
def test_scalar_error_recursion(a, a_c, cf):
    rng = np.random.default_rng(5)
    nt = 6 * cf
    K = nt // cf
    t = [np.array([v]) for v in rng.standard_normal(nt + 1)]
    exact = mgrit.sequential(t, lambda z: a * z)
    zC0 = [t[0]] + [np.array([v]) for v in rng.standard_normal(K - 1)]
    eps0 = [0.0] + [float(zC0[k][0] - exact[k * cf][0]) for k in range(1, K)]
    z = mgrit.solve(t, lambda z: a * z, lambda e: a_c * e, cf, 1, zC0=zC0)
    eps1 = [float(z[k * cf][0] - exact[k * cf][0]) for k in range(K)]
    want = mgrit.scalar_error_recursion(eps0, a, a_c, cf)
    assert np.allclose(eps1, want, rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("coarse_k", [None, 1])
def test_preconditioner_with_converged_mgrit_equals_substitution(coarse_k):
    """K - 1 F-iterations make every C-point exact whatever the coarse
    propagator is, so a cheaper coarse propagator (fewer inner GMRES
    iterations) still reproduces the substitution."""
    n, s, nt, cf = 10, 2, 7, 3
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    ops = precond.StageOps(p, inner_k=2, cycles=1, nu1=2, nu2=2)
    r = np.random.default_rng(6).standard_normal(p.U)
    z_sub = precond.apply_preconditioner(ops, r)
    K = -(-nt // cf)
    z_mg = precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=K - 1, coarse_k=coarse_k))
    assert np.allclose(z_mg, z_sub, rtol=0, atol=1e-12 * np.abs(z_sub).max())
    # a single iteration is an approximation, close but not equal
    z_1 = precond.apply_preconditioner(ops, r, mgrit=dict(cf=cf, iters=1, coarse_k=coarse_k))
    d = np.linalg.norm(z_1 - z_sub) / np.linalg.norm(z_sub)
    assert 1e-12 < d < 0.5
