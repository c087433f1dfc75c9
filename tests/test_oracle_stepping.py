"""Pins of the oracle's sequential stepping (not gpu)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import heat_inputs
from oracle import allatonce, mms, stepping


def _mms_problem(n, s, nt, T=1.0):
    p = allatonce.Problem(n, 2, s, nt, T)
    f = heat_inputs.mms_source(n, 2, p.stage_times())
    u0 = heat_inputs.sin_product(n, 2)
    return p, f, u0


@pytest.mark.parametrize("method", ["lu", "dst"])
def test_config0_closed_form(method):
    """32x32, s=2, nt=16: stepping equals phi times the scalar recursion."""
    p, f, u0 = _mms_problem(32, 2, 16)
    x = stepping.solve(p, f, u0, method=method)
    xs = mms.solution(p, u0)
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_temporal_order(s):
    """Error at T against the semi-discrete solution decays like tau^(2s-1)."""
    n = 4
    errs = []
    nts = [8, 16, 32]
    for nt in nts:
        p = allatonce.Problem(n, 2, s, nt, 1.0)
        y, _ = mms.scalar_sequence(p)
        errs.append(abs(y[-1] - mms.semidiscrete(n, 1.0)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > (2 * s - 1) - 0.35, (errs, rates)


def test_spatial_eigenvalue_second_order():
    lam = [mms.eigenvalue(n) for n in (15, 31, 63)]
    err = [abs(l - 2 * np.pi ** 2) for l in lam]
    assert abs(np.log2(err[0] / err[1]) - 2) < 0.1 and abs(np.log2(err[1] / err[2]) - 2) < 0.1


def test_s1_is_implicit_euler():
    """Radau IIA s=1 stepping equals (I + tau K) v_{n+1} = v_n + tau f(t_{n+1})."""
    rng = np.random.default_rng(2)
    p = allatonce.Problem(9, 2, 1, 5, 0.5)
    f = rng.standard_normal((5, 1, p.N))
    u0 = rng.standard_normal(p.N)
    x = stepping.solve(p, f, u0, method="lu")
    v, _ = allatonce.split(p, x)
    K = p.K()
    Mt = (sp.identity(p.N) + p.tau * K).tocsc()
    w = u0.copy()
    for n in range(5):
        w = spla.spsolve(Mt, w + p.tau * f[n, 0])
        assert np.allclose(v[n + 1], w, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,n,s,nt", [(2, 12, 3, 5), (3, 6, 2, 4), (3, 5, 3, 3)])
def test_lu_equals_dst(dim, n, s, nt):
    rng = np.random.default_rng(4)
    p = allatonce.Problem(n, dim, s, nt, 1.0)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    a = stepping.solve(p, f, u0, method="lu")
    b = stepping.solve(p, f, u0, method="dst")
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
