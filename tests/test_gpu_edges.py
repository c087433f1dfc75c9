"""Edge cases of the solve against the oracle: the smallest grids and step
counts, MGRIT with fewer steps than its coarsening factor or a ragged last
interval, a single stage, left preconditioning with MGRIT, and Q1 elements
with MGRIT and with the all-half preconditioner."""
import numpy as np
import pytest

from gpu_util import announce, rel_err, require_gpu, to_dev, to_host
from oracle import allatonce, stepping

pytestmark = pytest.mark.gpu


def _solve_vs_stepping(dim, n, s, nt, T=1.0, disc="fd", length=1.0, tol=1e-12, **kw):
    from paper_2609_16863_amd import HeatProblem
    p = allatonce.Problem(n, dim, s, nt, T, disc=disc, length=length)
    hp = HeatProblem(dim, n, s, nt, T, disc=disc, length=length, tol=tol, maxit=300, **kw)
    rng = np.random.default_rng(n * 100 + nt)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    announce("edge", dim, n, s, nt, disc, kw)
    x, st = hp.solve(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
    return st, rel_err(to_host(x), stepping.solve(p, f, u0))


@pytest.mark.parametrize("dim,n,s,nt", [(2, 2, 1, 1), (2, 3, 3, 1), (3, 2, 2, 1), (2, 5, 1, 2)])
def test_smallest_problems(dim, n, s, nt):
    require_gpu()
    st, err = _solve_vs_stepping(dim, n, s, nt)
    assert st["converged"] and err <= 1e-10, (st, err)


@pytest.mark.parametrize("nt,cf,fcf", [(3, 8, False), (9, 4, False), (11, 4, True), (5, 2, True)])
def test_mgrit_short_and_ragged_time_grids(nt, cf, fcf):
    require_gpu()
    st, err = _solve_vs_stepping(2, 20, 2, nt, schur="mgrit", mgrit_cf=cf, mgrit_fcf=fcf, precision="fp32")
    assert st["converged"] and err <= 1e-9, (st, err)


def test_left_preconditioning_with_mgrit():
    require_gpu()
    st, err = _solve_vs_stepping(2, 24, 3, 8, side="left", inner_k=10, schur="mgrit", mgrit_cf=4)
    assert st["converged"] and err <= 1e-8, (st, err)


@pytest.mark.parametrize("precision", ["fp64", "fp16_all"])
def test_q1_with_mgrit(precision):
    require_gpu()
    st, err = _solve_vs_stepping(2, 31, 2, 10, disc="q1", length=2.0, tol=1e-11, schur="mgrit", mgrit_cf=4,
                                 precision=precision)
    assert st["converged"] and err <= 1e-8, (st, err)
