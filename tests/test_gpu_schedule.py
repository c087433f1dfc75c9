"""Precision schedules of the V-cycle on the GPU (Sec. 4 cites per-level
decreasing precision, and a coarse-solve precision apart from the
smoother's, as ways to run the multigrid in mixed precision).

With the BF16/FP16 preconditioners, ``mg_low_from`` is the first multigrid
level stored in 16 bits (the levels above it stay FP32) and
``mg_coarse_fp32`` keeps the coarse solve (2D: the one-workgroup tail with
its exact coarsest solve; 3D: the exact coarsest level) in FP32.

* A schedule with no 16-bit level is the FP32 V-cycle bit for bit (the FP16
  levels' power-of-two scale is exact in FP32).
* Every schedule stays within the 16-bit bound of the oracle's exact V-cycle
  (2D constant and variable kappa, through the grid kernels, the one- and
  two-level register tails; 3D through the grid kernels), and moving
  levels to FP32 changes the result (the schedule is really applied).
* Iteration counts of the full solve stay flat across schedules (trend).
* The outer products with A in lowered precision as the residual falls
  (``relax_matvec``; Sec. 4 names the relaxation as future work): the GPU
  rounds the same products to the same tiers as the oracle's Algorithm 1
  on the same problem, and still reaches the target and x*.
"""
import numpy as np
import pytest

import heat_inputs
from gpu_util import announce, rel_err, require_gpu, to_dev
from gpu_util import to_host
from oracle import allatonce, multigrid, precond, stepping, tableau

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _oracle(p, stage, r_blocks):
    L, _ = tableau.crout(p.A)
    H = multigrid.Hierarchy(p.K(), p.n, p.dim, p.tau * L[stage, stage], multigrid.COARSE_MAX)
    omega = 0.8 if p.dim == 2 else 6.0 / 7.0
    return np.stack([multigrid.solve(H, b, 1, omega, 2, 2) for b in r_blocks])


def _cycle(hp, r, stage):
    rd = torch.from_numpy(np.ascontiguousarray(r.ravel())).to(hp.working_dtype()).cuda()
    z = hp.apply_mg(rd, stage, cycles=1)
    torch.cuda.synchronize()
    return z.double().cpu().numpy().reshape(r.shape)


# 2D: 150 (two-level register tail), 130 (one-level tail), 75 with variable
# kappa (stored 9-point stencils); 3D: 17 (grid kernels, exact coarsest level)
@pytest.mark.parametrize("dim,n,vark", [(2, 150, False), (2, 130, False), (2, 75, True), (3, 17, False)])
@pytest.mark.parametrize("precision,tol", [("fp16", 1e-3), ("bf16", 3e-2)])
def test_schedules_against_oracle_and_fp32(dim, n, vark, precision, tol):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    s, nt = 2, 3
    rng = np.random.default_rng(19 + n)
    kappa = np.exp(0.5 * rng.standard_normal(n ** dim)) if vark else None
    p = allatonce.Problem(n, dim, s, nt, 1.0, kappa=kappa)
    r = rng.standard_normal((nt, p.N))
    ref = _oracle(p, 1, r)
    z32 = _cycle(HeatProblem(dim, n, s, nt, 1.0, precision="fp32", kappa=kappa), r, 1)
    nodes, tail = HeatProblem(dim, n, s, nt, 1.0, precision=precision, kappa=kappa).mg_levels()
    levels = len(nodes)
    out = {}
    for low_from, coarse32 in [(1, False), (2, False), (tail if dim == 2 else levels - 1, False), (1, True),
                               (levels, False)]:
        hp = HeatProblem(dim, n, s, nt, 1.0, precision=precision, kappa=kappa, mg_low_from=low_from,
                         mg_coarse_fp32=coarse32)
        announce("schedule", dim, n, vark, precision, low_from, coarse32)
        z = _cycle(hp, r, 1)
        out[low_from, coarse32] = z
        assert rel_err(z, ref) <= tol, (low_from, coarse32, rel_err(z, ref))
    print({k: rel_err(v, ref) for k, v in out.items()}, "fp32", rel_err(z32, ref))
    # no 16-bit level: the FP32 cycle, bit for bit
    assert np.array_equal(out[levels, False], z32)
    # the schedules do change the arithmetic
    assert not np.array_equal(out[1, True], out[1, False])
    assert not np.array_equal(out[2, False], out[1, False])


def test_default_schedule_is_the_previous_two_tier_cycle():
    """mg_low_from = 0 and = 1 are the same schedule (every coarse level in
    16 bits)."""
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 150, 2, 3
    r = np.random.default_rng(3).standard_normal((nt, n * n))
    a = _cycle(HeatProblem(2, n, s, nt, 1.0, precision="fp16"), r, 0)
    b = _cycle(HeatProblem(2, n, s, nt, 1.0, precision="fp16", mg_low_from=1), r, 0)
    assert np.array_equal(a, b)


def test_solve_iterations_flat_across_schedules():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 128, 3, 16
    its = {}
    for prec, low_from, coarse32 in [("fp32", 0, False), ("fp16", 1, False), ("fp16", 3, False),
                                     ("fp16", 1, True), ("bf16", 1, False), ("bf16", 2, True)]:
        hp = HeatProblem(2, n, s, nt, 1.0, precision=prec, inner_k=3, tol=1e-8, mg_low_from=low_from,
                         mg_coarse_fp32=coarse32)
        rng = np.random.default_rng(1001)
        f = heat_inputs.bump_source(rng, n, 2, hp.stage_times())
        u0 = heat_inputs.smooth_initial(rng, n, 2)
        announce("schedule solve", prec, low_from, coarse32)
        _, st = hp.solve(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
        assert st["converged"], (prec, low_from, coarse32, st["relres"])
        its[prec, low_from, coarse32] = st["outer_iterations"]
    print(its)
    base = its["fp32", 0, False]
    assert all(abs(v - base) <= 2 for v in its.values()), its


def test_relaxed_matvec_matches_oracle_tiers_and_reaches_the_solution():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt, T = 12, 2, 6, 0.8
    rng = np.random.default_rng(31)
    p = allatonce.Problem(n, 2, s, nt, T)
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    ops = precond.StageOps(p, inner_k=3, nu1=2, nu2=2)
    K = p.K()
    rhs = allatonce.rhs(p, f, u0)
    xs = stepping.solve(p, f, u0)
    for tol in (1e-8, 1e-11):
        st_o = {}
        _, its_o, _ = precond.fgmres_split(lambda y: allatonce.apply_blockwise(p, y, K), None,
                                           lambda r: precond.apply_preconditioner(ops, r), rhs, restart=30,
                                           tol=tol, maxit=60, relax=True, stats=st_o)
        hp = HeatProblem(2, n, s, nt, T, tol=tol, maxit=60, inner_k=3, relax_matvec=True)
        announce("relaxed matvec", tol)
        x, st = hp.solve(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
        print(tol, st["outer_iterations"], st["relaxed_fp32"], st["relaxed_bf16"], st["relres"], "oracle", its_o,
              st_o)
        assert st["converged"] and st["relres"] <= tol
        assert abs(st["outer_iterations"] - its_o) <= 1
        assert abs(st["relaxed_fp32"] - st_o.get("fp32", 0)) <= 1
        assert abs(st["relaxed_bf16"] - st_o.get("bf16", 0)) <= 1
        assert st["relaxed_fp32"] + st["relaxed_bf16"] >= 2
        if tol == 1e-11:
            assert rel_err(to_host(x), xs) <= 1e-8
