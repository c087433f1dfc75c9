"""HIP-graph replay of the preconditioner equals direct launches, bitwise.

Each replay is separated by eager work and synchronisations, and every replay
is checked against the directly launched result (the kernels are
deterministic, so the comparison is exact)."""
import numpy as np
import pytest
import torch

from gpu_util import announce, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


# the MGRIT cases fork its last F-relaxation into concurrent chains: graph
# branches when captured, side streams when launched directly
@pytest.mark.parametrize("precision,dim,n,s,nt,mgrit", [("fp64", 2, 40, 3, 4, 0), ("fp32", 2, 72, 2, 3, 0),
                                                        ("bf16", 2, 33, 2, 2, 0), ("fp32", 3, 12, 2, 2, 0),
                                                        ("fp32", 2, 40, 3, 16, 4), ("fp64", 2, 33, 2, 13, 3)])
def test_graph_replay_is_bitwise_equal_to_direct(precision, dim, n, s, nt, mgrit):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    kw = dict(schur="mgrit", mgrit_cf=mgrit) if mgrit else {}
    hg = HeatProblem(dim, n, s, nt, 1.0, precision=precision, use_graph=True, **kw)
    hd = HeatProblem(dim, n, s, nt, 1.0, precision=precision, use_graph=False, **kw)
    rng = np.random.default_rng(9)
    r1, r2 = to_dev(rng.standard_normal(hg.U)), to_dev(rng.standard_normal(hg.U))
    announce("graph replay", precision, dim, n, s, nt, mgrit)
    z1, z2 = to_host(hd.apply_P(r1)), to_host(hd.apply_P(r2))
    for rep in range(3):
        g1 = to_host(hg.apply_P(r1))
        junk = (r2 * 3.0 + 1.0).sum()          # eager work between replays
        torch.cuda.synchronize()
        g2 = to_host(hg.apply_P(r2))
        assert np.array_equal(g1, z1), rep
        assert np.array_equal(g2, z2), rep
        assert np.isfinite(float(junk))


def test_graph_solve_matches_direct_solve():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    import heat_inputs
    kw = dict(precision="fp32", tol=1e-10)
    hg = HeatProblem(2, 48, 3, 6, 1.0, use_graph=True, **kw)
    hd = HeatProblem(2, 48, 3, 6, 1.0, use_graph=False, **kw)
    rng = np.random.default_rng(4)
    f = heat_inputs.bump_source(rng, 48, 2, hg.stage_times())
    u0 = heat_inputs.smooth_initial(rng, 48, 2)
    rhs = hg.assemble_rhs(to_dev(f.ravel()), to_dev(u0))
    announce("graph solve")
    xg, sg = hg.solve(rhs)
    xd, sd = hd.solve(rhs)
    assert sg["outer_iterations"] == sd["outer_iterations"]
    assert np.array_equal(to_host(xg), to_host(xd))
