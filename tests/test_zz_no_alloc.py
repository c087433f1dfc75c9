"""aao_solve_no_alloc through the C ABI against aao_solve.

The no-allocation variant runs the same kernels with the workspace placed in
the library's static device scratch.  Two calls in a row, the second on a
smaller problem, each equal to aao_solve on the same input; a problem larger
than the scratch is rejected.
"""
import ctypes

import numpy as np
import pytest

import heat_inputs
from gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _no_alloc_solve(hp, rhs):
    from paper_2609_16863_amd import _abi
    from paper_2609_16863_amd.binding import _ptr
    lib = _abi.load()
    x = torch.zeros_like(rhs)
    st = _abi.Stats()
    hp._sync_stream()
    code = lib.aao_solve_no_alloc(hp._h, _ptr(rhs), _ptr(x), ctypes.byref(st))
    torch.cuda.synchronize()
    return code, x, st


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_no_alloc_solve_equals_solve_twice(precision):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    cases = [(40, 3, 8), (24, 2, 5)]   # the second call is smaller
    for n, s, nt in cases:
        hp = HeatProblem(2, n, s, nt, 1.0, tol=1e-10, precision=precision)
        rng = np.random.default_rng(100 + n)
        f = heat_inputs.bump_source(rng, n, 2, hp.stage_times())
        u0 = heat_inputs.smooth_initial(rng, n, 2)
        rhs = hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0))
        announce("no_alloc", precision, n, s, nt)
        x_ref, st_ref = hp.solve(rhs)
        code, x, st = _no_alloc_solve(hp, rhs)
        assert code == 0, hp._lib.aao_last_error(hp._h)
        assert st.outer_iterations == st_ref["outer_iterations"]
        assert abs(st.relres - st_ref["relres"]) <= 1e-14
        err = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
        assert err <= 1e-13, err
        # the handle's own workspace still works afterwards
        x_again, _ = hp.solve(rhs)
        assert torch.equal(x_again, x_ref)


def test_no_alloc_rejects_problem_beyond_scratch():
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    hp = HeatProblem(2, 256, 3, 16, 1.0, precision="fp32")
    assert hp.workspace_bytes() > 64 << 20
    rhs = torch.ones(hp.U, dtype=torch.float64, device="cuda")
    announce("no_alloc too large")
    code, x, st = _no_alloc_solve(hp, rhs)
    assert code == -4
    assert b"static scratch" in hp._lib.aao_last_error(hp._h)
