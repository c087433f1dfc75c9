"""GPU parity of the all-at-once operator (apply_A / apply_AT), RHS assembly and
the log-kappa gradient against the oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu, to_dev, to_host
from oracle import adjoint, allatonce

pytestmark = pytest.mark.gpu

# tiny (dense), ragged tails (N not a multiple of the 256-thread tile), 3D
CASES = [(2, 3, 1, 3, False), (2, 4, 2, 4, True), (2, 5, 3, 2, False), (3, 3, 2, 3, False),
         (3, 3, 3, 2, True), (2, 37, 3, 5, False), (2, 37, 2, 5, True), (3, 11, 3, 3, False),
         # 2D row-marching tiles (64 rows; 512 columns for even n, 256 for odd n), ragged in x and y
         (2, 300, 3, 2, False), (2, 270, 2, 2, True), (2, 530, 1, 1, False), (2, 301, 1, 2, True),
         # 3D z-marching (32 planes per thread, 64 x 2 columns per wave for even n, 64 for odd n):
         # ragged x, y and z; several x blocks
         (3, 40, 3, 2, False), (3, 33, 2, 2, False), (3, 130, 1, 1, False), (3, 67, 2, 1, False)]


def _setup(dim, n, s, nt, vk, seed):
    from paper_2609_16863_amd import HeatProblem
    rng = np.random.default_rng(seed)
    kappa = np.exp(rng.standard_normal(n ** dim)) if vk else None
    if dim == 3 and vk:
        kappa = None   # variable diffusivity is 2D only
    p = allatonce.Problem(n, dim, s, nt, 0.9, kappa=kappa)
    hp = HeatProblem(dim, n, s, nt, 0.9, kappa=kappa)
    return p, hp, rng


def _bound(p, x):
    """Scale of the rounding error of one row: sum_j |A_ij| |x_j| <= (1 + 4 d tau kmax / h^2) |x|_max."""
    kmax = 1.0 if p.kappa is None else float(np.max(p.kappa))
    return 8 * (1 + 4 * p.dim * kmax * (1 + p.tau) / p.h ** 2 * 3) * np.abs(x).max()


@pytest.mark.parametrize("dim,n,s,nt,vk", CASES)
def test_apply_A_and_AT_match_oracle(dim, n, s, nt, vk):
    require_gpu()
    p, hp, rng = _setup(dim, n, s, nt, vk, 100 + n)
    announce("apply_A", dim, n, s, nt, vk)
    x = rng.standard_normal(p.U)
    y = to_host(hp.apply_A(to_dev(x)))
    yt = to_host(hp.apply_AT(to_dev(x)))
    if p.U <= 4000:
        Ad = allatonce.operator(p, sparse=False)
        ref, reft = Ad @ x, Ad.T @ x
    else:
        ref = allatonce.apply_blockwise(p, x)
        reft = allatonce.apply_blockwise(p, x, transpose=True)
    tol = 1e-15 * _bound(p, x)
    assert np.abs(y - ref).max() <= tol
    assert np.abs(yt - reft).max() <= tol


def test_assemble_rhs_matches_oracle():
    require_gpu()
    p, hp, rng = _setup(2, 19, 3, 4, False, 7)
    f = rng.standard_normal((4, 3, p.N))
    u0 = rng.standard_normal(p.N)
    r = to_host(hp.assemble_rhs(to_dev(f.ravel()), to_dev(u0)))
    assert np.array_equal(r, allatonce.rhs(p, f, u0))


@pytest.mark.parametrize("vk", [False, True])
def test_grad_logkappa_matches_oracle(vk):
    require_gpu()
    p, hp, rng = _setup(2, 13, 2, 3, vk, 9)
    x = rng.standard_normal(p.U)
    lam = rng.standard_normal(p.U)
    announce("grad_logkappa", vk)
    g = to_host(hp.grad_logkappa(to_dev(x), to_dev(lam)))
    ref = adjoint.grad_logkappa(p, x, lam)
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_full_size_sampled_rows():
    """512^2, s=3, nt=64 (the benchmark workload): sampled rows vs the oracle."""
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    n, s, nt = 512, 3, 64
    p = allatonce.Problem(n, 2, s, nt, 1.0)
    hp = HeatProblem(2, n, s, nt, 1.0, restart=1, inner_k=1)
    rng = np.random.default_rng(2024)
    x = rng.standard_normal(p.U)
    announce("apply_A full size", p.U)
    y = to_host(hp.apply_A(to_dev(x)))
    K = p.K()
    rows = np.concatenate([rng.integers(0, p.U, 3000), [0, p.N - 1, (nt + 1) * p.N - 1, p.U - 1]])
    ref = allatonce.apply_rows(p, x, rows, K)
    assert np.abs(y[rows] - ref).max() <= 1e-15 * _bound(p, x)
    # whole-vector property: v_0 rows are the identity
    assert np.array_equal(y[: p.N], x[: p.N])
