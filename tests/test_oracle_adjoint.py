"""Pins of the oracle's adjoint solve and gradients (not gpu)."""
import numpy as np
import pytest

from oracle import adjoint, allatonce, stepping


@pytest.mark.parametrize("dim,n,s,nt", [(2, 3, 2, 3), (2, 4, 3, 2), (3, 2, 2, 2)])
def test_adjoint_equals_dense_transpose_solve(dim, n, s, nt):
    rng = np.random.default_rng(21)
    p = allatonce.Problem(n, dim, s, nt, 1.0, kappa=np.exp(rng.standard_normal(n ** dim)))
    g = rng.standard_normal(p.U)
    lam = adjoint.solve(p, g)
    Ad = allatonce.operator(p, sparse=False)
    ref = np.linalg.solve(Ad.T, g)
    assert np.linalg.norm(lam - ref) <= 1e-12 * np.linalg.norm(ref)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(22)
    n, s, nt = 5, 2, 4
    theta = 0.5 * rng.standard_normal(n * n)
    p = allatonce.Problem(n, 2, s, nt, 0.5, kappa=np.exp(theta))
    f = rng.standard_normal((nt, s, p.N))
    u0 = rng.standard_normal(p.N)
    vt = rng.standard_normal((nt + 1) * p.N)
    L, gf, gu0, gth = adjoint.gradients(p, f, u0, vt)

    def loss(f_, u0_, th_):
        q = allatonce.Problem(n, 2, s, nt, 0.5, kappa=np.exp(th_))
        return adjoint.tracking_loss(q, stepping.solve(q, f_, u0_, method="lu"), vt)

    assert abs(loss(f, u0, theta) - L) < 1e-12 * abs(L)
    for k in range(6):
        df = rng.standard_normal(f.shape)
        du = rng.standard_normal(u0.shape)
        dth = rng.standard_normal(theta.shape)
        eps = 1e-5
        fd = (loss(f + eps * df, u0 + eps * du, theta + eps * dth)
              - loss(f - eps * df, u0 - eps * du, theta - eps * dth)) / (2 * eps)
        an = np.sum(gf * df) + gu0 @ du + gth @ dth
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, fd, an)
