"""Adjoint (transpose) all-at-once solve and gradients.

Test infrastructure only (see ``oracle/__init__.py``).

The transposed system A^T lam = g of eq. (2.4) is block upper triangular in
time, so it is solved by stepping backwards.  Transposing the blocks of
Sec. 2 (M = I, K symmetric):

    lam_{v,nt} = g_{v,nt}
    for n = nt-1 .. 0:
        (I_s (x) I + tau A^T (x) K) lam_{V,n} = g_{V,n} + tau (b (x) I) lam_{v,n+1}
        lam_{v,n} = g_{v,n} + lam_{v,n+1} - K sum_i lam_{V,n,i}

Gradients of a loss L(v) through the solve (A(theta) x = [b(u0); f]):
    dL/df_{n,i} = lam_{V,n,i},   dL/du0 = lam_{v,0},
    dL/dtheta_p = - sum_{n,i} lam_{V,n,i}^T (dK/dtheta_p) w_{n,i},
    w_{n,i} = v_n + tau sum_j a_ij V_{n,j},
with theta = log kappa at the nodes and K = sum over faces of
kappa_f / h^2 (e_p - e_q)(e_p - e_q)^T (boundary faces: e_p e_p^T).

Pinned by: a dense solve with the transposed matrix on tiny grids, the dot
test <A x, y> = <x, A^T y>, and central finite differences of the oracle's
own forward solve (tests/test_oracle_adjoint.py).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import allatonce, grid


def solve(prob, g):
    """lam = A^{-T} g by reverse stepping with an LU of the stage matrix."""
    nt, s, N, tau = prob.nt, prob.s, prob.N, prob.tau
    gv, gV = allatonce.split(prob, np.asarray(g, float))
    K = prob.K()
    lu = spla.splu(allatonce.theta_hat(prob, K))
    lv = np.empty((nt + 1, N))
    lV = np.empty((nt, s, N))
    lv[nt] = gv[nt]
    for n in range(nt - 1, -1, -1):
        r = gV[n] + tau * prob.b[:, None] * lv[n + 1][None, :]
        lV[n] = lu.solve(r.ravel(), trans="T").reshape(s, N)
        lv[n] = gv[n] + lv[n + 1] - K @ lV[n].sum(axis=0)
    return allatonce.join(lv, lV)


def stage_mixed_fields(prob, x):
    """w_{n,i} = v_n + tau sum_j a_ij V_{n,j}, shape (nt, s, N)."""
    v, V = allatonce.split(prob, np.asarray(x, float))
    return v[:-1, None, :] + prob.tau * np.einsum("ij,njp->nip", prob.A, V)


def grad_logkappa(prob, x, lam):
    """dL/dtheta (N values) from the forward solution x and adjoint lam."""
    n, dim, h = prob.n, prob.dim, prob.h
    shape = grid.field_shape(n, dim)
    kap = np.ones(shape) if prob.kappa is None else np.asarray(prob.kappa, float).reshape(shape)
    _, lV = allatonce.split(prob, np.asarray(lam, float))
    w = stage_mixed_fields(prob, x)
    L = lV.reshape((-1,) + shape)
    W = w.reshape((-1,) + shape)
    G = np.zeros(shape)
    for ax in range(dim):
        ax1 = ax + 1                                  # skip the (n, i) axis
        sl_lo = [slice(None)] * (dim + 1)
        sl_hi = [slice(None)] * (dim + 1)
        sl_lo[ax1] = slice(0, n - 1)
        sl_hi[ax1] = slice(1, n)
        dl = L[tuple(sl_lo)] - L[tuple(sl_hi)]
        dw = W[tuple(sl_lo)] - W[tuple(sl_hi)]
        face = (dl * dw).sum(axis=0) / (h * h)        # d(lam^T K w)/d kappa_f
        klo = np.take(kap, np.arange(0, n - 1), axis=ax)
        khi = np.take(kap, np.arange(1, n), axis=ax)
        dk_dlo = 2.0 * khi ** 2 / (klo + khi) ** 2
        dk_dhi = 2.0 * klo ** 2 / (klo + khi) ** 2
        lo_sl = [slice(None)] * dim
        hi_sl = [slice(None)] * dim
        lo_sl[ax] = slice(0, n - 1)
        hi_sl[ax] = slice(1, n)
        G[tuple(lo_sl)] += face * dk_dlo * klo
        G[tuple(hi_sl)] += face * dk_dhi * khi
        for end in (0, n - 1):
            bsl = [slice(None)] * (dim + 1)
            bsl[ax1] = slice(end, end + 1)
            fb = (L[tuple(bsl)] * W[tuple(bsl)]).sum(axis=0) / (h * h)
            gsl = [slice(None)] * dim
            gsl[ax] = slice(end, end + 1)
            G[tuple(gsl)] += fb * kap[tuple(gsl)]
    return -G.ravel()


def tracking_loss(prob, x, v_target):
    """L = 1/2 sum_{n=1..nt} ||v_n - v_n^tgt||^2 (v_0 = u0 is data)."""
    v, _ = allatonce.split(prob, np.asarray(x, float))
    vt = np.asarray(v_target, float).reshape(prob.nt + 1, prob.N)
    d = v[1:] - vt[1:]
    return 0.5 * float(np.sum(d * d))


def tracking_loss_grad_x(prob, x, v_target):
    """dL/dx = [0; v_1 - v_1^tgt; ...; 0 for the stage blocks]."""
    v, _ = allatonce.split(prob, np.asarray(x, float))
    vt = np.asarray(v_target, float).reshape(prob.nt + 1, prob.N)
    gv = np.zeros_like(v)
    gv[1:] = v[1:] - vt[1:]
    return allatonce.join(gv, np.zeros((prob.nt, prob.s, prob.N)))


def gradients(prob, f, u0, v_target):
    """Loss and its gradients w.r.t. (f, u0, log kappa) via the adjoint."""
    from . import stepping
    x = stepping.solve(prob, f, u0, method="lu")
    L = tracking_loss(prob, x, v_target)
    lam = solve(prob, tracking_loss_grad_x(prob, x, v_target))
    lv, lV = allatonce.split(prob, lam)
    return L, lV.copy(), lv[0].copy(), grad_logkappa(prob, x, lam)
