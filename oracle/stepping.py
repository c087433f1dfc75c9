"""Sequential Radau IIA time stepping: the exact solution of eq. (2.4).

Test infrastructure only (see ``oracle/__init__.py``).

Paper, Sec. 2: starting from v_0 = u0, for n = 0..nt-1 solve the stage system
eq. (2.3), (I_s (x) M + tau A (x) K) V_n = f_n - (e (x) K) v_n, then update
with eq. (2.2), v_{n+1} = v_n + tau sum_i b_i V_{n,i}.  Ordered by time the
all-at-once matrix is block lower triangular with nonsingular diagonal blocks,
so this stepping yields its unique solution x* (the result every FGMRES solve
of eq. (2.4) converges to).  The stage right-hand side is f_n - (e (x) K) v_n:
the paper prints "f_n - K v_n"; the Psi2 = e (x) K block fixes the reading.

With finite elements (prob.disc "q1" or "q2") the stage right-hand side is the load
vector M f_n (f_n at the nodes) and v_0 = u0 (b_0 = M u0); the update needs
no mass solve since every term of eq. (2.2) carries M.

Two exact stage solvers:
* ``"lu"``  -- sparse LU (SuperLU) of the stage matrix, factored once.
* ``"dst"`` -- constant diffusivity only: K is diagonalised by the
  orthonormal DST-I along each axis; each mode needs one s x s solve.

Pinned by: the closed-form discrete solution of the sin-sin-exp problem,
temporal order 2s-1, agreement with a dense solve of eq. (2.4), and LU == DST
(tests/test_oracle_stepping.py).
"""
import time

import numpy as np
import scipy.fft
import scipy.sparse.linalg as spla

from . import allatonce, grid


def _dst(x, dim, workers):
    axes = tuple(range(-dim, 0))
    return scipy.fft.dstn(x, type=1, norm="ortho", axes=axes, workers=workers)


def solve(prob, f, u0, method="auto", workers=None, timings=None):
    """Return x* = [v; V] (FP64, layout of eq. (2.4)) by sequential stepping.

    f: stage right-hand sides, shape (nt, s, N) (or flat); u0: (N,).
    ``timings`` (dict, optional) receives 'factor_s' and 'step_s'.
    """
    if method == "auto":
        method = "dst" if prob.kappa is None and prob.disc == "fd" else "lu"
    nt, s, N, tau = prob.nt, prob.s, prob.N, prob.tau
    f = np.asarray(f, float).reshape(nt, s, N)
    v = np.empty((nt + 1, N))
    V = np.empty((nt, s, N))
    v[0] = u0
    t0 = time.perf_counter()
    if method == "lu":
        K = prob.K()
        lu = spla.splu(allatonce.theta_hat(prob, K))
        if prob.fe:
            Mm = prob.M()
            f = (Mm @ f.reshape(-1, N).T).T.reshape(nt, s, N)
        t1 = time.perf_counter()
        for n in range(nt):
            Kv = K @ v[n]
            r = (f[n] - Kv[None, :]).ravel()
            V[n] = lu.solve(r).reshape(s, N)
            v[n + 1] = v[n] + tau * np.tensordot(prob.b, V[n], axes=(0, 0))
    elif method == "dst":
        if prob.kappa is not None or prob.disc != "fd":
            raise ValueError("DST stepping needs finite differences with constant diffusivity")
        shape = grid.field_shape(prob.n, prob.dim)
        lam = grid.dst_eigenvalues(prob.n, prob.dim).ravel()
        # per-mode inverse of I + tau lam A  (N, s, s)
        Mm = np.eye(s)[None] + tau * lam[:, None, None] * prob.A[None]
        Minv = np.linalg.inv(Mm)
        t1 = time.perf_counter()
        vhat = _dst(v[0].reshape(shape), prob.dim, workers).ravel()
        for n in range(nt):
            fhat = _dst(f[n].reshape((s,) + shape), prob.dim, workers).reshape(s, N)
            rhat = fhat - (lam * vhat)[None, :]
            Vhat = np.einsum("mij,jm->im", Minv, rhat)
            V[n] = _dst(Vhat.reshape((s,) + shape), prob.dim, workers).reshape(s, N)
            v[n + 1] = v[n] + tau * np.tensordot(prob.b, V[n], axes=(0, 0))
            vhat = vhat + tau * np.tensordot(prob.b, Vhat, axes=(0, 0))
    else:
        raise ValueError(method)
    t2 = time.perf_counter()
    if timings is not None:
        timings["factor_s"] = t1 - t0
        timings["step_s"] = t2 - t1
        timings["method"] = method
    return allatonce.join(v, V)


def solve_steps(prob, f, u0, nsteps, method="auto", workers=None, timings=None):
    """Run only the first ``nsteps`` steps (a bounded sample for timing)."""
    sub = allatonce.Problem(prob.n, prob.dim, prob.s, nsteps, prob.tau * nsteps, prob.kappa, prob.disc,
                            prob.length)
    f = np.asarray(f, float).reshape(prob.nt, prob.s, prob.N)[:nsteps]
    return solve(sub, f, u0, method=method, workers=workers, timings=timings)
