"""Closed-form discrete solution of the sin-sin-exp manufactured problem.

Test infrastructure only (see ``oracle/__init__.py``).

For u = sin(pi x) sin(pi y) e^{-t} on the unit square, u_t - Lap u = f gives
f = (2 pi^2 - 1) sin(pi x) sin(pi y) e^{-t}.  The grid function
phi = sin(pi x) sin(pi y) is an exact eigenvector of the 5-point K with
eigenvalue lam_h = (8/h^2) sin^2(pi h / 2), and f and u0 are multiples of
phi, so the solution of eq. (2.4) is phi times a scalar sequence:
    y_0 = 1;  (I_s + tau lam_h A) Y_n = F_n - lam_h y_n e,
    F_{n,i} = (2 pi^2 - 1) e^{-(t_n + c_i tau)};  y_{n+1} = y_n + tau b^T Y_n.
The semi-discrete (exact in time) solution is
    y(t) = alpha e^{-t} + (1 - alpha) e^{-lam_h t},  alpha = (2 pi^2 - 1)/(lam_h - 1).

Pinned by: the sequential-stepping oracle (an independent code path) and the
temporal order 2s-1 of Radau IIA against the semi-discrete y(t)
(tests/test_oracle_stepping.py).
"""
import numpy as np

from . import allatonce


def eigenvalue(n):
    h = 1.0 / (n + 1)
    return 8.0 / (h * h) * np.sin(np.pi * h / 2.0) ** 2


def scalar_sequence(prob):
    """(y of shape (nt+1,), Y of shape (nt, s)) for the 2D sin-sin-exp problem."""
    lam = eigenvalue(prob.n)
    s, tau = prob.s, prob.tau
    y = np.empty(prob.nt + 1)
    Y = np.empty((prob.nt, s))
    y[0] = 1.0
    Mat = np.eye(s) + tau * lam * prob.A
    for n in range(prob.nt):
        F = (2 * np.pi ** 2 - 1) * np.exp(-(n * tau + prob.c * tau))
        Y[n] = np.linalg.solve(Mat, F - lam * y[n])
        y[n + 1] = y[n] + tau * prob.b @ Y[n]
    return y, Y


def solution(prob, phi):
    """Full x* = [v; V] for the problem whose data are multiples of phi."""
    y, Y = scalar_sequence(prob)
    v = y[:, None] * phi[None, :]
    V = Y[:, :, None] * phi[None, None, :]
    return allatonce.join(v, V)


def semidiscrete(n, t):
    lam = eigenvalue(n)
    alpha = (2 * np.pi ** 2 - 1) / (lam - 1)
    return alpha * np.exp(-t) + (1 - alpha) * np.exp(-lam * t)
