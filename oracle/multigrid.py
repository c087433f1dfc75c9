"""Geometric multigrid V-cycle for the shifted blocks M + a K (M = I for
finite differences, the Q1 or Q2 mass matrix for finite elements).  For Q2
elements the coarse nodes (every second node) are the element vertices.

Test infrastructure only (see ``oracle/__init__.py``).

Paper, Sec. 4 and Sec. 5: applying the preconditioner needs an inexact inverse
of matrices of the form M + c K, done by a multigrid routine (the paper's runs
use an algebraic multigrid library; here it is geometric multigrid).  The
hierarchy and cycle below are this project's reading; they only affect
iteration counts, never the solution of eq. (2.4).

* Coarse nodes are every second fine node, 1-based fine indices 2, 4, ...,
  2 floor(n/2), so n_c = floor(n/2); coarsening stops once a level has at
  most ``coarse_max`` nodes (default COARSE_MAX = 256) and there are at
  least ``min_levels`` levels, and that level is solved exactly (Q2 elements
  take min_levels = 2: their fine level is always smoothed).
* Prolongation P: (tensor-)linear interpolation, boundary values zero.
* Restriction R = P^T / 2^d (full weighting); coarse operator R A P
  (Galerkin), so every level is symmetric positive definite.
* Smoother: weighted Jacobi x <- x + omega D^{-1} (b - A x), nu1 sweeps before
  and nu2 after the coarse correction; zero initial guess; exact solve on the
  coarsest level.
* ``cycles`` V-cycles are applied as a stationary iteration from x = 0.

Pinned by: convergence of repeated cycles to the direct solve, the
interpolation being exact for piecewise-linear grid functions, the Galerkin
operators of the constant-coefficient case equalling the Kronecker form built
from 1D Galerkin factors, and a measured contraction factor
(tests/test_oracle_multigrid.py).
"""
import numpy as np
import scipy.sparse as sp


COARSE_MAX = 256


def coarse_size(n):
    return n // 2


def interpolation_1d(n):
    """1D linear interpolation from floor(n/2) coarse to n fine interior nodes."""
    nc = coarse_size(n)
    rows, cols, vals = [], [], []
    for J in range(nc):
        f = 2 * J + 1                 # 0-based fine index of coarse node J
        rows += [f, f - 1]
        cols += [J, J]
        vals += [1.0, 0.5]
        if f + 1 < n:
            rows.append(f + 1)
            cols.append(J)
            vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def interpolation(n, dim):
    P1 = interpolation_1d(n)
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    return P


class Hierarchy:
    """Levels (A_l, P_l) for A_0 = M + a K (M = I unless given)."""

    def __init__(self, K, n, dim, a, coarse_max=COARSE_MAX, M=None, min_levels=1):
        self.dim = dim
        self.sizes = [n]
        M0 = sp.identity(K.shape[0], format="csr") if M is None else M
        self.ops = [(M0 + a * K).tocsr()]
        self.P = []
        while (self.sizes[-1] ** dim > coarse_max or len(self.ops) < min_levels) and self.sizes[-1] > 1:
            nf = self.sizes[-1]
            P = interpolation(nf, dim)
            R = P.T / (2.0 ** dim)
            self.P.append(P)
            self.ops.append((R @ self.ops[-1] @ P).tocsr())
            self.sizes.append(coarse_size(nf))

    @property
    def levels(self):
        return len(self.ops)


def jacobi(A, x, b, omega, sweeps):
    d = A.diagonal()
    for _ in range(sweeps):
        x = x + omega * (b - A @ x) / d
    return x


def vcycle(H, b, level=0, omega=0.8, nu1=1, nu2=1):
    """One V-cycle from a zero initial guess on ``level``."""
    A = H.ops[level]
    if level == H.levels - 1:
        return np.linalg.solve(A.toarray(), b)
    x = jacobi(A, np.zeros_like(b), b, omega, nu1)
    r = b - A @ x
    P = H.P[level]
    bc = (P.T @ r) / (2.0 ** H.dim)
    ec = vcycle(H, bc, level + 1, omega, nu1, nu2)
    x = x + P @ ec
    return jacobi(A, x, b, omega, nu2)


def solve(H, b, cycles=1, omega=0.8, nu1=1, nu2=1):
    """``cycles`` V-cycles as a stationary iteration from zero."""
    x = np.zeros_like(b)
    for _ in range(cycles):
        x = x + vcycle(H, b - H.ops[0] @ x, 0, omega, nu1, nu2)
    return x
