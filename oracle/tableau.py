"""Radau IIA Butcher tableau and the Crout factor used by Rana's preconditioner.

Test infrastructure only (see ``oracle/__init__.py``).

Paper: Sec. 2 defines a Runge--Kutta method by its tableau (A_RK, b_RK, c_RK);
Sec. 5 uses the Radau IIA family.  The tableau is not printed in the paper; it
is the collocation method whose nodes are the right Radau points.

Pinned by: order conditions B(2s-1) and stiff accuracy, textbook s = 1, 2, 3
values, and the stability function matching exp(z) to order 2s-1
(tests/test_oracle_tableau.py).
"""
import numpy as np
from numpy.polynomial import polynomial as npoly


def radau_iia(s):
    """Return (A, b, c) of the s-stage Radau IIA method.

    c are the zeros of d^{s-1}/dx^{s-1} [x^{s-1} (x-1)^s] (so c_s = 1);
    A solves the collocation conditions sum_j a_ij c_j^{q-1} = c_i^q / q for
    q = 1..s; b is the last row of A (stiffly accurate).
    """
    if s < 1:
        raise ValueError("s must be >= 1")
    p = np.array([1.0])
    for _ in range(s - 1):
        p = npoly.polymul(p, [0.0, 1.0])
    for _ in range(s):
        p = npoly.polymul(p, [-1.0, 1.0])
    d = npoly.polyder(p, s - 1)
    c = np.sort(np.real(npoly.polyroots(d)))
    # polish the roots with Newton steps on the derivative polynomial
    dd = npoly.polyder(d)
    for _ in range(3):
        c = c - npoly.polyval(c, d) / np.where(npoly.polyval(c, dd) == 0, 1.0,
                                                npoly.polyval(c, dd))
    c[-1] = 1.0
    vand = np.array([[cj ** q for q in range(s)] for cj in c])   # [j, q]
    rhs = np.array([[ci ** (q + 1) / (q + 1) for q in range(s)] for ci in c])
    A = np.linalg.solve(vand.T, rhs.T).T                          # A @ vand = rhs
    b = A[-1].copy()
    return A, b, c


def crout(A):
    """Crout factorisation A = L U with L lower triangular, U unit upper.

    Rana's preconditioner (cited in Sec. 3, Sec. 5) replaces A_RK in the stage
    matrix by its lower factor L, giving a block-lower-triangular stage
    preconditioner I_s (x) M + tau L (x) K whose diagonal blocks have the form
    M + a K with a = tau L_ii.
    """
    s = A.shape[0]
    L = np.zeros((s, s))
    U = np.eye(s)
    for j in range(s):
        for i in range(j, s):
            L[i, j] = A[i, j] - sum(L[i, k] * U[k, j] for k in range(j))
        for i in range(j + 1, s):
            U[j, i] = (A[j, i] - sum(L[j, k] * U[k, i] for k in range(j))) / L[j, j]
    return L, U


def stability_function(A, b, z):
    """R(z) = 1 + z b^T (I - z A)^{-1} e for the tableau (A, b)."""
    s = A.shape[0]
    return 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))
