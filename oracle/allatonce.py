"""The all-at-once system of eq. (2.4): layout, operator, right-hand side.

Test infrastructure only (see ``oracle/__init__.py``).

Paper, Sec. 2: with v = [v_0, ..., v_nt] (each N values) and
V = [V_0, ..., V_{nt-1}], V_n = [V_{n,1}, ..., V_{n,s}], the system is

    [ Phi   Psi1 ] [v]   [b]
    [ Psi2  Theta] [V] = [f]

    Phi   : block lower bidiagonal, M on the diagonal, -M below it
    Psi1  : -(tau b^T (x) M) in block (n+1, n), zero first block row
    Psi2  : (e (x) K) in block (n, n), zero last block column
    Theta : I_nt (x) (I_s (x) M + tau A (x) K)

with M = I for finite differences (disc "fd", the unit square or cube) and
the mass matrix of bilinear (disc "q1") or biquadratic (disc "q2") finite
elements on the square [0, length]^2 (``oracle.fe``).  b holds the initial condition: b_0 = M u0 and
b_{n>=1} = 0 for homogeneous Dirichlet data.  The stage right-hand side is
M f_{n,i} with f_{n,i} = f(x, t_n + c_i tau) at the nodes, t_n = n tau (for
finite elements, the load vector of the nodal interpolant of f; a reading:
the paper calls f_n the discretisation of the right-hand side).

The vector of unknowns is x = [v; V]: (nt+1) blocks of v, then nt*s blocks of
V in (step, stage) order; U = N (nt (s+1) + 1) values in total.

Pinned by: the layout formula against the DoF counts of Table 1; the dense
operator against sequential stepping (eq. (2.2)-(2.3)) and against the block
apply (tests/test_oracle_allatonce.py).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import fe, grid, tableau


@dataclass
class Problem:
    n: int                 # interior nodes per axis
    dim: int               # 2 or 3
    s: int                 # Radau IIA stages
    nt: int                # time steps
    T: float = 1.0         # final time
    kappa: Optional[np.ndarray] = None   # nodal diffusivity (N,), None = 1
    disc: str = "fd"       # "fd" (finite differences), "q1" / "q2" (bilinear / biquadratic elements, 2D)
    length: float = 1.0    # side of the square (q1, q2)

    A: np.ndarray = field(init=False, repr=False)
    b: np.ndarray = field(init=False, repr=False)
    c: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.A, self.b, self.c = tableau.radau_iia(self.s)
        if self.disc not in ("fd",) + fe.DISCS:
            raise ValueError(self.disc)
        if self.fe and (self.dim != 2 or self.kappa is not None):
            raise ValueError("finite elements: 2D, constant diffusivity")
        if self.disc == "q2" and self.n % 2 != 1:
            raise ValueError("q2 elements: odd n")
        self._mk = None

    @property
    def fe(self):
        return self.disc in fe.DISCS

    @property
    def N(self):
        return self.n ** self.dim

    @property
    def tau(self):
        return self.T / self.nt

    @property
    def h(self):
        return fe.spacing(self.n, self.length) if self.fe else grid.spacing(self.n)

    @property
    def U(self):
        return self.N * (self.nt * (self.s + 1) + 1)

    @property
    def UV(self):
        return self.N * self.nt * self.s

    def stage_times(self):
        """(nt, s) array of t_n + c_i tau."""
        return (np.arange(self.nt)[:, None] + self.c[None, :]) * self.tau

    def K(self):
        if self.fe:
            return self._fe()[1]
        return grid.stiffness(self.n, self.dim, self.kappa)

    def M(self):
        """Mass matrix: the identity for finite differences."""
        if self.fe:
            return self._fe()[0]
        return sp.identity(self.N, format="csr")

    def _fe(self):
        if self._mk is None:
            self._mk = fe.matrices(self.disc, self.n, self.length)
        return self._mk


def unknowns(N, nt, s):
    """Number of unknowns of eq. (2.4): (nt+1) v-blocks plus nt*s stage blocks."""
    return N * (nt * (s + 1) + 1)


def split(prob, x):
    """View x as v of shape (nt+1, N) and V of shape (nt, s, N)."""
    N, nt, s = prob.N, prob.nt, prob.s
    v = x[: (nt + 1) * N].reshape(nt + 1, N)
    V = x[(nt + 1) * N:].reshape(nt, s, N)
    return v, V


def join(v, V):
    return np.concatenate([np.asarray(v).ravel(), np.asarray(V).ravel()])


def rhs(prob, f, u0):
    """Right-hand side [b; f]: b_0 = M u0, b_{n>=1} = 0, the stage blocks M f
    in (nt, s, N) order (M = I for finite differences)."""
    v = np.zeros((prob.nt + 1, prob.N))
    fs = np.asarray(f, float).reshape(prob.nt, prob.s, prob.N)
    if prob.fe:
        M = prob.M()
        v[0] = M @ u0
        return join(v, (M @ fs.reshape(-1, prob.N).T).T.reshape(fs.shape))
    v[0] = u0
    return join(v, fs)


def blocks(prob, sparse=True):
    """The four blocks (Phi, Psi1, Psi2, Theta) of eq. (2.4) as Kronecker products."""
    kr = sp.kron if sparse else np.kron
    eye = (lambda m: sp.identity(m, format="csr")) if sparse else np.eye
    N, nt, s, tau = prob.N, prob.nt, prob.s, prob.tau
    K = prob.K() if sparse else prob.K().toarray()
    MN = prob.M() if sparse else prob.M().toarray()
    sub = np.eye(nt + 1, k=-1)                    # ones at (n+1, n)
    Phi = kr(np.eye(nt + 1) - sub, MN)
    Esub = np.zeros((nt + 1, nt))
    Esub[np.arange(1, nt + 1), np.arange(nt)] = 1.0
    Psi1 = -kr(Esub, kr(tau * prob.b[None, :], MN))
    Ediag = np.zeros((nt, nt + 1))
    Ediag[np.arange(nt), np.arange(nt)] = 1.0
    Psi2 = kr(Ediag, kr(np.ones((s, 1)), K))
    Theta_hat = kr(np.eye(s), MN) + tau * kr(prob.A, K)
    Theta = kr(np.eye(nt), Theta_hat)
    return Phi, Psi1, Psi2, Theta


def operator(prob, sparse=True):
    """The all-at-once matrix of eq. (2.4), dense (tiny problems) or sparse."""
    Phi, Psi1, Psi2, Theta = blocks(prob, sparse)
    if sparse:
        return sp.bmat([[Phi, Psi1], [Psi2, Theta]], format="csr")
    return np.block([[Phi, Psi1], [Psi2, Theta]])


def theta_hat(prob, K=None):
    """The stage matrix I_s (x) M + tau A (x) K of eq. (2.3), sparse."""
    K = prob.K() if K is None else K
    return (sp.kron(sp.identity(prob.s), prob.M())
            + prob.tau * sp.kron(prob.A, K)).tocsc()


def apply_rows(prob, x, rows, K=None):
    """Selected entries of y = A x, each computed from its own row of eq. (2.4).

    For full-size problems where A x cannot be formed on the host: row r of
    the v part (block n, node p) or of a stage block (n, i, node p) uses only
    the K-row of p.  ``rows`` are global indices into the layout of x.
    """
    if prob.disc != "fd":
        raise ValueError("apply_rows: finite differences only")
    K = prob.K() if K is None else K
    N, nt, s, tau = prob.N, prob.nt, prob.s, prob.tau
    x = np.asarray(x)
    out = np.empty(len(rows))
    nv = (nt + 1) * N

    def krow(base, p):
        lo, hi = K.indptr[p], K.indptr[p + 1]
        return float(K.data[lo:hi] @ x[base + K.indices[lo:hi]])

    for t, r in enumerate(rows):
        r = int(r)
        if r < nv:
            n, p = divmod(r, N)
            if n == 0:
                out[t] = x[p]
            else:
                Vb = nv + (n - 1) * s * N
                out[t] = x[r] - x[r - N] - tau * sum(prob.b[j] * x[Vb + j * N + p] for j in range(s))
        else:
            q, p = divmod(r - nv, N)
            n, i = divmod(q, s)
            Vb = nv + n * s * N
            kw = krow(n * N, p) + tau * sum(prob.A[i, j] * krow(Vb + j * N, p) for j in range(s))
            out[t] = x[r] + kw
    return out


def apply_blockwise(prob, x, K=None, transpose=False):
    """y = A x (or A^T x) one block row at a time, never forming A.

    Forward rows:  y_{v,0} = M v_0;
                   y_{v,n+1} = M (v_{n+1} - v_n - tau sum_i b_i V_{n,i});
                   y_{V,n,i} = M V_{n,i} + K (v_n + tau sum_j a_ij V_{n,j}).
    Transposed rows follow from the transposed blocks (M, K symmetric):
                   y_{v,n} = M (x_{v,n} - x_{v,n+1}) + K sum_i x_{V,n,i}  (n < nt),
                   y_{v,nt} = M x_{v,nt};
                   y_{V,n,j} = M x_{V,n,j} + tau K sum_i a_ij x_{V,n,i}
                               - tau b_j M x_{v,n+1}.
    """
    K = prob.K() if K is None else K
    Mm = prob.M()
    tau, A, b = prob.tau, prob.A, prob.b
    v, V = split(prob, np.asarray(x, float))
    yv = np.empty_like(v)
    yV = np.empty_like(V)
    if not transpose:
        yv[0] = Mm @ v[0]
        for n in range(prob.nt):
            yv[n + 1] = Mm @ (v[n + 1] - v[n] - tau * np.tensordot(b, V[n], axes=(0, 0)))
            for i in range(prob.s):
                w = v[n] + tau * np.tensordot(A[i], V[n], axes=(0, 0))
                yV[n, i] = Mm @ V[n, i] + K @ w
    else:
        yv[prob.nt] = Mm @ v[prob.nt]
        for n in range(prob.nt):
            yv[n] = Mm @ (v[n] - v[n + 1]) + K @ V[n].sum(axis=0)
            for j in range(prob.s):
                mix = tau * np.tensordot(A[:, j], V[n], axes=(0, 0))
                yV[n, j] = Mm @ V[n, j] + K @ mix - tau * b[j] * (Mm @ v[n + 1])
    return join(yv, yV)
