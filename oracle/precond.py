"""Block preconditioners of Sec. 3 and FGMRES (Algorithm 1).

Test infrastructure only (see ``oracle/__init__.py``).

Ideal preconditioner, eq. (3.1):  P = [[S, Psi1], [0, Theta]] with the Schur
complement S = Phi - Psi1 Theta^{-1} Psi2.  With M = I, S is block lower
bidiagonal with identity diagonal blocks and sub-diagonal blocks -I + X,
X = tau (b^T (x) I) Theta_hat^{-1} (e (x) K).

Practical preconditioner, eqs. (3.2)-(3.3): Theta is replaced by
Theta-tilde -- a fixed number k of GMRES iterations on each step's stage
matrix Theta_hat from a zero guess, right-preconditioned by Rana's
block-lower-triangular stage preconditioner -- and S by S-tilde built with
the same Theta-tilde:  S-tilde = blockdiag(M) [[I], [-I + X~, I], ...],
X~ = tau (b^T (x) I) Theta-tilde^{-1} (e (x) K).

Applying z = P^{-1} r is block back-substitution:
    z_V = Theta^{-1} r_V                          (independent per step)
    t_{v,0} = r_{v,0},  t_{v,n+1} = r_{v,n+1} + tau sum_i b_i z_{V,n,i}
    z_{v,0} = t_{v,0},  z_{v,n+1} = t_{v,n+1} + z_{v,n} - X z_{v,n}
(the M^{-1} step of S-tilde is the identity when M = I; with Q1 elements
t_v carries M in its coupling term, t_{v,n+1} = r_{v,n+1} + tau M sum_i b_i
z_{V,n,i}, and S-tilde^{-1} first applies M^{-1} to every block of t_v by 20
steps of Chebyshev semi-iteration, as the paper does, before the
substitution).

Rana's stage preconditioner (cited, not defined, in the paper; reading): the
Crout factor A_RK = L U (U unit upper) gives P_int = I_s (x) M + tau L (x) K,
solved by forward substitution over the stages with the diagonal blocks
M + tau L_ii K inverted by ``cycles`` multigrid V-cycles (or exactly).

Pinned by: (A P^{-1} - I)^2 = 0 (minimal polynomial of degree two, Sec. 3) on
dense tiny systems; FGMRES with the exact P converging in at most two steps;
the inner GMRES against a brute-force Krylov least-squares minimiser; Rana
with s = 1 being exact (tests/test_oracle_precond.py).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import allatonce, fe, multigrid, tableau


# ----------------------------------------------------------------------------
# GMRES (Algorithm 1 with P_L = I; modified Gram-Schmidt Arnoldi)
# ----------------------------------------------------------------------------
def gmres(apply_op, apply_prec, b, k, tol=0.0):
    """k iterations of right-preconditioned GMRES from x = 0 (no restart).

    Returns (x, iterations).  Stops early on an exact breakdown or when the
    least-squares residual drops to tol * beta.
    """
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0
    Vb = [b / beta]
    Z = []
    H = np.zeros((k + 1, k))
    m = 0
    for j in range(k):
        z = apply_prec(Vb[j])
        Z.append(z)
        w = apply_op(z)
        for i in range(j + 1):
            H[i, j] = Vb[i] @ w
            w = w - H[i, j] * Vb[i]
        H[j + 1, j] = np.linalg.norm(w)
        m = j + 1
        e1 = np.zeros(m + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: m + 1, :m], e1, rcond=None)
        res = np.linalg.norm(e1 - H[: m + 1, :m] @ y)
        if H[j + 1, j] == 0.0 or res <= tol * beta:
            break
        Vb.append(w / H[j + 1, j])
    e1 = np.zeros(m + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(H[: m + 1, :m], e1, rcond=None)
    x = np.zeros_like(b)
    for i in range(m):
        x = x + y[i] * Z[i]
    return x, m


# ----------------------------------------------------------------------------
# Stage-level pieces
# ----------------------------------------------------------------------------
class StageOps:
    """Theta_hat, Rana's preconditioner and the shifted-block solvers of one problem."""

    def __init__(self, prob, inner_k=3, inner_tol=0.0, cycles=1, omega=None,
                 nu1=1, nu2=1, exact_blocks=False, coarse_max=multigrid.COARSE_MAX, schur_k=None):
        self.prob = prob
        # inner GMRES iterations of the Theta-tilde solves inside S-tilde's
        # steps (None: inner_k, the paper's single inner solver)
        self.schur_k = schur_k or inner_k
        self.K = prob.K()
        self.Th = allatonce.theta_hat(prob, self.K)
        self.L, _ = tableau.crout(prob.A)
        self.inner_k = inner_k
        self.inner_tol = inner_tol
        self.cycles = cycles
        self.omega = omega if omega is not None else (0.8 if prob.dim == 2 else 6.0 / 7.0)
        self.nu1, self.nu2 = nu1, nu2
        self.exact_blocks = exact_blocks
        self.coarse_max = coarse_max
        tau = prob.tau
        self.M = prob.M()
        Mh = self.M if prob.fe else None
        ml = 2 if prob.disc == "q2" else 1
        self.hier = [multigrid.Hierarchy(self.K, prob.n, prob.dim, tau * self.L[i, i], coarse_max, M=Mh,
                                         min_levels=ml)
                     for i in range(prob.s)]
        self._lu_blocks = None
        self._lu_theta = None

    def block_solve(self, i, rhs):
        """Inexact (or exact) inverse of M + tau L_ii K."""
        if self.exact_blocks:
            if self._lu_blocks is None:
                self._lu_blocks = [spla.splu(h.ops[0].tocsc()) for h in self.hier]
            return self._lu_blocks[i].solve(rhs)
        return multigrid.solve(self.hier[i], rhs, self.cycles, self.omega, self.nu1, self.nu2)

    def rana(self, r):
        """Forward substitution with I_s (x) M + tau L (x) K; r, z shape (s, N)."""
        s, tau = self.prob.s, self.prob.tau
        z = np.zeros_like(r)
        for i in range(s):
            rhs = r[i].copy()
            for l in range(i):
                rhs -= tau * self.L[i, l] * (self.K @ z[l])
            z[i] = self.block_solve(i, rhs)
        return z

    def theta_apply(self, x):
        return self.Th @ x

    def theta_tilde_inv(self, r, k=None):
        """Theta-tilde^{-1} r for one step: inner GMRES(k) with Rana (k
        defaults to inner_k)."""
        s, N = self.prob.s, self.prob.N
        x, _ = gmres(self.theta_apply,
                     lambda v: self.rana(v.reshape(s, N)).ravel(),
                     np.asarray(r, float).ravel(), k or self.inner_k, self.inner_tol)
        return x.reshape(s, N)

    def theta_inv(self, r):
        """Exact Theta_hat^{-1} r for one step."""
        if self._lu_theta is None:
            self._lu_theta = spla.splu(self.Th)
        return self._lu_theta.solve(np.asarray(r, float).ravel()).reshape(self.prob.s, self.prob.N)


def schur_propagator(ops, exact=False):
    """Phi(z) = z - X-tilde z, X-tilde = tau (b^T (x) I) Theta-tilde^{-1} (e (x) K)
    (eq. (3.3)); with exact=True, Theta_hat^{-1} in place of Theta-tilde^{-1}."""
    prob = ops.prob
    solve_step = ops.theta_inv if exact else (lambda r: ops.theta_tilde_inv(r, ops.schur_k))

    def phi(z):
        y = solve_step(np.tile(ops.K @ z, (prob.s, 1)))
        return z - prob.tau * np.tensordot(prob.b, y, axes=(0, 0))
    return phi


def coarse_stage_ops(ops, cf, coarse_k=None):
    """StageOps of the same problem with the time step cf * tau (the MGRIT
    coarse propagator takes one S-tilde step of that size), with coarse_k
    inner GMRES iterations (None: the fine propagator's)."""
    p = ops.prob
    pc = allatonce.Problem(p.n, p.dim, p.s, 1, cf * p.tau, kappa=p.kappa, disc=p.disc, length=p.length)
    return StageOps(pc, inner_k=coarse_k or ops.inner_k, inner_tol=ops.inner_tol, cycles=ops.cycles, omega=ops.omega,
                    nu1=ops.nu1, nu2=ops.nu2, exact_blocks=ops.exact_blocks, coarse_max=ops.coarse_max)


def apply_preconditioner(ops, r, exact=False, mgrit=None):
    """z = P-tilde^{-1} r (or P^{-1} r when exact=True) by block back-substitution.

    mgrit: None for the forward substitution in S-tilde, or a dict with keys
    cf, iters and optionally relax ("F" / "FCF") and coarse_k (the coarse
    propagator's inner GMRES iterations) to apply S-tilde^{-1} by two-level
    MGRIT (``oracle.mgrit``) with the coarse step cf * tau.
    """
    from . import mgrit as _mgrit
    prob = ops.prob
    nt, s, N, tau = prob.nt, prob.s, prob.N, prob.tau
    rv, rV = allatonce.split(prob, np.asarray(r, float))
    solve_step = ops.theta_inv if exact else ops.theta_tilde_inv
    zV = np.empty((nt, s, N))
    for n in range(nt):
        zV[n] = solve_step(rV[n])
    tv = rv.copy()
    for n in range(nt):
        tv[n + 1] = rv[n + 1] + tau * (ops.M @ np.tensordot(prob.b, zV[n], axes=(0, 0)))
    if prob.fe:
        # S-tilde = blockdiag(M) (bidiagonal part): its block-diagonal mass
        # solve first, by Chebyshev semi-iteration (or exactly)
        if exact:
            lu = spla.splu(ops.M.tocsc())
            tv = np.array([lu.solve(t) for t in tv])
        else:
            tv = fe.chebyshev_mass(ops.M, tv, bounds=fe.jacobi_bounds(prob.disc))
    phi = schur_propagator(ops, exact)
    if mgrit is None:
        zv = np.array(_mgrit.sequential(list(tv), phi))
    else:
        cf = mgrit["cf"]
        phi_c = schur_propagator(coarse_stage_ops(ops, cf, mgrit.get("coarse_k")), exact)
        zv = np.array(_mgrit.solve(list(tv), phi, phi_c, cf, mgrit["iters"], mgrit.get("relax", "F")))
    return allatonce.join(zv, zV)


def dense_ideal_preconditioner(prob):
    """The matrix P of eq. (3.1) for tiny problems (dense)."""
    Phi, Psi1, Psi2, Theta = [np.asarray(B.toarray() if hasattr(B, "toarray") else B)
                              for B in allatonce.blocks(prob, sparse=True)]
    S = Phi - Psi1 @ np.linalg.solve(Theta, Psi2)
    Z = np.zeros((Theta.shape[0], Phi.shape[1]))
    return np.block([[S, Psi1], [Z, Theta]])


# ----------------------------------------------------------------------------
# Outer FGMRES (Algorithm 1, P_L = I, FP64), restarted
# ----------------------------------------------------------------------------
def fgmres(apply_A, apply_P, rhs, restart=30, tol=1e-8, maxit=100, x0=None):
    """Right-preconditioned restarted FGMRES; stops on the true relative residual.

    Returns (x, iterations, history of true relative residuals at exits).
    """
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, float)
    nb = np.linalg.norm(rhs)
    its = 0
    hist = []
    while True:
        r = rhs - apply_A(x)
        rel = np.linalg.norm(r) / nb if nb > 0 else 0.0
        hist.append(rel)
        if rel <= tol or its >= maxit:
            return x, its, hist
        beta = np.linalg.norm(r)
        Vb = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        m = 0
        for j in range(restart):
            its += 1
            z = apply_P(Vb[j])
            Z.append(z)
            w = apply_A(z)
            for i in range(j + 1):
                H[i, j] = Vb[i] @ w
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            m = j + 1
            e1 = np.zeros(m + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: m + 1, :m], e1, rcond=None)
            est = np.linalg.norm(e1 - H[: m + 1, :m] @ y)
            rho = est
            if est <= tol * nb or H[j + 1, j] == 0.0 or its >= maxit:
                break
            Vb.append(w / H[j + 1, j])
        for i in range(m):
            x = x + y[i] * Z[i]


# ----------------------------------------------------------------------------
# Algorithm 1: split-preconditioned FGMRES in four precisions
# ----------------------------------------------------------------------------
def fgmres_split(apply_A, apply_PL, apply_PR, b, restart=30, tol=1e-8, maxit=100, x0=None,
                 rnd=None, rnd_A=None, rnd_PL=None, rnd_PR=None, relax=False, stats=None):
    """Algorithm 1 of Sec. 4, restarted, in FP64 arithmetic with optional
    rounding of each step's result to a lower precision.

    relax: the iteration-dependent matrix-vector tolerance that Sec. 4 names
    (after Simoncini and Szyld) and leaves to future work.  The product
    s = A z_k of iteration k may carry a relative error up to
    eta_k = tol beta_0 / rho_{k-1}, rho_{k-1} the least-squares residual
    after the previous iteration (beta at a cycle's first): it is rounded to
    BF16 when eta_k >= 10 u_bf16, else to FP32 when eta_k >= 10 u_fp32
    (RELAX_TIERS), else kept.  The products that start a cycle stay exact.
    stats (a dict) receives the number of products rounded per tier.

    apply_PL / apply_PR: z = P_L^{-1} v / P_R^{-1} v (None = identity);
    rnd, rnd_A, rnd_PL, rnd_PR: functions rounding the results of the
    working-precision steps, of the products with A and of the two
    preconditioner applications (None = FP64).  Within one cycle:
        t = A x0, t~ = P_L^{-1} t, b~ = P_L^{-1} b, r0 = b~ - t~,
        beta = ||r0||, v1 = r0 / beta;  for k = 1, 2, ...:
        z_k = P_R^{-1} v_k, s = A z_k, w = P_L^{-1} s, modified Gram-Schmidt,
        y_k = argmin ||beta e1 - H_k y||, and the cycle stops once that
        least-squares residual is <= tol times the first cycle's beta; then
        x = x0 + Z_k y_k.  A new cycle starts from x (restart).
    Returns (x, iterations, true relative residuals ||b - A x|| / ||b||
    after each cycle).
    """
    ident = lambda v: v
    PL = apply_PL or ident
    PR = apply_PR or ident
    r_u = rnd or ident
    r_A = rnd_A or ident
    r_L = rnd_PL or ident
    r_R = rnd_PR or ident
    x = np.zeros_like(b) if x0 is None else np.array(x0, float)
    nb = np.linalg.norm(b)
    b_t = r_L(PL(b))
    beta0 = None
    its = 0
    hist = []
    while True:
        t = r_A(apply_A(x))
        t_t = r_L(PL(t)) if np.any(t) else np.zeros_like(t)
        r0 = r_u(b_t - t_t)
        beta = np.linalg.norm(r0)
        beta0 = beta if beta0 is None else beta0
        hist.append(np.linalg.norm(b - apply_A(x)) / nb)
        if beta <= tol * beta0 or its >= maxit or beta == 0.0:
            return x, its, hist
        Vb = [r_u(r0 / beta)]
        Z = []
        H = np.zeros((restart + 1, restart))
        m = 0
        done = False
        rho = beta
        for j in range(restart):
            its += 1
            z = r_R(PR(Vb[j]))
            Z.append(z)
            s_ = r_A(apply_A(z))
            if relax:
                eta = tol * beta0 / rho
                for name, u, rounder in RELAX_TIERS:
                    if eta >= 10.0 * u:
                        s_ = rounder(s_)
                        if stats is not None:
                            stats[name] = stats.get(name, 0) + 1
                        break
            w = r_L(PL(s_))
            for i in range(j + 1):
                H[i, j] = Vb[i] @ w
                w = r_u(w - H[i, j] * Vb[i])
            H[j + 1, j] = np.linalg.norm(w)
            m = j + 1
            e1 = np.zeros(m + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: m + 1, :m], e1, rcond=None)
            est = np.linalg.norm(e1 - H[: m + 1, :m] @ y)
            rho = est
            if est <= tol * beta0 or H[j + 1, j] == 0.0 or its >= maxit:
                done = True
                break
            Vb.append(r_u(w / H[j + 1, j]))
        for i in range(m):
            x = r_u(x + y[i] * Z[i])
        if done:
            hist.append(np.linalg.norm(b - apply_A(x)) / nb)
            return x, its, hist


def round_fp32(v):
    """Round to IEEE single precision (round to nearest even) and back."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(v):
    """Round to FP32, then to bfloat16 (8 significand bits, nearest even on
    the 16 dropped bits), and back."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


# (name, unit roundoff, rounding) from the lowest precision up
RELAX_TIERS = (("bf16", 2.0 ** -8, round_bf16), ("fp32", 2.0 ** -24, round_fp32))

