"""Two-level MGRIT for the S-tilde recurrence (Sec. 3, eq. (3.3); Sec. 5).

Test infrastructure only (see ``oracle/__init__.py``).

Applying S-tilde^{-1} (with M = I) solves the block lower bidiagonal system
of eq. (3.3) by forward substitution in time:

    z_0 = t_0,    z_{n+1} = t_{n+1} + Phi(z_n),    Phi(z) = z - X-tilde z.

The paper's parallel runs replace this substitution by an MGRIT routine
(XBraid), without giving its settings.  Reading (stated in the design doc): the
classical two-level multigrid-reduction-in-time scheme with coarsening factor
c, C-points at the steps kc (k = 0..K-1, K = ceil(nt / c)) and F-points in
between, F- or FCF-relaxation, and a coarse propagator Phi_c that is the
same S-tilde step taken with the step size c tau.

One iteration, with zC[k] the current value at the C-point kc:
  * F-relaxation: from each zC[k], propagate with Phi through the F-points
    of its interval (kc+1 .. min((k+1)c - 1, nt));
  * (FCF only) C-relaxation zC[k] = t_kc + Phi(z_{kc-1}), then F again;
  * g[k] = t_kc + Phi(z_{kc-1}), the fine propagation into C-point kc;
  * coarse solve in time for the C-point corrections
        e_0 = 0,  zC_new[k] = g[k] + Phi_c(e_{k-1}),  e_k = zC_new[k] - zC[k],
    i.e. e_k = Phi_c(e_{k-1}) + (g[k] - zC[k]) with the C-point residual.
After the iterations a last F-relaxation fills every F-point (including nt).
The initial guess is zC[0] = t_0 and zero at the other C-points.

Two facts pin it (tests/test_oracle_mgrit.py): K - 1 iterations reproduce
the forward substitution exactly for any propagators, since every iteration
makes one more C-point exact; and for a linear scalar recurrence the C-point
errors after one iteration follow the closed two-level error recursion
eps'_k = (a^c - a_c) eps_{k-1} + a_c eps'_{k-1}.
"""
import numpy as np


def sequential(t, phi):
    """Forward substitution z_0 = t_0, z_{n+1} = t_{n+1} + phi(z_n)."""
    z = [np.array(t[0], dtype=float)]
    for n in range(len(t) - 1):
        z.append(t[n + 1] + phi(z[n]))
    return z


def solve(t, phi, phi_c, cf, iters, relax="F", zC0=None):
    """Two-level MGRIT approximation of ``sequential(t, phi)``.

    t: sequence of nt + 1 blocks; phi / phi_c: fine / coarse propagators;
    cf >= 2 the coarsening factor; iters >= 0; relax "F" or "FCF";
    zC0: optional initial C-point values (default: t_0, then zeros).
    Returns the list of nt + 1 blocks.
    """
    nt = len(t) - 1
    K = -(-nt // cf)
    z = [None] * (nt + 1)
    zC = [np.array(t[0], dtype=float)] + [np.zeros_like(np.asarray(t[0], dtype=float)) for _ in range(K - 1)]
    if zC0 is not None:
        zC = [np.array(v, dtype=float) for v in zC0]

    def f_relax():
        for k in range(K):
            z[k * cf] = zC[k]
            for j in range(1, cf):
                n = k * cf + j
                if n > nt:
                    break
                z[n] = t[n] + phi(z[n - 1])

    for _ in range(iters):
        f_relax()
        if relax == "FCF":
            for k in range(1, K):
                zC[k] = t[k * cf] + phi(z[k * cf - 1])
            f_relax()
        g = [None] + [t[k * cf] + phi(z[k * cf - 1]) for k in range(1, K)]
        e_prev = None
        for k in range(1, K):
            znew = g[k] + (phi_c(e_prev) if e_prev is not None else 0.0)
            e_prev = znew - zC[k]
            zC[k] = znew
    f_relax()
    if nt % cf == 0 and nt > 0:
        # the last point closes an interval of full length: one more step
        z[nt] = t[nt] + phi(z[nt - 1])
    return z


def scalar_error_recursion(eps, a, a_c, cf):
    """C-point errors after one two-level iteration for z_{n+1} = t + a z_n
    with coarse propagator a_c: eps'_0 = 0 and
    eps'_k = (a^cf - a_c) eps_{k-1} + a_c eps'_{k-1}."""
    out = [0.0] * len(eps)
    for k in range(1, len(eps)):
        out[k] = (a ** cf - a_c) * eps[k - 1] + a_c * out[k - 1]
    return out
