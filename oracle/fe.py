"""Q1 and Q2 finite elements on a square and the Chebyshev mass solve
(Sec. 2, Sec. 5).

Test infrastructure only (see ``oracle/__init__.py``).

The paper discretises space by Q1 and Q2 finite elements, which brings a
mass matrix M into eq. (2.4): M v_{n+1} = M v_n + tau sum_i b_i M V_{n,i}
and (I_s (x) M + tau A (x) K) V_n = f_n - (e (x) K) v_n.  Here: bilinear (Q1)
or biquadratic (Q2) elements on a uniform mesh of the square [0, L]^2 (the
paper's [-1, 1]^2 is L = 2), n interior nodes per axis, node spacing
h = L / (n + 1), homogeneous Dirichlet data (boundary nodes eliminated).
Nodes are ordered x fastest, as for the finite-difference grid.  A Q1
element spans one node spacing; a Q2 element spans two (its vertices, edge
midpoints and centre are nodes), so n is odd for Q2 and the element side is
2h.  The paper's mesh parameter for Table 1 is the element side 2^(1-l) for
both (a reading, fixed by the DoF counts of that table).

M and K are assembled element by element from the local matrices of the
shape functions (4 bilinear or 9 biquadratic), computed by Gauss quadrature
on the reference square (2 x 2 or 3 x 3 points: exact for these integrands).

The paper applies M^{-1} inside S-tilde by 20 steps of Chebyshev
semi-iteration with the Jacobi splitting of M (Golub and Varga; Wathen and
Rees give the spectrum of D^{-1} M on squares: [1/4, 9/4] for Q1 and
[1/4, 25/16] for Q2).  ``chebyshev_mass`` is that iteration written from the
definition: the basic iteration y <- y + D^{-1} (t - M y) / theta (theta the
centre of the interval) accelerated by the three-term Chebyshev recurrence,
so the error after k steps is T_k(G / rho) / T_k(1 / rho) applied to the
initial error, G = I - D^{-1} M / theta, rho = (beta - alpha) / (beta + alpha).

Pinned by (tests/test_oracle_fe.py): the assembly against the tensor form
M = M1 (x) M1, K = T (x) M1 + M1 (x) T of the 1D matrices (Q1: the textbook
tridiagonal ones; Q2: the textbook quadratic element matrices); the
closed-form eigenpairs (Q1 sine modes); the Jacobi bounds against the
element eigenvalues; the Q2 eigenvalue convergence order; the Chebyshev
error on eigenvectors against the Chebyshev polynomial value; the
all-at-once solve with M against stepping; the Q1 and Q2 DoF counts of
Table 1.
"""
import numpy as np
import scipy.sparse as sp

# spectrum of D^{-1} M on squares (Jacobi-preconditioned mass matrix)
Q1_JACOBI_BOUNDS = (0.25, 2.25)
Q2_JACOBI_BOUNDS = (0.25, 1.5625)
CHEBYSHEV_STEPS = 20
DISCS = ("q1", "q2")


def jacobi_bounds(disc):
    return Q1_JACOBI_BOUNDS if disc == "q1" else Q2_JACOBI_BOUNDS


def spacing(n, length):
    return length / (n + 1)


def element_matrices(h):
    """Local 4 x 4 mass and stiffness matrices of one bilinear element of
    side h.  Local node a at corner (xa, ya) in {0, 1}^2, a = xa + 2 ya;
    shape function phi_a = l_xa(x) l_ya(y) with l_0 = 1 - s, l_1 = s on the
    reference interval; 2 x 2 Gauss points."""
    g = 0.5 + np.array([-1.0, 1.0]) / (2.0 * np.sqrt(3.0))
    w = np.array([0.5, 0.5])
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]

    def l(c, s):
        return s if c == 1 else 1.0 - s

    def dl(c):
        return 1.0 if c == 1 else -1.0

    Me = np.zeros((4, 4))
    Ke = np.zeros((4, 4))
    for qx, wx in zip(g, w):
        for qy, wy in zip(g, w):
            phi = np.array([l(cx, qx) * l(cy, qy) for cx, cy in corners])
            # gradients in physical coordinates (d/dx = (1/h) d/ds)
            gx = np.array([dl(cx) * l(cy, qy) for cx, cy in corners]) / h
            gy = np.array([l(cx, qx) * dl(cy) for cx, cy in corners]) / h
            wt = wx * wy * h * h
            Me += wt * np.outer(phi, phi)
            Ke += wt * (np.outer(gx, gx) + np.outer(gy, gy))
    return Me, Ke


def q1_matrices(n, length):
    """Sparse CSR (M, K) on the n x n interior nodes of [0, length]^2."""
    h = spacing(n, length)
    Me, Ke = element_matrices(h)
    N = n * n
    rows, cols, mv, kv = [], [], [], []
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]
    # elements (ex, ey), 0..n: lower-left corner at grid node (ex, ey) of the
    # (n + 2)^2 grid including the boundary; interior node (i, j) is grid
    # node (i + 1, j + 1)
    for ey in range(n + 1):
        for ex in range(n + 1):
            glob = []
            for cx, cy in corners:
                gi, gj = ex + cx - 1, ey + cy - 1
                glob.append(gi + n * gj if 0 <= gi < n and 0 <= gj < n else -1)
            for a in range(4):
                if glob[a] < 0:
                    continue
                for b in range(4):
                    if glob[b] < 0:
                        continue
                    rows.append(glob[a])
                    cols.append(glob[b])
                    mv.append(Me[a, b])
                    kv.append(Ke[a, b])
    M = sp.csr_matrix((mv, (rows, cols)), shape=(N, N))
    K = sp.csr_matrix((kv, (rows, cols)), shape=(N, N))
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


def q2_element_matrices(H):
    """Local 9 x 9 mass and stiffness matrices of one biquadratic element of
    side H.  Local node a at (xa, ya) in {0, 1, 2}^2 (positions 0, H/2, H),
    a = xa + 3 ya; phi_a = l_xa(x) l_ya(y) with the quadratic Lagrange
    polynomials of the reference points 0, 1/2, 1; 3 x 3 Gauss points."""
    g = 0.5 + np.array([-1.0, 0.0, 1.0]) * np.sqrt(0.6) / 2.0
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    pts = (0.0, 0.5, 1.0)

    def l(c, s):
        out = 1.0
        for q in range(3):
            if q != c:
                out *= (s - pts[q]) / (pts[c] - pts[q])
        return out

    def dl(c, s):
        tot = 0.0
        for skip in range(3):
            if skip == c:
                continue
            term = 1.0 / (pts[c] - pts[skip])
            for q in range(3):
                if q != c and q != skip:
                    term *= (s - pts[q]) / (pts[c] - pts[q])
            tot += term
        return tot

    nodes = [(cx, cy) for cy in range(3) for cx in range(3)]
    Me = np.zeros((9, 9))
    Ke = np.zeros((9, 9))
    for qx, wx in zip(g, w):
        for qy, wy in zip(g, w):
            phi = np.array([l(cx, qx) * l(cy, qy) for cx, cy in nodes])
            gx = np.array([dl(cx, qx) * l(cy, qy) for cx, cy in nodes]) / H
            gy = np.array([l(cx, qx) * dl(cy, qy) for cx, cy in nodes]) / H
            wt = wx * wy * H * H
            Me += wt * np.outer(phi, phi)
            Ke += wt * (np.outer(gx, gx) + np.outer(gy, gy))
    return Me, Ke


def q2_matrices(n, length):
    """Sparse CSR (M, K) of biquadratic elements on the n x n interior nodes
    of [0, length]^2; n odd, (n + 1) / 2 elements per axis of side 2h."""
    if n % 2 != 1:
        raise ValueError("Q2 elements need an odd number of interior nodes per axis")
    ne = (n + 1) // 2
    H = 2.0 * spacing(n, length)
    Me, Ke = q2_element_matrices(H)
    N = n * n
    rows, cols, mv, kv = [], [], [], []
    nodes = [(cx, cy) for cy in range(3) for cx in range(3)]
    # element (ex, ey) covers grid nodes 2 ex .. 2 ex + 2 (boundary nodes at
    # grid index 0 and n + 1); interior node i is grid node i + 1
    for ey in range(ne):
        for ex in range(ne):
            glob = []
            for cx, cy in nodes:
                gi, gj = 2 * ex + cx - 1, 2 * ey + cy - 1
                glob.append(gi + n * gj if 0 <= gi < n and 0 <= gj < n else -1)
            for a in range(9):
                if glob[a] < 0:
                    continue
                for b in range(9):
                    if glob[b] < 0:
                        continue
                    rows.append(glob[a])
                    cols.append(glob[b])
                    mv.append(Me[a, b])
                    kv.append(Ke[a, b])
    M = sp.csr_matrix((mv, (rows, cols)), shape=(N, N))
    K = sp.csr_matrix((kv, (rows, cols)), shape=(N, N))
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


def matrices(disc, n, length):
    return q1_matrices(n, length) if disc == "q1" else q2_matrices(n, length)


def element_side(disc, n, length):
    return spacing(n, length) * (1.0 if disc == "q1" else 2.0)


def node_coordinates(n, length):
    """(x, y) of the interior nodes, arrays of shape (n, n) (x along axis 1)."""
    h = spacing(n, length)
    x1 = (np.arange(n) + 1.0) * h
    Y, X = np.meshgrid(x1, x1, indexing="ij")
    return X, Y


def _lagrange(pts, c, s):
    out = 1.0
    for q in range(len(pts)):
        if q != c:
            out = out * (s - pts[q]) / (pts[c] - pts[q])
    return out


def load_vector(disc, n, length, f, points=5):
    """Load vector (integrals of f against each interior shape function) by
    Gauss quadrature with ``points`` x ``points`` nodes per element; f(x, y)
    takes arrays."""
    order = 1 if disc == "q1" else 2
    ne = (n + 1) // order
    H = element_side(disc, n, length)
    pts = np.linspace(0.0, 1.0, order + 1)
    gx, gw = np.polynomial.legendre.leggauss(points)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
    out = np.zeros(n * n)
    for ey in range(ne):
        for ex in range(ne):
            X = (ex + gx[None, :]) * H
            Y = (ey + gx[:, None]) * H
            fv = f(X, Y) * (gw[:, None] * gw[None, :]) * H * H
            for cy in range(order + 1):
                for cx in range(order + 1):
                    gi, gj = order * ex + cx - 1, order * ey + cy - 1
                    if not (0 <= gi < n and 0 <= gj < n):
                        continue
                    phi = _lagrange(pts, cy, gx)[:, None] * _lagrange(pts, cx, gx)[None, :]
                    out[gi + n * gj] += np.sum(fv * phi)
    return out


def chebyshev_mass(M, t, steps=CHEBYSHEV_STEPS, bounds=Q1_JACOBI_BOUNDS):
    """Approximate M^{-1} t by ``steps`` steps of Chebyshev semi-iteration with
    the Jacobi splitting, from zero.  t may hold several right-hand sides
    as rows (shape (m, N)) or be one vector.

    y_0 = 0, y_1 = D^{-1} t / theta, and for k >= 1
    y_{k+1} = w_{k+1} (y_k - y_{k-1} + D^{-1} (t - M y_k) / theta) + y_{k-1},
    w_2 = 1 / (1 - rho^2 / 2), w_{k+1} = 1 / (1 - rho^2 w_k / 4)."""
    alpha, beta = bounds
    theta = 0.5 * (alpha + beta)
    rho = (beta - alpha) / (beta + alpha)
    dinv = 1.0 / M.diagonal()
    t = np.asarray(t, float)
    Mt = (lambda Y: (M @ Y.T).T) if t.ndim == 2 else (lambda y: M @ y)
    y_prev = np.zeros_like(t)
    y = dinv * t / theta
    w = 1.0
    for k in range(1, steps):
        w = 1.0 / (1.0 - rho * rho / 2.0) if k == 1 else 1.0 / (1.0 - rho * rho * w / 4.0)
        y_next = w * (y - y_prev + dinv * (t - Mt(y)) / theta) + y_prev
        y_prev, y = y, y_next
    return y


def chebyshev_error_factor(g, rho, k):
    """T_k(g / rho) / T_k(1 / rho): the factor by which k steps of the
    semi-iteration scale the error on an eigenvector whose Jacobi iteration
    eigenvalue is g (|g| <= rho)."""
    return np.cos(k * np.arccos(g / rho)) / np.cosh(k * np.arccosh(1.0 / rho))


def load_sine(n, length, k):
    """Exact load vector of f(x, y) = sin(k x) sin(k y) on the Q1 space
    (integrals against each interior hat function): per axis, the hat
    function of node x_j integrates sin(k x) to
    sin(k x_j) 2 (1 - cos(k h)) / (k^2 h)."""
    h = spacing(n, length)
    x1 = (np.arange(n) + 1.0) * h
    g = np.sin(k * x1) * 2.0 * (1.0 - np.cos(k * h)) / (k * k * h)
    return np.outer(g, g).ravel()
