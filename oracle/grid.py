"""Finite-difference stiffness matrix K on the unit square / cube.

Test infrastructure only (see ``oracle/__init__.py``).

Paper: Sec. 2 writes the stage system with a mass matrix M and a stiffness
matrix K from finite elements.  Here space is discretised by the 5-point (2D)
or 7-point (3D) finite-difference Laplacian with homogeneous Dirichlet data,
so M = I and K = -Laplacian_h (symmetric positive definite).

Grid: n interior nodes per axis, spacing h = 1/(n+1), node (i, j[, k]) at
((i+1)h, (j+1)h[, (k+1)h]) for 0-based indices; a field is stored with x
fastest, flat index i + n*j (+ n*n*k).  As a NumPy array the shape is
(n, n) or (n, n, n) in C order with the x axis last.

Variable diffusivity kappa is given at the N interior nodes.  A face between
two interior nodes carries the harmonic mean 2 k_p k_q / (k_p + k_q); a face
between an interior node p and a boundary node carries k_p.

Pinned by: the closed-form DST eigenpairs of the constant-coefficient K,
symmetry, and the flux (divergence) form checked against a hand sum on tiny
grids (tests/test_oracle_grid.py).
"""
import numpy as np
import scipy.sparse as sp


def spacing(n):
    return 1.0 / (n + 1)


def field_shape(n, dim):
    return (n,) * dim


def node_coordinates(n, dim):
    """Coordinates of the interior nodes, each array of shape field_shape."""
    h = spacing(n)
    x1 = (np.arange(n) + 1.0) * h
    grids = np.meshgrid(*([x1] * dim), indexing="ij")
    # numpy axis 0 is the slowest (y in 2D, z in 3D); return (x, y[, z])
    return tuple(grids[::-1])


def stiffness(n, dim, kappa=None):
    """Sparse CSR matrix of K = -div(kappa grad) (5/7-point FD, Dirichlet)."""
    h = spacing(n)
    N = n ** dim
    shape = field_shape(n, dim)
    idx = np.arange(N).reshape(shape)
    kap = np.ones(shape) if kappa is None else np.asarray(kappa, float).reshape(shape)
    diag = np.zeros(N)
    rows, cols, vals = [], [], []
    for ax in range(dim):
        lo = np.take(idx, np.arange(0, n - 1), axis=ax).ravel()
        hi = np.take(idx, np.arange(1, n), axis=ax).ravel()
        klo = np.take(kap, np.arange(0, n - 1), axis=ax).ravel()
        khi = np.take(kap, np.arange(1, n), axis=ax).ravel()
        kf = 2.0 * klo * khi / (klo + khi)
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-kf, -kf]
        np.add.at(diag, lo, kf)
        np.add.at(diag, hi, kf)
        for end in (0, n - 1):
            pb = np.take(idx, [end], axis=ax).ravel()
            kb = np.take(kap, [end], axis=ax).ravel()
            np.add.at(diag, pb, kb)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return K / (h * h)


def dst_eigenvalues(n, dim):
    """Eigenvalues of the constant-coefficient K, as an array of field_shape.

    K = sum over axes of the 1D matrix tridiag(-1, 2, -1)/h^2, whose
    eigenvalues are (4/h^2) sin^2(k pi h / 2), k = 1..n, with eigenvectors
    sin(k pi x) sampled at the nodes (orthonormal DST-I basis).
    """
    h = spacing(n)
    lam1 = 4.0 / (h * h) * np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    grids = np.meshgrid(*([lam1] * dim), indexing="ij")
    return sum(grids)
