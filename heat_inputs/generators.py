"""Generators behind ``heat_inputs`` (see the package docstring)."""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int
    s: int
    nt: int
    T: float
    restart: int
    seed: int
    data: str          # "mms" or "bumps"

    @property
    def N(self):
        return self.n ** self.dim


WORKLOADS = {
    # 2D 32x32, Radau IIA s=2, 16 steps, manufactured sin-sin-exp solution
    "heat2d_n32_s2_nt16_mms": Workload("heat2d_n32_s2_nt16_mms", 2, 32, 2, 16, 1.0, 30, 0, "mms"),
    # 2D 512x512, s=3, 64 steps (~50M stage unknowns), Gaussian-bump source
    "heat2d_n512_s3_nt64": Workload("heat2d_n512_s3_nt64", 2, 512, 3, 64, 1.0, 30, 1001, "bumps"),
    # 3D 128^3, s=3, 32 steps (~200M stage unknowns)
    "heat3d_n128_s3_nt32": Workload("heat3d_n128_s3_nt32", 3, 128, 3, 32, 1.0, 20, 1002, "bumps"),
}


def nodes(n, dim):
    """Tuple (x, y[, z]) of flat coordinate arrays of the interior nodes."""
    h = 1.0 / (n + 1)
    x1 = (np.arange(n) + 1.0) * h
    g = np.meshgrid(*([x1] * dim), indexing="ij")   # axis 0 slowest
    return tuple(a.ravel() for a in g[::-1])


def sin_product(n, dim):
    """prod_a sin(pi x_a) at the interior nodes."""
    out = np.ones(n ** dim)
    for xa in nodes(n, dim):
        out = out * np.sin(np.pi * xa)
    return out


def mms_source(n, dim, times):
    """f = (d pi^2 - 1) prod sin(pi x_a) e^{-t} for u = prod sin(pi x_a) e^{-t}."""
    phi = sin_product(n, dim)
    t = np.asarray(times, float)
    return (dim * np.pi ** 2 - 1.0) * np.exp(-t)[..., None] * phi


@dataclass(frozen=True)
class PaperCase:
    """A parallel test case of Sec. 5.2 (Table 4): Q2 elements on [-1, 1]^2
    (here [0, 2]^2), n interior nodes per axis, Radau IIA with s stages over
    nt steps up to tf, outer FGMRES restarted every 15 iterations."""
    name: str
    n: int
    s: int
    nt: int
    tf: float
    restart: int = 15
    length: float = 2.0

    @property
    def N(self):
        return self.n * self.n


PAPER_CASES = {
    # test case #1: h = 1.563e-2 (element side), 65025 nodes, 256 steps of 8.236e-2
    "paper_case1_q2_n255_s3_nt256": PaperCase("paper_case1_q2_n255_s3_nt256", 255, 3, 256, 21.084),
    # test case #2: h = 7.813e-3, 261121 nodes, 512 steps of 5.437e-2
    "paper_case2_q2_n511_s3_nt512": PaperCase("paper_case2_q2_n511_s3_nt512", 511, 3, 512, 27.838),
}


def paper_case_inputs(case, times):
    """Nodal source, initial value and exact solution of the test cases'
    manufactured solution v = exp((tf - t) / 10) phi + 1, phi the cosine
    bump of [-1, 1]^2 (on [0, 2]^2: sin(pi x / 2) sin(pi y / 2), at the nodes
    the unit square's sin(pi x) sin(pi y)).  The constant 1 is the boundary
    value; the interior unknowns carry v - 1, whose source is
    f = (pi^2 / 2 - 1/10) exp((tf - t) / 10) phi.  Returns f (times' shape
    plus N), u0 (N,) and exact(t) -> (N,) for v - 1."""
    phi = sin_product(case.n, 2)
    t = np.asarray(times, float)
    f = (np.pi ** 2 / 2.0 - 0.1) * np.exp((case.tf - t) / 10.0)[..., None] * phi
    u0 = np.exp(case.tf / 10.0) * phi
    return f, u0, (lambda tt: np.exp((case.tf - tt) / 10.0) * phi)


def _bump_params(rng, dim, nbumps=8):
    a = rng.standard_normal(nbumps)
    centers = rng.uniform(0.15, 0.85, (nbumps, dim))
    widths = rng.uniform(0.03, 0.12, nbumps)
    om = rng.uniform(0.5, 3.0, nbumps)
    ph = rng.uniform(0.0, 2.0 * np.pi, nbumps)
    return a, centers, widths, om, ph


def bump_source(rng, n, dim, times, nbumps=8):
    """Sum of Gaussian bumps with sinusoidal time modulation; shape times.shape + (N,)."""
    a, centers, widths, om, ph = _bump_params(rng, dim, nbumps)
    X = nodes(n, dim)
    t = np.asarray(times, float)
    G = np.empty((nbumps, n ** dim))
    for k in range(nbumps):
        r2 = sum((X[d] - centers[k, d]) ** 2 for d in range(dim))
        G[k] = np.exp(-r2 / (2.0 * widths[k] ** 2))
    Mt = a[None, :] * np.sin(2.0 * np.pi * om[None, :] * t.reshape(-1, 1) + ph[None, :])
    return (Mt @ G).reshape(t.shape + (n ** dim,))


def smooth_initial(rng, n, dim, modes=8):
    """Smooth field vanishing on the boundary: sine modes <= 8 weighted by 1/|k|^2."""
    c = rng.standard_normal((modes,) * dim)
    h = 1.0 / (n + 1)
    x1 = (np.arange(n) + 1.0) * h
    S = np.sin(np.pi * np.arange(1, modes + 1)[:, None] * x1[None, :])   # (mode, node)
    k = np.arange(1, modes + 1, dtype=float)
    if dim == 2:
        w = c / (k[:, None] ** 2 + k[None, :] ** 2)       # [kx, ky]
        u = np.einsum("ab,ai,bj->ji", w, S, S)            # [y, x]
    else:
        w = c / (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
        u = np.einsum("abc,ai,bj,ck->kji", w, S, S, S)    # [z, y, x]
    return u.ravel()


def lognormal_kappa(rng, n, dim, patches=8, lo=0.1, hi=10.0):
    """Piecewise-constant lognormal diffusivity on patches^d cells, at the nodes."""
    logk = rng.standard_normal((patches,) * dim)
    kp = np.clip(np.exp(logk), lo, hi)
    X = nodes(n, dim)
    cell = [np.minimum((xa * patches).astype(int), patches - 1) for xa in X]
    if dim == 2:
        return kp[cell[0], cell[1]]
    return kp[cell[0], cell[1], cell[2]]


def workload_inputs(w, times):
    """(f of shape (nt, s, N), u0 of shape (N,)) for a Workload.

    ``times`` are the stage times t_n + c_i tau, shape (nt, s), which the
    caller computes from its own Runge--Kutta tableau.
    """
    times = np.asarray(times, float)
    assert times.shape == (w.nt, w.s)
    if w.data == "mms":
        return mms_source(w.n, w.dim, times), sin_product(w.n, w.dim)
    rng = np.random.default_rng(w.seed)
    f = bump_source(rng, w.n, w.dim, times)
    u0 = smooth_initial(rng, w.n, w.dim)
    return f, u0


def batch_problem_specs(count=64, seed=1003):
    """Uneven batch of 2D problems: list of dicts (n, s, nt, rng-seed)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed * 1000 + i)
        n = int(rng.choice([64, 128, 192, 256, 384]))
        nt = int(rng.integers(8, 65))
        s = int(rng.integers(1, 4))
        out.append({"n": n, "s": s, "nt": nt, "T": 1.0, "seed": seed * 1000 + i})
    return out


def gradient_problem_specs(count=8, seed=1004, target_seed=2004):
    """Batch of 2D problems for the gradient check (n=256, s=2, nt=64)."""
    return [{"n": 256, "s": 2, "nt": 64, "T": 1.0, "seed": seed * 1000 + i,
             "target_seed": target_seed * 1000 + i} for i in range(count)]


def spec_inputs(spec, times, dim=2):
    """(kappa, f, u0) of one batch/gradient problem spec, from its seed:
    lognormal patch diffusivity, bump source at the stage ``times`` (shape
    (nt, s)) and smooth initial condition, drawn in that order."""
    rng = np.random.default_rng(spec["seed"])
    kappa = lognormal_kappa(rng, spec["n"], dim).ravel()
    f = bump_source(rng, spec["n"], dim, np.asarray(times, float))
    u0 = smooth_initial(rng, spec["n"], dim)
    return kappa, f, u0


def spec_target_inputs(spec, times, dim=2):
    """(f, u0) generating the tracking target of a gradient problem spec
    (its ``target_seed``; the diffusivity is the problem's own)."""
    rng = np.random.default_rng(spec["target_seed"])
    return bump_source(rng, spec["n"], dim, np.asarray(times, float)), smooth_initial(rng, spec["n"], dim)
