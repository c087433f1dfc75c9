"""Python binding of the all-at-once heat solver (argument marshalling only).

Every operation runs in the HIP library (libaao_heat.so); PyTorch supplies
device memory (the workspace and the caller's vectors) and the stream.  There
is no fallback: a missing library or GPU raises.
"""
import ctypes

import numpy as np
import torch

from . import _abi


class AAOError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_abi.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# Solver options of aao_opts (include/aao_heat.h) with the library's defaults
# where the binding does not choose its own.
SOLVER_DEFAULTS = dict(restart=30, maxit=100, tol=1e-8, inner_k=3, cycles=1, nu1=2, nu2=2, omega=0.0,
                       precision="fp64", use_graph=True, mg_tail_max=0, coarse_max=0, inner_tol=0.0,
                       schur="sweep", mgrit_cf=8, mgrit_iters=1, mgrit_fcf=False, side="right",
                       outer_precision="fp64", mg_low_from=0, mg_coarse_fp32=False, relax_matvec=False,
                       mgrit_coarse_k=0, schur_k=0, inner_orth="cgs2", outer_orth="cgs2")


def _solver_options(kw):
    unknown = sorted(set(kw) - set(SOLVER_DEFAULTS))
    if unknown:
        raise TypeError(f"unknown solver option(s): {', '.join(unknown)}")
    return dict(SOLVER_DEFAULTS, **kw)


def _make_opts(lib, o):
    opts = _abi.Opts()
    lib.aao_default_opts(ctypes.byref(opts))
    opts.restart, opts.maxit, opts.tol = o["restart"], o["maxit"], o["tol"]
    opts.inner_k, opts.cycles, opts.nu1, opts.nu2 = o["inner_k"], o["cycles"], o["nu1"], o["nu2"]
    opts.omega = o["omega"]
    opts.precision = _abi.PRECISIONS[o["precision"]]
    opts.use_graph = int(bool(o["use_graph"]))
    opts.mg_tail_max = int(o["mg_tail_max"])
    opts.coarse_max = int(o["coarse_max"])
    opts.inner_tol = float(o["inner_tol"])
    opts.schur = _abi.SCHUR[o["schur"]]
    opts.mgrit_cf = int(o["mgrit_cf"])
    opts.mgrit_iters = int(o["mgrit_iters"])
    opts.mgrit_fcf = int(bool(o["mgrit_fcf"]))
    opts.side = _abi.SIDES[o["side"]]
    opts.outer_precision = _abi.OUTER[o["outer_precision"]]
    opts.mg_low_from = int(o["mg_low_from"])
    opts.mg_coarse_fp32 = int(bool(o["mg_coarse_fp32"]))
    opts.relax_matvec = int(bool(o["relax_matvec"]))
    opts.mgrit_coarse_k = int(o["mgrit_coarse_k"])
    opts.schur_k = int(o["schur_k"])
    opts.inner_orth = _abi.ORTH[o["inner_orth"]]
    opts.outer_orth = _abi.ORTH[o["outer_orth"]]
    return opts


def _stats_dict(st, code):
    return {"outer_iterations": st.outer_iterations, "restarts": st.restarts, "relres": st.relres,
            "time_ms": st.time_ms, "precond_ms": st.precond_ms, "theta_ms": st.theta_ms,
            "schur_ms": st.schur_ms, "inner_solves": st.inner_solves,
            "inner_iterations": st.inner_iterations, "relaxed_fp32": st.relaxed_fp32,
            "relaxed_bf16": st.relaxed_bf16,
            "history": list(st.history[: st.history_len]), "converged": code == 0}


class HeatProblem:
    """All-at-once Radau IIA system for the heat equation on one GPU.

    Parameters follow the paper's problem statement (Sec. 2): ``dim``-D unit
    domain with ``n`` interior nodes per axis, ``s``-stage Radau IIA, ``nt``
    steps to final time ``T``; ``kappa`` optional nodal diffusivity (N values,
    2D only).  ``disc`` = "q1" or "q2" selects bilinear or biquadratic
    finite elements with their mass matrix on the square [0, length]^2 (2D,
    kappa = 1; "q2" needs odd ``n``) in place of finite differences.  Solver options: FGMRES ``restart``/``maxit``/``tol``, inner
    GMRES iterations ``inner_k``, V-cycles ``cycles`` with ``nu1``/``nu2``
    Jacobi sweeps, and the preconditioner ``precision``
    ("fp64" | "fp32" | "bf16" | "fp16" | "fp16_all", the last approach A4);
    ``use_graph`` replays the
    preconditioner as a captured HIP graph; ``coarse_max`` is the size of the
    exactly solved coarsest multigrid level (0: 256 nodes); ``inner_tol`` stops
    an inner GMRES solve early at that relative residual (0: always
    ``inner_k`` iterations).  ``schur`` = "sweep" applies S-tilde^{-1} by
    forward substitution in time, "mgrit" by two-level MGRIT with
    coarsening factor ``mgrit_cf``, ``mgrit_iters`` iterations and F- (or,
    with ``mgrit_fcf``, FCF-) relaxation; ``schur_k`` and ``mgrit_coarse_k``
    are the inner GMRES iterations of S-tilde's steps and of MGRIT's coarse
    propagator (0: ``inner_k``); ``inner_orth`` = "cgs2" (two classical
    Gram-Schmidt passes) or "cgs1" (one) in the inner GMRES; ``outer_orth``
    = "cgs2" or "gram" (the second pass from the basis' Gram matrix: one
    sweep over the basis per iteration) in the outer FGMRES.  ``side`` places P-tilde on the
    "right", "left" or both ("split") sides of Algorithm 1;
    ``outer_precision`` = "fp32" runs the outer solve in simulated single
    precision (approach A3).  ``mg_low_from`` (first multigrid level in 16
    bits) and ``mg_coarse_fp32`` (coarse solve kept FP32) set the V-cycle's
    precision schedule for "bf16"/"fp16"; ``relax_matvec`` lowers the
    precision of the products with A as the residual falls.  All solver
    options and their
    defaults are in SOLVER_DEFAULTS.
    """

    def __init__(self, dim, n, s, nt, T=1.0, kappa=None, *, disc="fd", length=1.0, device="cuda", **solver):
        self._lib = _abi.load()
        self.dim, self.n, self.s, self.nt, self.T = dim, n, s, nt, float(T)
        self.disc, self.length = disc, float(length)
        self._kappa = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
        desc = _abi.Desc(dim, n, s, nt, float(T),
                         None if self._kappa is None else self._kappa.ctypes.data, _abi.DISCS[disc],
                         float(length))
        o = _solver_options(solver)
        self.options = dict(o, device=device)
        opts = _make_opts(self._lib, o)
        precision = o["precision"]
        self.precision = precision
        h = ctypes.c_void_p()
        code = self._lib.aao_create_problem(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(h))
        if code != 0:
            raise AAOError(code, self._lib.aao_last_error(None).decode())
        self._h = h
        Nv, Uv = ctypes.c_int64(), ctypes.c_int64()
        self._lib.aao_sizes(h, ctypes.byref(Nv), ctypes.byref(Uv))
        self.N, self.U = Nv.value, Uv.value
        self.device = torch.device(device)
        self._ws = None
        self.tune_state = None
        if self.device.type == "cuda":
            self._attach_workspace()

    # -- lifecycle -----------------------------------------------------------
    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(self._lib.aao_workspace_size(self._h, ctypes.byref(b)))
        return b.value

    def _attach_workspace(self):
        nbytes = self.workspace_bytes()
        self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self._sync_stream()
        self._check(self._lib.aao_set_workspace(self._h, _ptr(self._ws), nbytes))

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.aao_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _check(self, code):
        if code not in (0, 1):
            raise AAOError(code, self._lib.aao_last_error(self._h).decode())
        return code

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._lib.aao_set_stream(self._h, ctypes.c_void_p(s))

    def _vec(self, t, numel, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() == numel):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor with {numel} values")
        return t

    def set_kappa(self, values, log=False):
        """Replace the nodal diffusivity (N float64 CUDA values; theta =
        log kappa with ``log=True``) of a problem created with a kappa array.
        The library rebuilds its diffusivity tables in place."""
        values = self._vec(values.detach().contiguous() if isinstance(values, torch.Tensor) else values,
                           self.N, "kappa")
        self._sync_stream()
        self._check(self._lib.aao_set_kappa(self._h, _ptr(values), int(bool(log))))

    def tableau(self):
        A = np.zeros(self.s * self.s)
        b = np.zeros(self.s)
        c = np.zeros(self.s)
        self._check(self._lib.aao_get_tableau(self._h, A.ctypes.data, b.ctypes.data, c.ctypes.data))
        return A.reshape(self.s, self.s), b, c

    def stage_times(self):
        _, _, c = self.tableau()
        tau = self.T / self.nt
        return (np.arange(self.nt)[:, None] + c[None, :]) * tau

    def empty(self):
        return torch.empty(self.U, dtype=torch.float64, device=self.device)

    # -- operators -----------------------------------------------------------
    def apply_A(self, x, out=None):
        x = self._vec(x, self.U, "x")
        out = self.empty() if out is None else self._vec(out, self.U, "out")
        self._sync_stream()
        self._check(self._lib.aao_apply_A(self._h, _ptr(x), _ptr(out)))
        return out

    def apply_AT(self, x, out=None):
        x = self._vec(x, self.U, "x")
        out = self.empty() if out is None else self._vec(out, self.U, "out")
        self._sync_stream()
        self._check(self._lib.aao_apply_AT(self._h, _ptr(x), _ptr(out)))
        return out

    def apply_P(self, r, out=None, inner_k=None, cycles=None):
        r = self._vec(r, self.U, "r")
        out = self.empty() if out is None else self._vec(out, self.U, "out")
        self._sync_stream()
        if inner_k is None and cycles is None:
            self._check(self._lib.aao_apply_P(self._h, _ptr(r), _ptr(out)))
        else:
            self._check(self._lib.aao_apply_P_with(self._h, _ptr(r), _ptr(out), int(inner_k),
                                                   int(cycles)))
        return out

    def working_dtype(self):
        """Element type of the preconditioner's vectors (apply_mg operands)."""
        return {"fp64": torch.float64, "fp16_all": torch.float16}.get(self.precision, torch.float32)

    def mg_levels(self):
        """(nodes per level, first level solved in one workgroup's LDS)."""
        nodes = np.zeros(64, dtype=np.int64)
        L, t = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.aao_mg_levels(self._h, 64, nodes.ctypes.data, ctypes.byref(L), ctypes.byref(t)))
        return [int(v) for v in nodes[: L.value]], t.value

    def apply_mg(self, r, stage, out=None, cycles=1, transpose=False):
        """`cycles` V-cycles on the blocks of r (count x N) for I + tau L_ii K, i = stage."""
        dt = self.working_dtype()
        if not (isinstance(r, torch.Tensor) and r.is_cuda and r.dtype == dt and r.is_contiguous()
                and r.numel() % self.N == 0 and r.numel() > 0):
            raise ValueError(f"r must be a contiguous {dt} CUDA tensor of count * {self.N} values")
        count = r.numel() // self.N
        if out is None:
            out = torch.empty_like(r)
        elif not (out.is_cuda and out.dtype == dt and out.is_contiguous() and out.numel() == r.numel()):
            raise ValueError("out must match r")
        self._sync_stream()
        self._check(self._lib.aao_apply_mg(self._h, int(bool(transpose)), int(stage), count, int(cycles),
                                           _ptr(r), _ptr(out)))
        return out

    def profile_vcycle(self, count=1, stage=0, reps=10):
        """Mean microseconds of every kernel launch of one V-cycle on `count`
        blocks, in situ and alone (see aao_profile_vcycle):
        ([(label, us_in_situ, us_alone), ...], cycle_us)."""
        cap = 512
        us = np.zeros(cap)
        ua = np.zeros(cap)
        labels = ctypes.create_string_buffer(cap * 48)
        nl, tot = ctypes.c_int(), ctypes.c_double()
        self._sync_stream()
        self._check(self._lib.aao_profile_vcycle(self._h, int(stage), int(count), int(reps), labels, len(labels),
                                                 us.ctypes.data, ua.ctypes.data, cap, ctypes.byref(nl),
                                                 ctypes.byref(tot)))
        names = labels.value.decode().splitlines()
        n = nl.value
        return list(zip(names, us[:n].tolist(), ua[:n].tolist())), tot.value

    def autotune(self, reps=5, cache=None):
        """Choose the multigrid launch shapes by timing (see aao_autotune);
        returns the tuner's report as a dict."""
        t = _abi.Tune()
        self._sync_stream()
        self._check(self._lib.aao_autotune(self._h, int(reps), None if cache is None else str(cache).encode(),
                                           ctypes.byref(t)))
        self.tune_state = {"tall_min_b": t.tall_min_b, "tail_extend": t.tail_extend, "from_cache": t.from_cache,
                           "blocks": list(t.blocks), "weight": list(t.weight), "us": [list(row) for row in t.us]}
        return self.tune_state

    def set_launch_shapes(self, tall_min_b, tail_extend):
        """Apply a launch-shape choice (see aao_set_launch_shapes)."""
        self._check(self._lib.aao_set_launch_shapes(self._h, int(tall_min_b), int(bool(tail_extend))))
        self.tune_state = dict(self.tune_state or {}, tall_min_b=int(tall_min_b), tail_extend=int(bool(tail_extend)))

    def assemble_rhs(self, f, u0, out=None):
        f = self._vec(f, self.N * self.nt * self.s, "f")
        u0 = self._vec(u0, self.N, "u0")
        out = self.empty() if out is None else self._vec(out, self.U, "out")
        self._sync_stream()
        self._check(self._lib.aao_assemble_rhs(self._h, _ptr(f), _ptr(u0), _ptr(out)))
        return out

    def _solve(self, fn, rhs, x0):
        rhs = self._vec(rhs, self.U, "rhs")
        x = torch.zeros_like(rhs) if x0 is None else self._vec(x0, self.U, "x0").clone()
        st = _abi.Stats()
        self._sync_stream()
        code = self._check(fn(self._h, _ptr(rhs), _ptr(x), ctypes.byref(st)))
        return x, _stats_dict(st, code)

    def solve(self, rhs, x0=None):
        """FGMRES solve of A x = rhs; returns (x, stats)."""
        return self._solve(self._lib.aao_solve, rhs, x0)

    def solve_adjoint(self, g, lam0=None):
        """FGMRES solve of A^T lam = g; returns (lam, stats)."""
        return self._solve(self._lib.aao_solve_adjoint, g, lam0)

    def grad_logkappa(self, x, lam, out=None):
        x = self._vec(x, self.U, "x")
        lam = self._vec(lam, self.U, "lam")
        out = (torch.empty(self.N, dtype=torch.float64, device=self.device) if out is None
               else self._vec(out, self.N, "out"))
        self._sync_stream()
        self._check(self._lib.aao_grad_logkappa(self._h, _ptr(x), _ptr(lam), _ptr(out)))
        return out


class HeatBatch:
    """Independent all-at-once problems solved together (same options).

    ``problems`` is a list of dicts with keys dim, n, s, nt and optionally T
    and kappa.  Batch vectors are single float64 CUDA tensors holding the
    problems' vectors back to back; ``split``/``join`` convert to and from
    per-problem views.  ``streams`` HIP streams run the problems concurrently.
    Solver keyword options are those of HeatProblem.
    """

    def __init__(self, problems, *, streams=4, device="cuda", **solver):
        self._lib = _abi.load()
        self.count = len(problems)
        self._kappas = []
        descs = (_abi.Desc * self.count)()
        for i, p in enumerate(problems):
            k = p.get("kappa")
            k = None if k is None else np.ascontiguousarray(k, dtype=np.float64)
            self._kappas.append(k)
            descs[i] = _abi.Desc(p["dim"], p["n"], p["s"], p["nt"], float(p.get("T", 1.0)),
                                 None if k is None else k.ctypes.data, _abi.DISCS[p.get("disc", "fd")],
                                 float(p.get("length", 1.0)))
        self.problems = [dict(p) for p in problems]
        o = _solver_options(solver)
        self.options = dict(o, device=device)
        self.tol = o["tol"]
        opts = _make_opts(self._lib, o)
        h = ctypes.c_void_p()
        code = self._lib.aao_create_batch(descs, self.count, ctypes.byref(opts), int(streams), ctypes.byref(h))
        if code != 0:
            raise AAOError(code, self._lib.aao_batch_last_error(None).decode())
        self._h = h
        ou = np.zeros(self.count + 1, dtype=np.int64)
        on = np.zeros(self.count + 1, dtype=np.int64)
        of = np.zeros(self.count + 1, dtype=np.int64)
        self._lib.aao_batch_offsets(h, ou.ctypes.data, on.ctypes.data, of.ctypes.data)
        self.off_unknowns, self.off_nodes, self.off_forcing = ou, on, of
        self.U, self.N, self.F = int(ou[-1]), int(on[-1]), int(of[-1])
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t()
        self._check(self._lib.aao_batch_workspace_size(h, ctypes.byref(nbytes)))
        self._ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        self._sync_stream()
        self._check(self._lib.aao_batch_set_workspace(h, _ptr(self._ws), nbytes.value))

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.aao_batch_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code not in (0, 1):
            raise AAOError(code, self._lib.aao_batch_last_error(self._h).decode())
        return code

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._lib.aao_batch_set_stream(self._h, ctypes.c_void_p(s))

    def _vec(self, t, numel, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() == numel):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor with {numel} values")
        return t

    def set_kappa(self, i, values, log=False):
        """Replace problem i's nodal diffusivity (N_i float64 CUDA values, or
        log kappa with ``log=True``); see HeatProblem.set_kappa."""
        h = ctypes.c_void_p()
        self._check(self._lib.aao_batch_problem(self._h, int(i), ctypes.byref(h)))
        n = int(self.off_nodes[i + 1] - self.off_nodes[i])
        values = self._vec(values.detach().contiguous(), n, "kappa")
        torch.cuda.current_stream(self.device).synchronize()
        code = self._lib.aao_set_kappa(h, _ptr(values), int(bool(log)))
        if code != 0:
            raise AAOError(code, self._lib.aao_last_error(h).decode())

    def split(self, t, kind="unknowns"):
        """Per-problem views of a batch tensor (kind: unknowns | nodes | forcing)."""
        off = {"unknowns": self.off_unknowns, "nodes": self.off_nodes, "forcing": self.off_forcing}[kind]
        return [t[int(off[i]): int(off[i + 1])] for i in range(self.count)]

    def join(self, parts, kind="unknowns"):
        return torch.cat([p.reshape(-1) for p in parts]).contiguous()

    def assemble_rhs(self, f, u0, out=None):
        f = self._vec(f, self.F, "f")
        u0 = self._vec(u0, self.N, "u0")
        out = torch.empty(self.U, dtype=torch.float64, device=self.device) if out is None else \
            self._vec(out, self.U, "out")
        self._sync_stream()
        self._check(self._lib.aao_batch_assemble_rhs(self._h, _ptr(f), _ptr(u0), _ptr(out)))
        return out

    def _solve(self, fn, rhs, x0):
        rhs = self._vec(rhs, self.U, "rhs")
        x = torch.zeros_like(rhs) if x0 is None else self._vec(x0, self.U, "x0").clone()
        st = (_abi.Stats * self.count)()
        self._sync_stream()
        code = self._check(fn(self._h, _ptr(rhs), _ptr(x), st))
        return x, [_stats_dict(st[i], 0 if st[i].relres <= self.tol else 1) for i in range(self.count)]

    def solve(self, rhs, x0=None):
        """FGMRES solves of every problem; returns (x, [stats per problem])."""
        return self._solve(self._lib.aao_batch_solve, rhs, x0)

    def solve_adjoint(self, g, lam0=None):
        return self._solve(self._lib.aao_batch_solve_adjoint, g, lam0)

    def grad_logkappa(self, x, lam, out=None):
        x = self._vec(x, self.U, "x")
        lam = self._vec(lam, self.U, "lam")
        out = torch.empty(self.N, dtype=torch.float64, device=self.device) if out is None else \
            self._vec(out, self.N, "out")
        self._sync_stream()
        self._check(self._lib.aao_batch_grad_logkappa(self._h, _ptr(x), _ptr(lam), _ptr(out)))
        return out
