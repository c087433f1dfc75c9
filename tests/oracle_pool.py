"""Run oracle computations in a pool of fresh CPU processes.

The GPU tests at the workloads' full sizes need the oracle on many problems
at once (64 LU-stepped problems in the uneven batch, 8 gradient problems).
Workers are spawned processes that import only numpy/scipy and ``oracle``
(never torch or the HIP library), each single-threaded, so the pool uses
the host's cores without touching the GPU.
"""
import concurrent.futures
import multiprocessing
import os

import numpy as np

import heat_inputs


def host_workers(cap=16):
    return max(1, min(cap, len(os.sched_getaffinity(0))))


def _problem(sp, kappa=None):
    from oracle import allatonce
    return allatonce.Problem(sp["n"], 2, sp["s"], sp["nt"], float(sp.get("T", 1.0)), kappa=kappa)


def batch_reference(sp):
    """x* of one problem of the uneven batch recipe (LU stepping)."""
    from oracle import stepping
    times = _problem(sp).stage_times()
    kappa, f, u0 = heat_inputs.spec_inputs(sp, times)
    return stepping.solve(_problem(sp, kappa), f, u0, method="lu")


def gradient_reference(sp):
    """(target v, loss, dL/df, dL/du0, dL/dlog kappa) of one gradient problem."""
    from oracle import adjoint, allatonce, stepping
    times = _problem(sp).stage_times()
    kappa, f, u0 = heat_inputs.spec_inputs(sp, times)
    p = _problem(sp, kappa)
    ft, ut = heat_inputs.spec_target_inputs(sp, times)
    vt = allatonce.split(p, stepping.solve(p, ft, ut, method="lu"))[0]
    L, gf, gu0, gk = adjoint.gradients(p, f, u0, vt)
    return vt, L, gf, gu0, gk


def run(fn, items, workers=None):
    """[fn(item) for item in items], computed by spawned single-threaded workers."""
    workers = workers or host_workers()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = multiprocessing.get_context("spawn")
        with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
            return list(ex.map(fn, items))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
