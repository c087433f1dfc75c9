"""Benchmark: all-at-once Radau IIA heat solve on one MI355X.

One step = one full FGMRES solve to a true FP64 relative residual of 1e-8 of
the all-at-once system (paper eq. (2.4)) with the block preconditioner
(eqs. (3.2)-(3.3)) applied in FP32 (the mixed-precision arm, approach A2).
The same solve with the FP64 preconditioner (approach A1) is timed beside
it, with the same inner settings (4 inner GMRES iterations, one V-cycle with
2 + 2 Jacobi sweeps per shifted block).  Workload: 2D heat on a 512 x 512
interior grid, Radau IIA s = 3, 64 time steps to T = 1, FGMRES(30); seeded
Gaussian-bump source and smooth random initial condition (synthetic,
generated on the host).

Prints one JSON line (rank 0).  `roofline` reports apply_A's algorithmic HBM
bytes / its average launch time, and `roofline_vcycle` the same for one
V-cycle on the 64 stage blocks of the batched Theta-tilde phase, both
measured here with HIP events on the stream the kernels run on; `traffic` is
the counter-measured HBM bytes per launch from profiles/ while the kernel
source is unchanged.  `cpu_baseline` times the FP64 CPU oracle (sequential
stepping with an exact DST stage solve) on a bounded number of time steps,
scaled to the full 64 steps.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve time to relres 1e-8, mixed vs FP64 precond; stencil/V-cycle HBM GB/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat2d_n512_s3_nt64")
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--inner-k", type=int, default=4)
    ap.add_argument("--cycles", type=int, default=1)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--tail-max", type=int, default=0,
                    help="largest multigrid level (nodes) solved in one workgroup's LDS (0 = library default)")
    ap.add_argument("--coarse-max", type=int, default=0,
                    help="nodes of the exactly solved coarsest multigrid level (0 = library default)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-preconditioner arm")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=8, help="time steps in the CPU oracle sample")
    ap.add_argument("--roofline-reps", type=int, default=20)
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline launches (apply_A, V-cycle, a 1 GiB device copy); for counter runs")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the all-at-once solve "
                          "is measured at its single-GPU shape (time slabs per GPU would be the "
                          "sharding, with the S-tilde sweep pipelined across slabs)"}))
        sys.exit(2)
    import torch

    import heat_inputs
    from paper_2609_16863_amd import HeatProblem

    w = heat_inputs.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    common = dict(restart=w.restart, tol=1e-8, inner_k=args.inner_k, cycles=args.cycles,
                  nu1=args.nu, nu2=args.nu, mg_tail_max=args.tail_max, coarse_max=args.coarse_max)
    t_setup = time.perf_counter()
    hp_mix = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, precision=args.mixed, **common)
    f, u0 = heat_inputs.workload_inputs(w, hp_mix.stage_times())
    f_d = torch.from_numpy(np.ascontiguousarray(f.ravel())).to(dev)
    u0_d = torch.from_numpy(u0).to(dev)
    rhs = hp_mix.assemble_rhs(f_d, u0_d)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] {w.name}: U = {hp_mix.U:,} unknowns, setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    if args.roofline_only:
        x = torch.randn(hp_mix.U, dtype=torch.float64, device=dev)
        out = {"roofline": measure_roofline(hp_mix, x, args.roofline_reps),
               "roofline_vcycle": measure_vcycle(hp_mix, args.mixed, args.roofline_reps) if w.dim == 2 else None,
               "copy_reference": measure_copy(1 << 30, 5)}
        print(json.dumps(out))
        return

    def run(hp, label, K, W):
        times, stats, x = [], None, None
        for it in range(W + K):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = hp.solve(rhs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if not st["converged"]:
                raise RuntimeError(f"{label} solve did not converge: {st}")
            if it >= W:
                times.append(dt)
            stats = st
            print(f"[bench] {label} solve {it - W if it >= W else 'warmup'}: {dt * 1e3:.1f} ms, "
                  f"{st['outer_iterations']} its, relres {st['relres']:.2e}", file=sys.stderr, flush=True)
        return times, stats, x

    # ---- timed region: K mixed-precision solves -----------------------------
    torch.cuda.synchronize()
    times_mix, st_mix, x_mix = run(hp_mix, args.mixed, args.steps, args.warmup)
    total_s = sum(times_mix)
    ms_per_step = 1e3 * total_s / args.steps

    # ---- FP64-preconditioner arm --------------------------------------------
    fp64 = None
    if not args.no_fp64:
        hp64 = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, precision="fp64", **common)
        times64, st64, x64 = run(hp64, "fp64", args.steps, args.warmup)
        fp64 = {"solve_s": float(np.mean(times64)), "outer_iterations": st64["outer_iterations"],
                "relres": st64["relres"],
                "mixed_vs_fp64_speedup": float(np.mean(times64) / np.mean(times_mix))}
        del hp64, x64
        torch.cuda.empty_cache()

    # ---- roofline of the dominant kernel (live, HIP events) ------------------
    roofline = measure_roofline(hp_mix, x_mix, args.roofline_reps)

    roofline_vcycle = measure_vcycle(hp_mix, args.mixed, args.roofline_reps) if w.dim == 2 else None

    # ---- CPU oracle baseline on a bounded sample -----------------------------
    cpu = None
    fwd_err = None
    if not args.no_cpu:
        cpu, fwd_err = cpu_baseline(w, f, u0, x_mix, args.cpu_steps)

    out = {
        "metric": METRIC, "value": total_s / args.steps, "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": f"f64 (preconditioner {args.mixed})", "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "n": w.n, "s": w.s, "nt": w.nt,
                   "unknowns": hp_mix.U, "restart": w.restart, "tol": 1e-8,
                   "inner_k": args.inner_k, "cycles": args.cycles, "nu1": args.nu, "nu2": args.nu,
                   "mg_tail_max": args.tail_max, "coarse_max": args.coarse_max,
                   "preconditioner": args.mixed, "parallelism": "single GPU"},
        "outer_iterations": st_mix["outer_iterations"], "relres": st_mix["relres"],
        "precond_ms_per_solve": st_mix["precond_ms"],
        "fp64_preconditioner": fp64,
        "forward_error_vs_oracle_sampled_steps": fwd_err,
        "roofline": roofline, "roofline_vcycle": roofline_vcycle, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def measure_roofline(hp, x, reps):
    """apply_A: 16 B per unknown (read x once, write y once) per launch."""
    import torch
    y = torch.empty_like(x)
    sec = _event_time(lambda: hp.apply_A(x, y), reps)
    nbytes = 16.0 * hp.U
    gbs = nbytes / sec / 1e9
    traffic = measured_traffic("k_apply_A_2d") if hp.n == 512 and hp.s == 3 and hp.nt == 64 else None
    return {"kernel": "k_apply_A_2d" if hp.dim == 2 else "k_apply_A", "bound": "hbm", "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "B per launch",
            "bytes_per_launch": nbytes, "avg_launch_us": sec * 1e6}


def measured_traffic(name):
    """HBM bytes per launch of a roofline kernel from the committed counter
    summary (rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by a plain copy of
    known size), or None when the kernel's source changed since they were
    taken (its sha256 no longer matches) or no summary exists."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "roofline_heat2d_n512_s3_nt64.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        m = re.match(r"traffic (\S+) source=(\S+) sha256=([0-9a-f]+) bytes_per_launch=(\d+)", line.strip())
        if m and m.group(1) == name:
            src = os.path.join(ROOT, m.group(2))
            if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == m.group(3):
                return float(m.group(4))
    return None


def _event_time(fn, reps):
    """Average seconds per call of fn over reps calls, by HIP events on the
    current stream (the library runs on it: the binding sets the handle's
    stream to torch's current stream before each call)."""
    import torch
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def measure_vcycle(hp, precision, reps):
    """One V-cycle (from zero) on all nt stage blocks of stage 0, the batched
    shifted-block solve of Theta-tilde.  Algorithmic bytes of the fused 2D
    level kernels, per block: level l above the LDS tail moves
    5 N_l p_l + 2 N_{l+1} p_{l+1} (pre-smooth + restriction read b_l and write
    the smoothed x_l and b_{l+1}; prolongation + post-smoothing read x_l, the
    correction and b_l and write x_l); the tail reads b and writes x at its
    first level.  p_l: 8 (FP64), 4 (FP32, and level 0 of BF16/FP16), 2 (BF16/FP16
    coarse levels)."""
    import torch
    nodes, l0 = hp.mg_levels()
    L = len(nodes)
    pw = 8 if precision == "fp64" else 4
    pc = {"fp64": 8, "fp32": 4}.get(precision, 2)
    p = [pw] + [pc] * (L - 1)
    per_block = 0
    for l in range(min(l0, L - 1)):
        per_block += 5 * nodes[l] * p[l] + 2 * nodes[l + 1] * p[l + 1]
    if l0 < L:
        per_block += 2 * nodes[l0] * p[l0]
    B = hp.nt
    r = torch.randn(B * hp.N, dtype=hp.working_dtype(), device="cuda")
    z = torch.empty_like(r)
    sec = _event_time(lambda: hp.apply_mg(r, 0, out=z, cycles=1), reps)
    nbytes = float(per_block * B)
    gbs = nbytes / sec / 1e9
    traffic = (measured_traffic("vcycle") if hp.n == 512 and hp.s == 3 and hp.nt == 64 and precision == "fp32"
               else None)
    return {"kernel": "V-cycle: k_down2d per level, k_tail, k_up2d per level", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_unit": "B per launch", "bytes_per_launch": nbytes,
            "avg_launch_us": sec * 1e6, "blocks": B, "levels": nodes, "tail_level": l0}


def measure_copy(nbytes, reps):
    """Reference: a plain device-to-device copy of nbytes (read + write)."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    sec = _event_time(lambda: b.copy_(a), reps)
    return {"bytes": nbytes, "avg_launch_us": sec * 1e6, "GBs": 2 * nbytes / sec / 1e9}


def cpu_baseline(w, f, u0, x_gpu, nsteps):
    from oracle import allatonce, stepping
    import torch
    p = allatonce.Problem(w.n, w.dim, w.s, w.nt, w.T)
    tm = {}
    t0 = time.perf_counter()
    xs = stepping.solve_steps(p, f, u0, nsteps, timings=tm)
    dt = time.perf_counter() - t0
    full = tm["factor_s"] + tm["step_s"] * (w.nt / nsteps)
    # forward error of the GPU solution on the sampled steps (stepping is
    # sequential, so the first nsteps steps of x* are exactly these)
    sub = allatonce.Problem(w.n, w.dim, w.s, nsteps, p.tau * nsteps)
    vs, Vs = allatonce.split(sub, xs)
    xg = x_gpu.cpu().numpy()
    vg, Vg = allatonce.split(p, xg)
    ev = np.linalg.norm(vg[: nsteps + 1] - vs) / np.linalg.norm(vs)
    eV = np.linalg.norm(Vg[:nsteps] - Vs) / np.linalg.norm(Vs)
    cpu = {"value": full, "unit": "s", "cores": 1, "kind": "oracle",
           "sample": f"{nsteps} of {w.nt} time steps of sequential Radau IIA stepping with exact DST "
                     f"stage solves ({tm['method']}), {dt:.1f} s measured, scaled to {w.nt} steps",
           "host_cores_available": len(os.sched_getaffinity(0))}
    return cpu, {"v": float(ev), "V": float(eV), "steps": nsteps}


if __name__ == "__main__":
    main()
