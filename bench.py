"""Benchmark: all-at-once Radau IIA heat solve on one MI355X.

One step = one full FGMRES solve to a true FP64 relative residual of 1e-8 of
the all-at-once system (paper eq. (2.4)) with the block preconditioner
(eqs. (3.2)-(3.3)) applied in FP32 (the mixed-precision arm, approach A2),
its S-tilde solve done by one two-level MGRIT iteration (coarsening factor 4;
the parallel route of Sec. 5.2).  The block-diagonal Theta-tilde solve runs
4 inner GMRES iterations, S-tilde's steps and MGRIT's coarse level one, each
with one classical Gram-Schmidt pass and one V-cycle of 2 + 2 Jacobi sweeps
per shifted block; the outer FGMRES takes its second Gram-Schmidt pass from
the basis' Gram matrix.  The same solve with the FP64 preconditioner (approach
A1) is timed beside it with equal inner settings, and both again with
S-tilde by forward substitution.  Workload: 2D
heat on a 512 x 512 interior grid, Radau IIA s = 3, 64 time steps to T = 1,
FGMRES(30); seeded Gaussian-bump source and smooth random initial condition
(synthetic, generated on the host).  The multigrid launch shapes come from
the library's autotuner (aao_autotune) before timing.

Prints one JSON line.  Besides the contract keys it reports the Theta-tilde /
S-tilde time split and inner-iteration counts, the forward error against the
oracle on all time steps, per-kernel launch times of the V-cycle at the block
counts P-tilde uses, `roofline` for the dominant kernel (live, HIP events on
the launch stream; traffic from the committed counter summary while its
source is unchanged), apply_A and the 64-block V-cycle as secondary
rooflines, `cpu_baseline` (the oracle's DST stepping on all 64 steps with
every host core), and `extra` timings of the 3D 128^3 workload in four
preconditioner precisions, of the 64-problem uneven batch, and of the
paper's parallel test case #1 (Q2 elements, 255^2 nodes, s = 3, 256 steps)
with its own solver settings (test case #2, 535M unknowns, on request).
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
PBYTES = {"fp64": (8, 8), "fp32": (4, 4), "bf16": (4, 2), "fp16": (4, 2)}   # (level 0, coarse levels)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="heat2d_n512_s3_nt64")
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--inner-k", type=int, default=4)
    ap.add_argument("--cycles", type=int, default=1)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--schur", default="mgrit", choices=["mgrit", "sweep"],
                    help="S-tilde by two-level MGRIT or by forward substitution")
    ap.add_argument("--mgrit-cf", type=int, default=4)
    ap.add_argument("--mgrit-iters", type=int, default=1)
    ap.add_argument("--inner-orth", default="cgs1", choices=["cgs2", "cgs1"],
                    help="Gram-Schmidt passes of the inner GMRES")
    ap.add_argument("--outer-orth", default="gram", choices=["cgs2", "gram"],
                    help="Gram-Schmidt of the outer FGMRES")
    ap.add_argument("--schur-k", type=int, default=1,
                    help="inner GMRES iterations inside S-tilde's steps (0 = inner k)")
    ap.add_argument("--mgrit-coarse-k", type=int, default=1,
                    help="inner GMRES iterations of MGRIT's coarse propagator (0 = inner k)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch shapes")
    ap.add_argument("--launch-shapes", default=None,
                    help="TALL_MIN_B,TAIL_EXTEND: set the multigrid launch shapes instead of autotuning "
                         "(for runs under a profiler, which distorts the tuner's timings)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-preconditioner arm")
    ap.add_argument("--no-variants", action="store_true", help="skip the S-tilde substitution arms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the 3D, batch and paper-case timings")
    ap.add_argument("--paper-case2", action="store_true",
                    help="also time the paper's test case #2 (Q2, 511^2 nodes, 512 steps: 535M unknowns)")
    ap.add_argument("--paper-case-only", action="store_true",
                    help="only the paper's test case #1 (Q2) with its solver settings; for kernel traces")
    ap.add_argument("--roofline-reps", type=int, default=20)
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline launches (V-cycle kernels, apply_A, a 1 GiB copy); for counter runs")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "ROOFLINE_JSON"),
                    help="print the counter summary of the dominant kernel from two --roofline-only counter runs "
                         "(FETCH_SIZE, WRITE_SIZE counter_collection CSVs) and that run's JSON; needs no GPU")
    return ap.parse_args()


def main():
    args = parse()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the all-at-once solve "
                          "is measured at its single-GPU shape (time slabs per GPU would be the "
                          "sharding, with S-tilde by MGRIT across slabs)"}))
        sys.exit(2)
    import torch

    import heat_inputs
    from paper_2609_16863_amd import HeatProblem

    if args.paper_case_only:
        name = "paper_case1_q2_n255_s3_nt256"
        res = paper_case(heat_inputs.PAPER_CASES[name], args.mgrit_cf, args.mgrit_coarse_k, args.schur_k,
                         args.inner_orth, args.outer_orth)
        print(json.dumps({name: res}))
        return
    w = heat_inputs.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    common = dict(restart=w.restart, tol=1e-8, inner_k=args.inner_k, cycles=args.cycles, nu1=args.nu,
                  nu2=args.nu, schur=args.schur, mgrit_cf=args.mgrit_cf, mgrit_iters=args.mgrit_iters,
                  mgrit_coarse_k=args.mgrit_coarse_k, schur_k=args.schur_k, inner_orth=args.inner_orth,
                  outer_orth=args.outer_orth)
    t_setup = time.perf_counter()
    hp_mix = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, precision=args.mixed, **common)
    f, u0 = heat_inputs.workload_inputs(w, hp_mix.stage_times())
    f_d = torch.from_numpy(np.ascontiguousarray(f.ravel())).to(dev)
    u0_d = torch.from_numpy(u0).to(dev)
    rhs = hp_mix.assemble_rhs(f_d, u0_d)
    del f_d
    if args.launch_shapes:
        tall, ext = (int(v) for v in args.launch_shapes.split(","))
        hp_mix.set_launch_shapes(tall, ext)
        tune = dict(hp_mix.tune_state, source="given")
    elif args.no_autotune:
        tune = None
    else:
        tune = dict(hp_mix.autotune(reps=5), source="autotune")

    def shapes(hp):
        if tune is not None:
            hp.set_launch_shapes(tune["tall_min_b"], tune["tail_extend"])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    log(f"{w.name}: U = {hp_mix.U:,} unknowns, setup {setup_s:.1f} s, launch shapes {tune and (tune['tall_min_b'], tune['tail_extend'])}")
    if args.roofline_only:
        prof = vcycle_kernels(hp_mix, args.mixed, args.roofline_reps)
        x = torch.randn(hp_mix.U, dtype=torch.float64, device=dev)
        out = {"vcycle_kernels": prof, "apply_A": measure_apply_A(hp_mix, x, args.roofline_reps),
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
            log(f"{label} solve {it - W if it >= W else 'warmup'}: {dt * 1e3:.1f} ms, "
                f"{st['outer_iterations']} its, relres {st['relres']:.2e}, "
                f"theta {st['theta_ms']:.1f} ms, S-tilde {st['schur_ms']:.1f} ms")
        return times, stats, x

    def summary(times, st):
        return {"solve_s": float(np.mean(times)), "outer_iterations": st["outer_iterations"],
                "relres": st["relres"], "theta_ms": st["theta_ms"], "schur_ms": st["schur_ms"],
                "inner_solves": st["inner_solves"], "inner_iterations": st["inner_iterations"]}

    # ---- timed region: K mixed-precision solves -----------------------------
    torch.cuda.synchronize()
    times_mix, st_mix, x_mix = run(hp_mix, f"{args.mixed}/{args.schur}", args.steps, args.warmup)
    total_s = sum(times_mix)
    ms_per_step = 1e3 * total_s / args.steps
    x_host = x_mix.cpu().numpy()

    # ---- FP64-preconditioner arm and the substitution variants ---------------
    fp64 = None
    if not args.no_fp64:
        hp64 = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, precision="fp64", **common)
        shapes(hp64)
        times64, st64, _ = run(hp64, f"fp64/{args.schur}", args.steps, args.warmup)
        fp64 = summary(times64, st64)
        fp64["mixed_vs_fp64_speedup"] = float(np.mean(times64) / np.mean(times_mix))
        del hp64
        torch.cuda.empty_cache()
    variants = {}
    if not args.no_variants:
        other = "sweep" if args.schur == "mgrit" else "mgrit"
        for prec in ([args.mixed] + ([] if args.no_fp64 else ["fp64"])):
            hv = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, precision=prec, **dict(common, schur=other))
            shapes(hv)
            tv, sv, _ = run(hv, f"{prec}/{other}", 2, 1)
            variants[f"{prec}_{other}"] = summary(tv, sv)
            del hv
            torch.cuda.empty_cache()

    # ---- rooflines (live, HIP events on the launch stream) -------------------
    prof = vcycle_kernels(hp_mix, args.mixed, args.roofline_reps)
    dom = prof["dominant"]
    roofline = {k: v for k, v in prof["by_kernel"][dom].items() if k not in ("launches", "members")}
    roofline["kernel"] = dom
    roofline["traffic"] = measured_traffic(traffic_key(dom), w, args.mixed)
    apply_a = measure_apply_A(hp_mix, x_mix, args.roofline_reps)
    apply_a["traffic"] = measured_traffic(apply_a["kernel"], w, args.mixed)
    vc64 = prof["kernels"]["vcycle"][str(w.nt)]

    # ---- CPU oracle baseline and the forward error ---------------------------
    cpu = fwd_err = None
    if not args.no_cpu:
        cpu, fwd_err = cpu_baseline(w, f, u0, x_host)
    del x_mix

    # ---- the other workloads (3D in four precisions, the uneven batch) --------
    extra = None if args.no_extras else extras(args, tune is not None and tune["source"] == "autotune")

    out = {
        "metric": METRIC, "value": total_s / args.steps, "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": f"f64 (preconditioner {args.mixed})", "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "n": w.n, "s": w.s, "nt": w.nt,
                   "unknowns": hp_mix.U, "restart": w.restart, "tol": 1e-8,
                   "inner_k": args.inner_k, "cycles": args.cycles, "nu1": args.nu, "nu2": args.nu,
                   "schur": args.schur, "mgrit_cf": args.mgrit_cf, "mgrit_iters": args.mgrit_iters,
                   "mgrit_coarse_k": args.mgrit_coarse_k or args.inner_k, "schur_k": args.schur_k or args.inner_k,
                   "inner_orth": args.inner_orth, "outer_orth": args.outer_orth,
                   "preconditioner": args.mixed, "launch_shapes": tune and {k: tune[k] for k in
                                                                            ("tall_min_b", "tail_extend", "source")},
                   "parallelism": "single GPU"},
        "outer_iterations": st_mix["outer_iterations"], "relres": st_mix["relres"],
        "phases_ms_per_solve": {"theta": st_mix["theta_ms"], "schur": st_mix["schur_ms"]},
        "inner": {"solves": st_mix["inner_solves"], "iterations": st_mix["inner_iterations"]},
        "fp64_preconditioner": fp64, "schur_variants": variants,
        "forward_error_vs_oracle": fwd_err,
        "roofline": roofline, "roofline_apply_A": apply_a,
        "roofline_vcycle_64_blocks": vc64, "vcycle_kernels": prof,
        "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(out))


def vcycle_kernels(hp, precision, reps):
    """Per-launch times of one V-cycle at the block counts P-tilde uses (one
    S-tilde step; an MGRIT relaxation batch; all nt Theta-tilde blocks), with
    each kernel's algorithmic bytes: per block, a tiled down kernel at level l
    reads b_l and writes the smoothed x_l and b_{l+1}  [p(2 N_l) + p' N_{l+1}];
    an up kernel reads x_l, the correction and b_l and writes x_l
    [p(3 N_l) + p' N_{l+1}]; the register tail reads b and writes x at its
    first level [2 p N_tail]; p / p' the storage bytes of the two levels.
    The dominant kernel is the one with the most time per application of
    P-tilde: sum over block counts of (V-cycles per application) x (mean
    launch time), with the V-cycle counts of the autotuner's report."""
    nodes, tail = hp.mg_levels()
    p0, pc = PBYTES[precision]
    pl = [p0] + [pc] * (len(nodes) - 1)
    nt, s, k = hp.nt, hp.s, hp.options["inner_k"]
    cf = hp.options["mgrit_cf"]
    K = -(-nt // cf)
    ks = hp.options["schur_k"] or k
    per_solve = ks * s * hp.options["cycles"]   # V-cycles per inner GMRES solve of an S-tilde step
    weight = {}

    def add(B, n):
        if B >= 1 and n > 0:
            weight[B] = weight.get(B, 0) + n

    if hp.options["schur"] == "mgrit":
        # per iteration: F-relaxation steps j = 1..cf-1 over the intervals
        # that reach kc + j, the step into the K-1 C-points, and K-2 coarse
        # steps (the first correction needs none); then the last F-relaxation
        it = hp.options["mgrit_iters"]
        for j in range(1, cf):
            add(min(K, (nt - j) // cf + 1) if j <= nt else 0, per_solve * (it + 1))
        add(K - 1, per_solve * it)
        kc = hp.options["mgrit_coarse_k"] or k
        add(1, kc * s * hp.options["cycles"] * it * max(K - 2, 0))
        if nt % cf == 0:
            add(1, per_solve)
    else:
        add(1, per_solve * nt)
    add(nt, k * s * hp.options["cycles"])   # Theta-tilde: every step at once, inner_k iterations
    counts = sorted(weight)

    def kbytes(label):
        name, lev = label.split("@")
        lev = int(lev)
        if name == "k_down2d":
            return pl[lev] * 2 * nodes[lev] + pl[lev + 1] * nodes[lev + 1]
        if name == "k_up2d":
            return pl[lev] * 3 * nodes[lev] + pl[lev + 1] * nodes[lev + 1]
        if name in ("k_tail_fast", "k_tail"):
            return 2 * pl[lev] * nodes[lev]
        if name == "k_down3d_march":   # reads b, writes x2, b_{l+1} (and x_{l+1} when that level sweeps)
            first_sweep = lev + 2 < len(nodes)
            return 2 * pl[lev] * nodes[lev] + (2 if first_sweep else 1) * pl[lev + 1] * nodes[lev + 1]
        if name == "k_up3d_march":     # reads x2, b and the correction, writes x
            return 3 * pl[lev] * nodes[lev] + pl[lev + 1] * nodes[lev + 1]
        if name == "k_restrict":       # reads r, writes b_{l+1} (and x_{l+1} when that level sweeps)
            first_sweep = lev + 2 < len(nodes)
            return pl[lev] * nodes[lev] + (2 if first_sweep else 1) * pl[lev + 1] * nodes[lev + 1]
        if name == "k_residual":       # reads x and b, writes r
            return 3 * pl[lev] * nodes[lev]
        if name == "k_smooth":         # reads x and b, writes x (zero-start sweeps of the coarse
            return 3 * pl[lev] * nodes[lev]   # levels are formed in the restriction)
        if name == "k_prolong":        # reads x and the correction, writes x
            return 2 * pl[lev] * nodes[lev] + pl[lev + 1] * nodes[lev + 1]
        return None

    tall_min = hp.tune_state["tall_min_b"] if hp.tune_state else 8
    side = [int(round(v ** (1.0 / hp.dim))) for v in nodes]
    nu2 = hp.options["nu2"]

    nu1 = hp.options["nu1"]

    def march_shape(label, B):
        """(strips, rows of a segment, waves at 16-row segments) of the
        row-marching kernels for this launch: one wave per strip of
        64 - 2 nu2 (up) or 62 - 2 nu1 (down) columns."""
        name, lev = label.split("@")
        nf = side[int(lev)]
        ow = 64 - 2 * nu2 if name == "k_up2d" else 62 - 2 * nu1
        strips = -(-nf // ow)
        waves16 = strips * -(-nf // 16) * B
        return strips, (32 if waves16 > 8 * 4 * 256 else 16), waves16

    def marches(label, B):
        """Level 0 of the constant-coefficient 2D operator from tall_min
        blocks runs the row-marching kernels (the profiled cycle starts from
        zero and forms no coupling terms), and so do its tensor levels when
        the launch has 4 waves per SIMD at 16-row segments."""
        name, lev = label.split("@")
        if name not in ("k_up2d", "k_down2d") or hp.dim != 2 or hp.disc != "fd" or hp._kappa is not None:
            return False
        if B < tall_min:
            return False
        return lev == "0" or march_shape(label, B)[2] >= 4 * 4 * 256

    def march_grid(label, B):
        """Workgroups of a row-marching launch: four waves each."""
        strips, seg, _ = march_shape(label, B)
        nf = side[int(label.split("@")[1])]
        return -(-(strips * -(-nf // seg) * B) // 4)

    def grid_workgroups(label, B):
        """Workgroups of one launch (what a counter run reports per dispatch):
        the 2D tiled level kernels cover the coarse level in tiles of 16 x 8
        (short) or 16 x 16 (tall) coarse nodes, 256 threads each, per block;
        the tail runs one workgroup per block."""
        name, lev = label.split("@")
        if name in ("k_down3d_march", "k_up3d_march"):
            # 32 x 32-thread tiles with 26 x 26 (down) or 28 x 28 (up) cores,
            # chunks of 32 planes (16 when that leaves under 512 workgroups)
            nf = side[int(lev)]
            ntx = -(-nf // (26 if name == "k_down3d_march" else 28))
            zlen = nf if nf < 32 else 32
            if ntx * ntx * -(-nf // zlen) * B < 512 and nf > 16:
                zlen = 16
            return ntx * ntx * -(-nf // zlen) * B
        if hp.dim != 2:
            return None
        if marches(label, B):
            return march_grid(label, B)
        if name in ("k_down2d", "k_up2d"):
            nc = side[int(lev) + 1]
            ty = 16 if (precision != "fp64" and B >= tall_min) else 8
            return -(-nc // 16) * -(-nc // ty) * B
        if name in ("k_tail_fast", "k_tail"):
            return B
        return None

    kernels, totals = {"vcycle": {}}, {}
    for B in counts:
        launches, total_us = hp.profile_vcycle(count=B, stage=0, reps=reps)
        vc_bytes = 0
        for label, us, us_alone in launches:
            nb = kbytes(label)
            entry = {"avg_launch_us": us, "alone_us": us_alone, "bound": "hbm", "peak": HBM_PEAK_GBS,
                     "unit": "GB/s"}
            if nb is not None:
                entry["bytes_per_launch"] = float(nb * B)
                entry["achieved"] = nb * B / (us * 1e-6) / 1e9
                entry["frac"] = entry["achieved"] / HBM_PEAK_GBS
                vc_bytes += nb * B
            kernels.setdefault(label, {})[str(B)] = entry
            totals[label] = totals.get(label, 0.0) + weight.get(B, 0) * us
        gbs = vc_bytes / (total_us * 1e-6) / 1e9
        kernels["vcycle"][str(B)] = {"avg_launch_us": total_us, "bytes_per_launch": float(vc_bytes),
                                     "achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "bound": "hbm",
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "blocks": B, "levels": nodes,
                                     "tail_level": tail}
    # group the launches by compiled kernel (what a kernel trace reports):
    # level 0 and the coarse levels are different instantiations, and so are
    # the short and tall tiles of the tiled kernels
    def symbol(label, B):
        name, lev = label.split("@")
        if marches(label, B):
            return name + ("_march<level 0>" if lev == "0" else "_march<coarse levels>")
        sym = name + ("<level 0" if lev == "0" else "<coarse levels")
        if name in ("k_down2d", "k_up2d") and precision != "fp64":
            sym += ", tall tiles" if B >= tall_min else ", short tiles"
        return sym + ">"

    groups = {}
    for label, per_b in kernels.items():
        if label == "vcycle":
            continue
        for b, e in per_b.items():
            B = int(b)
            g = groups.setdefault(symbol(label, B), {"launches": 0.0, "us": 0.0, "alone": 0.0, "bytes": 0.0,
                                                     "labels": set(), "members": []})
            if weight.get(B, 0):
                g["members"].append({"label": label, "blocks": B, "weight": weight[B],
                                     "workgroups": grid_workgroups(label, B),
                                     "bytes_per_launch": e.get("bytes_per_launch")})
            g["launches"] += weight.get(B, 0)
            g["us"] += weight.get(B, 0) * e["avg_launch_us"]
            g["alone"] += weight.get(B, 0) * e["alone_us"]
            g["bytes"] += weight.get(B, 0) * e.get("bytes_per_launch", 0.0)
            g["labels"].add(f"{label} x{B}")
    # launch durations: each launch replayed alone from a graph (its kernel
    # time plus the short gap between graph nodes, which is what a kernel
    # trace's average tracks); the in-situ times add the dispatch gap after
    # an event to every launch
    all_us = sum(g["alone"] for g in groups.values())
    table = {}
    for sym, g in groups.items():
        if g["launches"] == 0:
            continue
        avg = g["alone"] / g["launches"]
        gbs = g["bytes"] / (g["alone"] * 1e-6) / 1e9
        table[sym] = {"launches_per_application": g["launches"], "avg_launch_us": avg,
                      "in_situ_us": g["us"] / g["launches"],
                      "bytes_per_launch": g["bytes"] / g["launches"], "achieved": gbs,
                      "frac": gbs / HBM_PEAK_GBS, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "share_of_vcycle_time": g["alone"] / all_us, "launches": sorted(g["labels"]),
                      "members": g["members"]}
    dom = max(table, key=lambda k: table[k]["share_of_vcycle_time"])
    return {"kernels": kernels, "weights": {str(b): weight.get(b, 0) for b in counts},
            "by_kernel": table, "dominant": dom}


def measure_apply_A(hp, x, reps):
    """apply_A: 16 B per unknown (read x once, write y once) per launch."""
    import torch
    y = torch.empty_like(x)
    sec = _event_time(lambda: hp.apply_A(x, y), reps)
    nbytes = 16.0 * hp.U
    gbs = nbytes / sec / 1e9
    return {"kernel": "k_apply_A_2d" if hp.dim == 2 else "k_apply_A_3d", "bound": "hbm", "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_launch": nbytes, "avg_launch_us": sec * 1e6}


def traffic_key(symbol):
    """The kernel group's name in the counter summary (no spaces)."""
    return symbol.replace(" ", "")


def _counter_rows(path, counter):
    """(kernel name, workgroups, value in KiB) per dispatch of a rocprofv3
    counter_collection CSV."""
    import csv
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            wg = int(r.get("Workgroup_Size") or 1) or 1
            out.append((r["Kernel_Name"], int(r["Grid_Size"]) // wg, float(r["Counter_Value"])))
    return out


def _kernel_matches(name, base, level0):
    """name is an instantiation of the multigrid kernel `base` (tiled or
    row-marching) for level 0 (first template argument 0 or 1: the fine-grid
    kinds) or for the coarse levels (2 or 3: tensor or stored-stencil
    Galerkin operators)."""
    i = name.find(base + "<")
    if i < 0:
        return False
    first = name[i + len(base) + 1:].split(",")[0].split(">")[0].strip()
    if not first.lstrip("-").isdigit():   # no level kind in the template: a level-0 kernel (3D marches)
        return level0
    return (int(first) <= 1) == level0


def traffic_summary(fetch_csv, write_csv, roof_json):
    """Markdown summary of the HBM traffic of every V-cycle kernel group (the
    benchmark's dominant kernel is one of them) and of apply_A from two
    counter runs of `bench.py --roofline-only` (FETCH_SIZE, WRITE_SIZE),
    scaled by what the counters read for the 1 GiB copy in the same runs."""
    import hashlib
    import statistics
    roof = json.loads([ln for ln in open(roof_json) if ln.startswith("{")][-1])
    prof = roof["vcycle_kernels"]
    fetch, write = _counter_rows(fetch_csv, "FETCH_SIZE"), _counter_rows(write_csv, "WRITE_SIZE")
    nbytes = roof["copy_reference"]["bytes"]

    def copy_kib(rows):
        # the reference copy is the run's last copy dispatch (--roofline-only
        # times it last; earlier copies, such as the right-hand side's, have
        # other sizes)
        vals = [v for name, wg, v in rows if "copyBuffer" in name]
        if not vals:
            raise SystemExit("no copy dispatch in the counter run")
        return vals[-1]

    f_scale = nbytes / 1024 / copy_kib(fetch)
    w_scale = nbytes / 1024 / copy_kib(write)
    lines = [f"copy reference: {nbytes:,} B read and written; FETCH_SIZE reads {copy_kib(fetch):,.0f} KiB "
             f"(scale {f_scale:.3f}), WRITE_SIZE {copy_kib(write):,.0f} KiB (scale {w_scale:.3f})", "",
             f"dominant kernel group in this run: {prof['dominant']}", "",
             "| group | launch | blocks | workgroups | launches per P-tilde | FETCH_SIZE KiB | WRITE_SIZE KiB "
             "| scaled bytes | algorithmic bytes | ratio |", "|---|---|---|---|---|---|---|---|---|---|"]
    per_group = {}
    unmatched = []
    for sym, grp in sorted(prof["by_kernel"].items()):
        base = sym.split("<")[0]
        level0 = "<level 0" in sym
        tot_w = tot_meas = tot_alg = 0.0
        if any(m["workgroups"] is None or m["bytes_per_launch"] is None for m in grp["members"]):
            unmatched.append(sym)   # no grid size (3D grid kernels) or no byte count: not matched
            continue
        for m in grp["members"]:
            fv = [v for name, wg, v in fetch if wg == m["workgroups"] and _kernel_matches(name, base, level0)]
            wv = [v for name, wg, v in write if wg == m["workgroups"] and _kernel_matches(name, base, level0)]
            if not fv or not wv:
                raise SystemExit(f"no dispatch of {base} with {m['workgroups']} workgroups")
            fk, wk = statistics.median(fv), statistics.median(wv)
            meas = fk * 1024 * f_scale + wk * 1024 * w_scale
            alg = m["bytes_per_launch"]
            lines.append(f"| {sym} | `{m['label']}` | {m['blocks']} | {m['workgroups']} | {m['weight']:g} | {fk:,.0f} | "
                         f"{wk:,.0f} | {meas:,.0f} | {alg:,.0f} | {meas / alg:.3f} |")
            tot_w += m["weight"]
            tot_meas += m["weight"] * meas
            tot_alg += m["weight"] * alg
        per_group[sym] = (tot_meas / tot_w, tot_alg / tot_w)
    if unmatched:
        lines += ["", "groups without a known grid size or byte count (not matched): " + ", ".join(unmatched)]
    lines += ["", "| group | measured bytes per launch | algorithmic bytes per launch | ratio |", "|---|---|---|---|"]
    for sym, (meas, alg) in per_group.items():
        lines.append(f"| {sym} | {meas:,.0f} | {alg:,.0f} | {meas / alg:.3f} |")
    lines.append("")
    # apply_A, the secondary roofline, from the same runs
    ka = roof["apply_A"]["kernel"]
    fa = [v for name, wg, v in fetch if f"{ka}<" in name]
    wa = [v for name, wg, v in write if f"{ka}<" in name]
    if not fa or not wa:
        raise SystemExit(f"no dispatch of {ka}")
    fk, wk = statistics.median(fa), statistics.median(wa)
    meas_a = fk * 1024 * f_scale + wk * 1024 * w_scale
    alg_a = roof["apply_A"]["bytes_per_launch"]
    lines += [f"{ka}: FETCH_SIZE {fk:,.0f} KiB, WRITE_SIZE {wk:,.0f} KiB per launch (median of {len(fa)}); "
              f"{meas_a:,.0f} B measured, {alg_a:,.0f} B algorithmic (ratio {meas_a / alg_a:.3f})", ""]

    def sha(src):
        return hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()

    src = "paper_2609_16863_amd/csrc/kern_mg.hip"
    for sym, (meas, _) in per_group.items():
        lines.append(f"traffic {traffic_key(sym)} source={src} sha256={sha(src)} bytes_per_launch={meas:.0f}")
    src = "paper_2609_16863_amd/csrc/kern_allatonce.hip"
    lines.append(f"traffic {ka} source={src} sha256={sha(src)} bytes_per_launch={meas_a:.0f}")
    print("\n".join(lines))


def measured_traffic(kernel, w, precision):
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary (rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by a plain copy of
    known size), or None when the kernel's source changed since they were
    taken (its sha256 no longer matches) or no summary exists."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{w.name}_{precision}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        m = re.match(r"traffic (\S+) source=(\S+) sha256=([0-9a-f]+) bytes_per_launch=(\d+)", line.strip())
        if m and m.group(1) == kernel:
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


def measure_copy(nbytes, reps):
    """Reference: a plain device-to-device copy of nbytes (read + write)."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    sec = _event_time(lambda: b.copy_(a), reps)
    return {"bytes": nbytes, "avg_launch_us": sec * 1e6, "GBs": 2 * nbytes / sec / 1e9}


def cpu_baseline(w, f, u0, x_gpu):
    """The oracle (sequential Radau IIA stepping with exact DST stage solves,
    FFTs on every host core) on the whole workload, and the GPU solution's
    forward error against it on all steps."""
    from oracle import allatonce, stepping
    cores = len(os.sched_getaffinity(0))
    p = allatonce.Problem(w.n, w.dim, w.s, w.nt, w.T)
    tm = {}
    t0 = time.perf_counter()
    xs = stepping.solve(p, f, u0, method="dst", workers=cores, timings=tm)
    dt = time.perf_counter() - t0
    vs, Vs = allatonce.split(p, xs)
    vg, Vg = allatonce.split(p, x_gpu)
    ev = np.linalg.norm(vg - vs) / np.linalg.norm(vs)
    eV = np.linalg.norm(Vg - Vs) / np.linalg.norm(Vs)
    cpu = {"value": dt, "unit": "s", "cores": cores, "kind": "oracle",
           "sample": f"the whole workload: {w.nt} steps of sequential Radau IIA stepping with exact DST "
                     f"stage solves (scipy.fft on {cores} workers), setup {tm['factor_s']:.2f} s + "
                     f"stepping {tm['step_s']:.2f} s"}
    return cpu, {"v": float(ev), "V": float(eV), "steps": w.nt}


def extras(args, autotune):
    """3D 128^3 (s = 3, nt = 32, FGMRES(20)) with the preconditioner in FP64,
    FP32, BF16 and FP16, the 64-problem uneven batch (FP32) and the paper's
    Q2 test cases, each timed over a few solves after a warm-up."""
    import torch

    import heat_inputs
    from paper_2609_16863_amd import HeatBatch, HeatProblem
    out = {}
    tableaux = {}

    def stage_times(s, nt, T):
        # the library's Radau IIA nodes c (from a tiny handle per s)
        if s not in tableaux:
            tableaux[s] = HeatProblem(2, 2, s, 1, 1.0).tableau()[2]
        return (np.arange(nt)[:, None] + tableaux[s][None, :]) * (T / nt)

    w3 = heat_inputs.WORKLOADS["heat3d_n128_s3_nt32"]
    res3, shapes3 = {}, {}
    for prec in ["fp64", "fp32", "bf16", "fp16"]:
        hp = HeatProblem(w3.dim, w3.n, w3.s, w3.nt, w3.T, restart=w3.restart, tol=1e-8, inner_k=args.inner_k,
                         precision=prec, schur=args.schur, mgrit_cf=args.mgrit_cf,
                         mgrit_coarse_k=args.mgrit_coarse_k, schur_k=args.schur_k, inner_orth=args.inner_orth,
                         outer_orth=args.outer_orth)
        if autotune:   # launch shapes from the library's autotuner, as for the main workload
            t = hp.autotune(reps=3)
            shapes3[prec] = {"tall_min_b": t["tall_min_b"], "tail_extend": t["tail_extend"]}
        f, u0 = heat_inputs.workload_inputs(w3, hp.stage_times())
        rhs = hp.assemble_rhs(torch.from_numpy(np.ascontiguousarray(f.ravel())).cuda(), torch.from_numpy(u0).cuda())
        del f
        times, st = [], None
        for it in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = hp.solve(rhs)
            torch.cuda.synchronize()
            if it > 0:
                times.append(time.perf_counter() - t0)
            del x
        log(f"3D {prec}: {np.mean(times) * 1e3:.0f} ms, {st['outer_iterations']} its")
        res3[prec] = {"solve_s": float(np.mean(times)), "outer_iterations": st["outer_iterations"],
                      "relres": st["relres"], "theta_ms": st["theta_ms"], "schur_ms": st["schur_ms"]}
        if prec == "fp64":
            apply3 = measure_apply_A(hp, rhs, args.roofline_reps)
        del hp, rhs
        torch.cuda.empty_cache()
    out[w3.name] = {"unknowns": w3.n ** 3 * (w3.nt * (w3.s + 1) + 1), "restart": w3.restart, "inner_k": args.inner_k,
                    "schur": args.schur, "mgrit_cf": args.mgrit_cf, "mgrit_coarse_k": args.mgrit_coarse_k,
                    "schur_k": args.schur_k, "inner_orth": args.inner_orth, "outer_orth": args.outer_orth,
                    "solves": res3, "roofline_apply_A": apply3, "launch_shapes": shapes3 or "library default"}
    specs = heat_inputs.batch_problem_specs()
    data = []
    for sp in specs:
        times = stage_times(sp["s"], sp["nt"], 1.0)
        data.append(heat_inputs.spec_inputs(sp, times))
    hb = HeatBatch([dict(dim=2, n=sp["n"], s=sp["s"], nt=sp["nt"], kappa=kap) for sp, (kap, _, _) in zip(specs, data)],
                   streams=4, precision="fp32", tol=1e-8, inner_k=args.inner_k, schur=args.schur, mgrit_cf=args.mgrit_cf,
                   mgrit_coarse_k=args.mgrit_coarse_k, schur_k=args.schur_k, inner_orth=args.inner_orth,
                   outer_orth=args.outer_orth)
    rhs = hb.assemble_rhs(torch.from_numpy(np.concatenate([d[1].ravel() for d in data])).cuda(),
                          torch.from_numpy(np.concatenate([d[2].ravel() for d in data])).cuda())
    times = []
    for it in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = hb.solve(rhs)
        torch.cuda.synchronize()
        if it > 0:
            times.append(time.perf_counter() - t0)
        del x
    its = [s["outer_iterations"] for s in st]
    log(f"uneven batch: {np.mean(times) * 1e3:.0f} ms, outer its {min(its)}..{max(its)}")
    out["batch64_uneven_kappa"] = {"problems": len(specs), "unknowns": hb.U, "solve_s": float(np.mean(times)),
                                   "outer_iterations_min_max": [min(its), max(its)],
                                   "converged": all(s["converged"] for s in st), "preconditioner": "fp32",
                                   "schur": args.schur, "streams": 4, "inner_k": args.inner_k,
                                   "inner_orth": args.inner_orth, "outer_orth": args.outer_orth}
    hb.close()
    torch.cuda.empty_cache()
    cases = ["paper_case1_q2_n255_s3_nt256"] + (["paper_case2_q2_n511_s3_nt512"] if args.paper_case2 else [])
    for name in cases:
        out[name] = paper_case(heat_inputs.PAPER_CASES[name], args.mgrit_cf, args.mgrit_coarse_k, args.schur_k,
                               args.inner_orth, args.outer_orth)
    return out


# The paper's CPU figures for its parallel test cases (Sec. 5.2, Tables 5 and
# 6; MPI-Fortran on Xeon Platinum 8358 cores): outer (inner) iterations and
# total seconds T_p on p = 1, 8, 64 processes.  Context only: another machine.
PAPER_TABLE = {
    "paper_case1_q2_n255_s3_nt256": {
        "single": {"its": "9 (24)", "T_s": {"1": 2469.4, "8": 464.9, "64": 135.0}},
        "double": {"its": "7 (23)", "T_s": {"1": 3316.0, "8": 585.3, "64": 149.9}}},
    "paper_case2_q2_n511_s3_nt512": {
        "single": {"its": "11 (33)", "T_s": {"1": 36272.4, "8": 6683.2, "64": 1677.8}},
        "double": {"its": "8 (30)", "T_s": {"1": 77926.6, "8": 11745.0, "64": 2592.2}}},
}


def paper_case(case, mgrit_cf, mgrit_coarse_k, schur_k, inner_orth, outer_orth, reps=2):
    """One of the paper's parallel test cases (Q2 elements, Sec. 5.2) with the
    paper's solver settings: left-preconditioned FGMRES(15), tol 1e-8, the
    inner GMRES on Theta-tilde stopped after 3 iterations or at 1e-3 (P-tilde
    in FP32) and after 5 or at 1e-6 (FP64), S-tilde by MGRIT with the fine
    propagator on the coarse level too (coarsening factor 8); plus the FP32
    P-tilde on the right with the benchmark's MGRIT (mgrit_cf, with
    mgrit_coarse_k inner iterations on the coarse level and schur_k in the
    S-tilde steps).  Left
    preconditioning stops on the preconditioned residual, so it wants P-tilde
    close to linear: the cheaper coarse propagator is kept to the right.
    Reports the solve time (mean of ``reps`` after a warm-up), the
    iterations, the true relative residual, and the largest nodal error
    against the manufactured solution relative to max |v|."""
    import torch

    import heat_inputs
    from paper_2609_16863_amd import HeatProblem
    paper_mgrit = dict(mgrit_cf=8, mgrit_coarse_k=0)
    settings = {"left_fp32": dict(side="left", precision="fp32", inner_k=3, inner_tol=1e-3, **paper_mgrit),
                "left_fp64": dict(side="left", precision="fp64", inner_k=5, inner_tol=1e-6, **paper_mgrit),
                "right_fp32": dict(side="right", precision="fp32", inner_k=3, inner_tol=1e-3, mgrit_cf=mgrit_cf,
                                   mgrit_coarse_k=mgrit_coarse_k, schur_k=schur_k, inner_orth=inner_orth,
                                   outer_orth=outer_orth)}
    res = {}
    for label, kw in settings.items():
        hp = HeatProblem(2, case.n, case.s, case.nt, case.tf, disc="q2", length=case.length, restart=case.restart,
                         tol=1e-8, maxit=100, schur="mgrit", **kw)
        times_st = hp.stage_times()
        f, u0, exact = heat_inputs.paper_case_inputs(case, times_st)
        rhs = hp.assemble_rhs(torch.from_numpy(np.ascontiguousarray(f.ravel())).cuda(), torch.from_numpy(u0).cuda())
        del f
        times = []
        for it in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = hp.solve(rhs)
            torch.cuda.synchronize()
            if it > 0:
                times.append(time.perf_counter() - t0)
            if it < reps:
                del x
        v = x[: (case.nt + 1) * case.N].view(case.nt + 1, case.N).cpu().numpy()
        del x
        tau = case.tf / case.nt
        err, vmax = 0.0, 0.0
        for m in range(case.nt + 1):
            ex = exact(m * tau)
            err = max(err, float(np.max(np.abs(v[m] - ex))))
            vmax = max(vmax, float(np.max(np.abs(ex + 1.0))))
        log(f"{case.name} {label}: {np.mean(times) * 1e3:.0f} ms, {st['outer_iterations']} its "
            f"({st['inner_iterations']} inner), relres {st['relres']:.1e}, error {err / vmax:.1e}")
        res[label] = {"solve_s": float(np.mean(times)), "outer_iterations": st["outer_iterations"],
                      "inner_iterations": st["inner_iterations"], "converged": st["converged"],
                      "true_relres": st["relres"], "max_error_vs_manufactured": err / vmax,
                      "theta_ms": st["theta_ms"], "schur_ms": st["schur_ms"], "mgrit_cf": kw["mgrit_cf"],
                      "mgrit_coarse_k": kw["mgrit_coarse_k"] or kw["inner_k"],
                      "schur_k": kw.get("schur_k", 0) or kw["inner_k"],
                      "inner_orth": kw.get("inner_orth", "cgs2"), "outer_orth": kw.get("outer_orth", "cgs2")}
        del hp, rhs, v
        torch.cuda.empty_cache()
    res["left_fp32_vs_fp64_speedup"] = res["left_fp64"]["solve_s"] / res["left_fp32"]["solve_s"]
    return {"elements": "Q2", "nodes": case.N, "s": case.s, "nt": case.nt, "tf": case.tf,
            "unknowns": case.N * (case.nt * (case.s + 1) + 1), "restart": case.restart, "schur": "mgrit",
            "solves": res, "paper_cpu_for_context": PAPER_TABLE[case.name]}


if __name__ == "__main__":
    main()
