"""Parity at the workloads' own shapes, every output compared with the oracle.

* 512^2, Radau IIA s = 3, nt = 64 (67.4M unknowns), FGMRES(30): the solve in
  the benchmark's configuration (FP32 and FP64 preconditioner, S-tilde by
  MGRIT) and with the S-tilde substitution, against sequential stepping
  with exact DST stage solves: all 64 steps, v and V separately.
* 128^3, s = 3, nt = 32 (270.5M unknowns), FGMRES(20), preconditioner in
  FP64, FP32, BF16 and FP16: all 32 steps against DST stepping.
* The uneven batch (64 problems of the seed-1003 recipe: n in
  {64..384}, nt in [8, 64], s in {1, 2, 3}, lognormal patch diffusivity),
  one batch solve with the FP32 preconditioner, every problem against its
  own LU stepping (computed in a pool of CPU processes).  Its residual
  tolerance is 1e-10: the stiffest problems (n = 384, kappa up to 10, so
  tau kappa / h^2 ~ 6e4) stall near 2e-11, the FP64 attainable accuracy.
* The gradient batch (8 problems, 256^2, s = 2, nt = 64, lognormal
  diffusivity): the tracking loss and its gradients with respect to f, u0
  and log kappa from the FP32-preconditioned adjoint solve, against the
  oracle's adjoint gradients; and central differences of GPU forward solves
  (tol 1e-11) on 20 random directions (seed 3004) in (f, u0, log kappa).

The solution is unique, so the bar is the forward error against the oracle,
<= 1e-8 relative; the solves run to a tighter relative residual than the
benchmark's 1e-8 because A's condition number grows like tau / h^2.
"""
import numpy as np
import pytest

import heat_inputs
import oracle_pool
from gpu_util import announce, rel_err, require_gpu, to_dev, to_host
from oracle import allatonce, stepping

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_REF = {}


def _reference(name, times):
    """x* of a workload by DST stepping on the host's cores (cached)."""
    if name not in _REF:
        w = heat_inputs.WORKLOADS[name]
        f, u0 = heat_inputs.workload_inputs(w, times)
        p = allatonce.Problem(w.n, w.dim, w.s, w.nt, w.T)
        _REF.clear()
        _REF[name] = (f, u0, stepping.solve(p, f, u0, method="dst", workers=oracle_pool.host_workers()))
    return _REF[name]


def _check_all_steps(w, x_dev, ref):
    p = allatonce.Problem(w.n, w.dim, w.s, w.nt, w.T)
    xg = to_host(x_dev)
    vg, Vg = allatonce.split(p, xg)
    vs, Vs = allatonce.split(p, ref)
    ev, eV = rel_err(vg, vs), rel_err(Vg, Vs)
    # the worst single step too, so an error confined to late steps shows
    worst = max(rel_err(vg[n], vs[n]) for n in range(1, w.nt + 1))
    return ev, eV, worst


@pytest.mark.parametrize("precision,schur", [("fp32", "mgrit"), ("fp64", "mgrit"), ("fp32", "sweep")])
def test_heat2d_n512_all_steps(precision, schur):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    w = heat_inputs.WORKLOADS["heat2d_n512_s3_nt64"]
    hp = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, restart=w.restart, tol=1e-10, maxit=200, inner_k=4,
                     precision=precision, schur=schur, mgrit_cf=8)
    # the benchmark's launch configuration: shapes from the autotuner
    tune = hp.autotune(reps=3)
    f, u0, ref = _reference(w.name, hp.stage_times())
    announce("512^2 all steps", precision, schur, "shapes", tune["tall_min_b"], tune["tail_extend"])
    x, st = hp.solve(hp.assemble_rhs(to_dev(np.ravel(f)), to_dev(u0)))
    assert st["converged"], st
    ev, eV, worst = _check_all_steps(w, x, ref)
    print(f"[512^2 {precision} {schur}] its {st['outer_iterations']} relres {st['relres']:.2e} "
          f"v {ev:.2e} V {eV:.2e} worst step {worst:.2e}")
    assert ev <= 1e-8 and eV <= 1e-8 and worst <= 1e-8
    del x, hp
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp16"])
def test_heat3d_n128_all_steps(precision):
    require_gpu()
    from paper_2609_16863_amd import HeatProblem
    w = heat_inputs.WORKLOADS["heat3d_n128_s3_nt32"]
    hp = HeatProblem(w.dim, w.n, w.s, w.nt, w.T, restart=w.restart, tol=1e-10, maxit=300, inner_k=3,
                     precision=precision, schur="mgrit", mgrit_cf=8)
    f, u0, ref = _reference(w.name, hp.stage_times())
    announce("128^3 all steps", precision)
    x, st = hp.solve(hp.assemble_rhs(to_dev(np.ravel(f)), to_dev(u0)))
    assert st["converged"], st
    ev, eV, worst = _check_all_steps(w, x, ref)
    print(f"[128^3 {precision}] its {st['outer_iterations']} relres {st['relres']:.2e} "
          f"v {ev:.2e} V {eV:.2e} worst step {worst:.2e}")
    assert ev <= 1e-8 and eV <= 1e-8 and worst <= 1e-8
    del x, hp
    torch.cuda.empty_cache()


def test_uneven_batch_64_problems():
    require_gpu()
    from paper_2609_16863_amd import HeatBatch
    specs = heat_inputs.batch_problem_specs()
    assert len(specs) == 64
    announce("uneven batch: oracle pool")
    refs = oracle_pool.run(oracle_pool.batch_reference, specs)
    data = []
    for sp in specs:
        times = allatonce.Problem(sp["n"], 2, sp["s"], sp["nt"], 1.0).stage_times()
        data.append(heat_inputs.spec_inputs(sp, times))
    announce("uneven batch: GPU", len(specs))
    hb = HeatBatch([dict(dim=2, n=sp["n"], s=sp["s"], nt=sp["nt"], kappa=k) for sp, (k, _, _) in zip(specs, data)],
                   streams=4, precision="fp32", tol=1e-10, maxit=300, inner_k=3, schur="mgrit", mgrit_cf=8)
    f = to_dev(np.concatenate([d[1].ravel() for d in data]))
    u0 = to_dev(np.concatenate([d[2].ravel() for d in data]))
    x, stats = hb.solve(hb.assemble_rhs(f, u0))
    del f, u0
    worst = 0.0
    for i, (sp, ref) in enumerate(zip(specs, refs)):
        assert stats[i]["converged"], (i, sp, stats[i])
        e = rel_err(to_host(hb.split(x)[i]), ref)
        worst = max(worst, e)
        assert e <= 1e-8, (i, sp, e)
    print(f"[uneven batch] worst forward error {worst:.2e}, outer its "
          f"{min(s['outer_iterations'] for s in stats)}..{max(s['outer_iterations'] for s in stats)}")
    hb.close()
    torch.cuda.empty_cache()


def test_gradient_batch_8x256():
    require_gpu()
    from paper_2609_16863_amd import HeatBatch
    specs = heat_inputs.gradient_problem_specs()
    announce("gradient batch: oracle pool")
    refs = oracle_pool.run(oracle_pool.gradient_reference, specs)
    data = []
    for sp in specs:
        times = allatonce.Problem(sp["n"], 2, sp["s"], sp["nt"], 1.0).stage_times()
        data.append(heat_inputs.spec_inputs(sp, times))
    # tol 1e-11: near the FP64 attainable residual of these problems
    # (tau kappa / h^2 up to 1e4); the loss then carries ~1e-11 relative error
    opts = dict(precision="fp32", tol=1e-11, maxit=300, inner_k=3, schur="mgrit", mgrit_cf=8)
    hb = HeatBatch([dict(dim=2, n=sp["n"], s=sp["s"], nt=sp["nt"], kappa=k) for sp, (k, _, _) in zip(specs, data)],
                   streams=4, **opts)
    ps = [allatonce.Problem(sp["n"], 2, sp["s"], sp["nt"], 1.0) for sp in specs]
    targets = [r[0] for r in refs]

    def forward_losses(f_list, u_list):
        x, st = hb.solve(hb.assemble_rhs(to_dev(np.concatenate([a.ravel() for a in f_list])),
                                         to_dev(np.concatenate(u_list))))
        assert all(s["converged"] for s in st), [(s["relres"], s["outer_iterations"]) for s in st]
        out, xs = [], []
        for p, xi, vt in zip(ps, hb.split(x), targets):
            v, _ = allatonce.split(p, to_host(xi))
            out.append(0.5 * float(np.sum((v[1:] - vt[1:]) ** 2)))
            xs.append(v)
        return out, x

    announce("gradient batch: forward + adjoint")
    losses, x = forward_losses([d[1] for d in data], [d[2] for d in data])
    gx = []
    for p, xi, vt in zip(ps, hb.split(x), targets):
        v, _ = allatonce.split(p, to_host(xi))
        gv = np.zeros_like(v)
        gv[1:] = v[1:] - vt[1:]
        gx.append(allatonce.join(gv, np.zeros((p.nt, p.s, p.N))))
    lam, st = hb.solve_adjoint(to_dev(np.concatenate(gx)))
    assert all(s["converged"] for s in st), [(s["relres"], s["outer_iterations"]) for s in st]
    gk = [to_host(g) for g in hb.split(hb.grad_logkappa(x, lam), "nodes")]
    grads = []
    for i, (p, ref) in enumerate(zip(ps, refs)):
        lv, lV = allatonce.split(p, to_host(hb.split(lam)[i]))
        _, Lr, gfr, gu0r, gkr = ref
        assert abs(losses[i] - Lr) <= 1e-9 * abs(Lr), i
        assert rel_err(lV, gfr) <= 1e-7, i
        assert rel_err(lv[0], gu0r) <= 1e-7, i
        assert rel_err(gk[i], gkr) <= 1e-7, i
        grads.append((lV.reshape(data[i][1].shape), lv[0], gk[i]))
    del lam, x

    # central differences of the total loss on 20 random directions in
    # (f, u0, log kappa); the diffusivity moves through aao_set_kappa
    rng = np.random.default_rng(3004)
    theta = [np.log(d[0]) for d in data]

    def total_loss(eps, dirs):
        for i in range(len(specs)):
            hb.set_kappa(i, to_dev(theta[i] + eps * dirs[i][2]), log=True)
        ls, _ = forward_losses([d[1] + eps * dd[0] for d, dd in zip(data, dirs)],
                               [d[2] + eps * dd[1] for d, dd in zip(data, dirs)])
        return sum(ls)

    announce("gradient batch: 20 central differences")
    worst = 0.0
    for k in range(20):
        dirs = [(rng.standard_normal(d[1].shape), rng.standard_normal(d[2].shape), rng.standard_normal(d[0].shape))
                for d in data]
        lin = sum(float(np.sum(g[0] * dd[0]) + g[1] @ dd[1] + g[2] @ dd[2]) for g, dd in zip(grads, dirs))
        eps = 1e-4 * np.sqrt(sum(np.sum(t * t) for t in theta)) / np.sqrt(sum(np.sum(dd[2] ** 2) for dd in dirs))
        fd = (total_loss(eps, dirs) - total_loss(-eps, dirs)) / (2 * eps)
        err = abs(fd - lin) / abs(lin)
        worst = max(worst, err)
        assert err <= 1e-5, (k, fd, lin)
    for i in range(len(specs)):
        hb.set_kappa(i, to_dev(theta[i]), log=True)
    print(f"[gradient batch] worst central-difference mismatch {worst:.2e}")
    hb.close()
    torch.cuda.empty_cache()
