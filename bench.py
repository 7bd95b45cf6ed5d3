#!/usr/bin/env python3
"""Newton-step benchmark on one MI355X.

A step is one full Newton iteration of the indentation problem: residual and
tangent reassembled on every multigrid level at the injected state, block
inverses and coarse factorisation, FGMRES + geometric-multigrid solve to a
1e-8 relative FP64 residual, state update.  The state is restored from a
device-resident copy before every step, so each step solves the same (first,
lifted) Newton system of the first load step.

Default workload: 64^3 hex elements (274,625 nodes, 2,471,625 dof), 5 levels,
8x8-element patch pushed 0.01, initial eta from seed 20110880.  The headline
value is the FP32-multigrid (mixed) path; the all-FP64 multigrid path is timed
on the same system and reported beside it.

Prints one JSON line (see the README/DESIGN for the fields).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import synth  # noqa: E402

METRIC = "Newton-step solve time & DOF/s at 1e-8 rel. residual, FP32-GMG vs FP64 GMG"
HBM_PEAK_GBS = 8000.0
# calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the same kernels at 64^3
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_patch64_mixed.txt")

WORKLOADS = {
    "tiny": synth.tiny,
    "medium": synth.medium,
    "large": synth.large,
    "scale": synth.scale_limit,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_precision(prob, precision, steps, warmup, timing, tune=True, matrix_free=-1):
    from paper_2011_08802_amd import mvpf
    gp = mvpf.Problem(prob, precision, rtol=1e-8)
    if matrix_free >= 0:
        gp.set_tuning("matrix_free", 0, matrix_free)
    gp.init_random(prob.seed)
    u0, e0, en0, _ = gp.get_state()
    u0, e0, en0 = u0.clone(), e0.clone(), en0.clone()
    depth = prob.depth_increment
    shapes = None
    if tune:  # untimed setup: pick launch shapes on this Newton system
        gp.newton_system(depth)
        shapes = gp.autotune()

    def step(rec):
        gp.set_state(u0, e0, en0, 0.0)
        t0 = time.perf_counter()
        gp.newton_system(depth)
        t1 = time.perf_counter()
        x, st = gp.solve(want_x=False)
        t2 = time.perf_counter()
        gp.newton_update()
        if rec is not None:
            rec.append(dict(system_ms=1e3 * (t1 - t0), solve_ms=st.solve_ms, its=st.iterations,
                            rel_res=st.rel_residual, converged=st.converged))

    for _ in range(warmup):
        step(None)
    recs = []
    if timing:
        gp.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(recs)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    kstats = {}
    if timing:
        for name in ("pbj_sweep", "residual", "spmv_outer"):
            n, ms, by = gp.kernel_stats(name)
            if n:
                kstats[name] = dict(launches=n, avg_ms=ms / n, bytes=by, gbs=by / (ms / n) / 1e6)
        gp.kernel_timing(False)
    # solution of the (same) Newton system for the error statement
    gp.set_state(u0, e0, en0, 0.0)
    gp.newton_system(depth)
    x, st = gp.solve()
    mf = gp.get_tuning("matrix_free")
    gp.close()
    return dict(total_s=total, recs=recs, kernels=kstats, x=x.cpu().numpy(), shapes=shapes, matrix_free=mf)


def pade_assembly(prob, reps=5):
    """Assembly cost per Pade order of the Hencky strain (Eqs. pade11, pade22,
    pade33; compared in the paper's Table 3): median Newton-system time and
    median time of the finest-level Gauss-point Hessian kernel, same state."""
    from dataclasses import replace
    from paper_2011_08802_amd import mvpf
    out = {}
    for order in (11, 22, 33):
        pr = replace(prob, material=replace(prob.material, pade=order))
        gp = mvpf.Problem(pr, "mixed", rtol=1e-8)
        gp.init_random(pr.seed)
        gp.newton_system(pr.depth_increment)  # warm-up
        gp.kernel_timing(True)
        sys_ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gp.newton_system(pr.depth_increment)
            torch.cuda.synchronize()
            sys_ms.append(1e3 * (time.perf_counter() - t0))
        n, ms, _ = gp.kernel_stats("qp_hessian")
        gp.kernel_timing(False)
        gp.close()
        out[str(order)] = dict(system_ms_median=statistics.median(sys_ms), qp_hessian_ms=ms / max(n, 1))
    return out


def run_batch(probs, precision, steps, warmup, tune=True):
    """The batched workload: all problems' Newton systems, one lockstep
    batched solve (V-cycles of all problems in one graph launch per Arnoldi
    step), all updates."""
    from paper_2011_08802_amd import mvpf
    B = mvpf.Batch(probs, precision, rtol=1e-8)
    init = []
    for i, p in enumerate(probs):
        gp = B.problem(i)
        gp.init_random(p.seed)
        u0, e0, en0, _ = gp.get_state()
        init.append((u0.clone(), e0.clone(), en0.clone()))
    depths = [p.depth_increment for p in probs]
    if tune:
        B.newton_system(depths)
        for i in range(len(probs)):
            B.problem(i).autotune()

    def step(rec):
        for i, (u0, e0, en0) in enumerate(init):
            B.problem(i).set_state(u0, e0, en0, 0.0)
        t0 = time.perf_counter()
        B.newton_system(depths)
        t1 = time.perf_counter()
        st = B.solve()
        B.newton_update()
        if rec is not None:
            rec.append(dict(system_ms=1e3 * (t1 - t0), solve_ms=st[0].solve_ms,
                            its=[x.iterations for x in st], converged=all(x.converged for x in st),
                            rel_res=max(x.rel_residual for x in st)))

    for _ in range(warmup):
        step(None)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(recs)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    B.close()
    return dict(total_s=total, recs=recs)


def run_sequential(probs, precision, steps):
    """The same problems solved one after the other (no batching), for comparison."""
    from paper_2011_08802_amd import mvpf
    gps = []
    for p in probs:
        gp = mvpf.Problem(p, precision, rtol=1e-8)
        gp.init_random(p.seed)
        u0, e0, en0, _ = gp.get_state()
        gps.append((gp, p, (u0.clone(), e0.clone(), en0.clone())))
    solve_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tot = 0.0
        for gp, p, (u0, e0, en0) in gps:
            gp.set_state(u0, e0, en0, 0.0)
            gp.newton_system(p.depth_increment)
            _, st = gp.solve(want_x=False)
            gp.newton_update()
            tot += st.solve_ms
        solve_ms.append(tot)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    for gp, _, _ in gps:
        gp.close()
    return dict(ms_per_step=1e3 * total / steps, solve_ms_median=statistics.median(solve_ms))


def batched_main(a):
    probs = synth.batched(32)
    ndof = sum(p.n_dof for p in probs)
    sizes = [p.nx for p in probs]
    log(f"[bench] batched workload: {len(probs)} problems, sizes {sizes}, {ndof} dof in total")
    res = {}
    for prec in ("mixed",) + (() if a.no_fp64 else ("fp64",)):
        log(f"[bench] batch {prec} ...")
        r = run_batch(probs, prec, a.steps, a.warmup, not a.no_tune)
        recs = r["recs"]
        res[prec] = dict(ms_per_step=1e3 * r["total_s"] / len(recs),
                         value=ndof * len(recs) / r["total_s"],
                         solve_ms_median=statistics.median(x["solve_ms"] for x in recs),
                         system_ms_median=statistics.median(x["system_ms"] for x in recs),
                         fgmres_iterations_max=max(max(x["its"]) for x in recs),
                         fgmres_iterations_min=min(min(x["its"]) for x in recs),
                         rel_residual_max=max(x["rel_res"] for x in recs),
                         converged=all(x["converged"] for x in recs))
        res[prec]["solve_dof_per_s"] = ndof / (res[prec]["solve_ms_median"] / 1e3)
    log("[bench] same problems one by one (mixed) ...")
    seq = run_sequential(probs, "mixed", max(1, min(a.steps, 2)))
    ms = res["mixed"]
    out = {
        "metric": METRIC,
        "value": ms["value"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(probs)} patch-indentation problems, n^3 hex with n in "
                               f"{{16,24,32,40,48}}, random crystal rotations, depths U[0.005,0.02], "
                               f"{ndof} dof in total, 4-5-level GMG V(2,2) (n halved while even and at least 2), FGMRES(30) rtol 1e-8",
                   "sizes": sizes, "precision": "mixed"},
        "mixed": ms,
        "sequential_mixed": seq,
        "speedup_solve_batched_vs_sequential": seq["solve_ms_median"] / ms["solve_ms_median"],
    }
    if "fp64" in res:
        out["fp64_gmg"] = res["fp64"]
        out["speedup_solve_mixed_vs_fp64"] = res["fp64"]["solve_ms_median"] / ms["solve_ms_median"]
    print(json.dumps(out), flush=True)


def indent_main(a):
    """Whole indentation runs (load to 0.03, unload to 0) of the sphere-contact
    workload with the adaptive step rule; a step here is one such run."""
    from paper_2011_08802_amd import mvpf
    prob = synth.indentation()
    ndof = prob.n_dof
    run = dict(synth.INDENT_RUN)
    if a.indent_depth > 0:
        run["depth_max"] = a.indent_depth
    # once martensite forms the systems are much harder than the patch workload's: V(4,4) with
    # damping 0.4 and FGMRES(60) take the whole run from 125 s (V(3,3), 0.5, FGMRES(30)) to 80 s
    nu = a.sweeps if a.sweeps > 0 else 4
    sweeps = dict(nu_pre=nu, nu_post=nu, omega=0.4, restart=60)
    log(f"[bench] indentation workload: {prob.nx}x{prob.ny}x{prob.nz}, {ndof} dof, run {run}, smoother {sweeps}")
    res = {}
    for prec in ("mixed",) + (() if a.no_fp64 else ("fp64",)):
        gp = mvpf.Problem(prob, prec, rtol=1e-8, **sweeps)
        gp.init_random(prob.seed)
        u0, e0, en0, _ = gp.get_state()
        u0, e0, en0 = u0.clone(), e0.clone(), en0.clone()
        if not a.no_tune:  # untimed: launch shapes on the first contact system
            gp.newton_system(run["dd_init"])
            gp.autotune()
        timing = prec == "mixed" and not a.no_timing
        runs = []
        for k in range(a.warmup + a.steps):
            gp.set_state(u0, e0, en0, 0.0)
            if timing and k == a.warmup:
                gp.kernel_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs, rc = gp.indent(on_step=lambda r, i: log(
                f"[indent {prec} run {k}] step {i}: depth {r.depth:.5f} load {r.load:.5f} newton "
                f"{r.newton_iterations} fgmres {r.linear_iterations} rejected {r.rejected}"), **run)
            torch.cuda.synchronize()
            if k >= a.warmup:
                runs.append((time.perf_counter() - t0, recs, rc))
        kst = {}
        if timing:
            n, ms, by = gp.kernel_stats("pbj_sweep")
            if n:
                kst = dict(launches=n, avg_ms=ms / n, bytes=by, gbs=by / (ms / n) / 1e6)
            gp.kernel_timing(False)
        gp.close()
        total = sum(r[0] for r in runs)
        recs = runs[-1][1]
        newton = sum(r.newton_iterations for r in recs)
        res[prec] = dict(
            run_s=total / len(runs), ok=all(r[2] == 0 for r in runs), accepted_steps=len(recs),
            rejected_steps=sum(r.rejected for r in recs), newton_iterations=newton,
            fgmres_iterations=sum(r.linear_iterations for r in recs),
            assemble_s=sum(r.assemble_ms for r in recs) / 1e3, setup_s=sum(r.setup_ms for r in recs) / 1e3,
            solve_s=sum(r.solve_ms for r in recs) / 1e3,
            value=ndof * newton * len(runs) / total,
            load_max=max(r.load for r in recs),
            p_delta=[[round(r.depth, 6), round(r.load, 6)] for r in recs], sweep=kst)
    ms = res["mixed"]
    out = {
        "metric": METRIC,
        "value": ms["value"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * ms["run_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"spherical indentation {prob.nx}x{prob.ny}x{prob.nz} Q1 hex (1x1x0.5), "
                               f"{ndof} dof, rigid sphere R={prob.radius} in penalty contact "
                               f"(eps_N={prob.eps_n:g}), load to {run['depth_max']} and unload, adaptive "
                               f"steps (7 desired / 12 max Newton iterations), {prob.n_levels}-level GMG "
                               f"V({nu},{nu}) damping 0.4, FGMRES(60) rtol 1e-8; a step = one whole "
                               f"run; value = dof x Newton iterations per second", "precision": "mixed",
                   "levels": prob.n_levels, **run},
        "mixed": ms,
    }
    if ms["sweep"]:
        k = ms["sweep"]
        out["roofline"] = {"bound": "hbm", "achieved": k["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": k["gbs"] / HBM_PEAK_GBS, "traffic": None,
                           "kernel": "finest-level FP32 smoother sweep (matrix-free: mf_element + mf_gather<2>)",
                           "bytes_per_launch": k["bytes"], "avg_ms": k["avg_ms"], "launches": k["launches"]}
    if "fp64" in res:
        out["fp64_gmg"] = res["fp64"]
    print(json.dumps(out), flush=True)


def sweep_traffic(prob, matrix_free):
    """Measured HBM bytes of one finest-level smoother sweep from the committed
    counter summary, for the workload it was taken on (64^3), else None.
    Assembled: pass 1 on two wavefronts per tile + pass 2; matrix-free: the
    element kernel + the gather with the Jacobi update."""
    if (prob.nx, prob.ny, prob.nz) != (64, 64, 64) or not os.path.exists(COUNTERS):
        return None
    npad = prob.n_nodes + (-prob.n_nodes) % 64
    ntiles = npad // 64
    nepad = (prob.nx * prob.ny * prob.nz + 63) // 64 * 64
    if matrix_free:
        want = {
            "mvpf::mf_element_kernel<float,float,float,3,20,false>": nepad * 8,
            "mvpf::mf_gather_kernel<2,float,float,float>": (npad + 255) // 256 * 256,
        }
    else:
        want = {
            "mvpf::defect_upper_split_kernel<float>": ((ntiles + 1) // 2 + 7) // 8 * 8 * 256,
            "mvpf::pbj_lower_kernel<float>": ((npad + 255) // 256 + 7) // 8 * 8 * 256,
        }
    total = 0.0
    found = set()
    with open(COUNTERS) as f:
        for line in f:
            parts = line.split()
            if len(parts) < 7 or parts[0] not in want:
                continue
            try:
                g = int(parts[1])
                rd, wr = float(parts[-2]), float(parts[-1])
            except ValueError:
                continue
            if g == want[parts[0]] and parts[0] not in found:
                found.add(parts[0])
                total += (rd + wr) * 1e6
    return total if len(found) == 2 else None


def cpu_baseline(n=16, levels=4, prob=None):
    """The oracle (test infrastructure) on a bounded sample of the workload:
    one Newton iteration (autodiff assembly of the tangent, multigrid setup,
    FGMRES+GMG to 1e-8) of the same indentation problem at n^3 elements, or
    of `prob` itself when the workload is small enough (8^3)."""
    from oracle import solver as S
    from oracle.fem import Mesh, NDOF
    from oracle.material import Card
    threads = min(16, os.cpu_count() or 1)
    torch.set_num_threads(threads)
    p = prob or synth.Problem(n, n, n, n_levels=levels, patch=max(2, n // 8), depth_increment=0.01)
    n, levels = p.nx, p.n_levels
    card = Card(p.material)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    mask, target = S.dirichlet(m, p.kind, p.patch, p.radius, depth=p.depth_increment)
    t0 = time.perf_counter()
    sysk = S.NewtonSystem(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, S.increment(mask, target, U))
    mg = S.Multigrid(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, K_fine=sysk.K)
    t1 = time.perf_counter()
    x, st = S.fgmres(sysk.A, sysk.b, mg.precondition, rtol=1e-8)
    t2 = time.perf_counter()
    return dict(value=p.n_dof / (t2 - t0), unit="DOF/s", cores=threads, kind="oracle",
                sample=f"one Newton iteration of the patch-indentation workload at {n}^3 elements "
                       f"{'(the whole workload) ' if prob is not None else ''}"
                       f"({p.n_dof} dof, {levels} levels): autodiff assembly + MG setup {t1 - t0:.1f} s, "
                       f"FGMRES+GMG {st.iterations} its {t2 - t1:.1f} s",
                solve_dof_per_s=p.n_dof / (t2 - t1), iterations=st.iterations)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=list(WORKLOADS) + ["batched", "indent"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-multigrid comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes (no autotuning)")
    ap.add_argument("--no-pade", action="store_true", help="skip the assembly cost per Pade order")
    ap.add_argument("--matrix-free", type=int, default=-1,
                    help="finest level applied from its Gauss-point Hessians (1) or assembled (0); -1: the default")
    ap.add_argument("--sweeps", type=int, default=0,
                    help="indentation workload: pre- and post-smoothing sweeps (default 3)")
    ap.add_argument("--indent-depth", type=float, default=0.0,
                    help="indentation workload: maximum depth (default: the workload's 0.03)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run an elementwise copy of this many MiB (counter calibration)")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (the structured grid would "
              "shard into z-slabs, one per GPU, with one node-plane halo per operator application)",
              file=sys.stderr)
        sys.exit(2)
    if a.calib_copy_mb:
        x = torch.ones(a.calib_copy_mb << 18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    if a.workload == "batched":
        batched_main(a)
        return
    if a.workload == "indent":
        indent_main(a)
        return
    prob = WORKLOADS[a.workload]()
    ndof = prob.n_dof
    log(f"[bench] workload {a.workload}: {prob.nx}x{prob.ny}x{prob.nz}, {ndof} dof, {prob.n_levels} levels")
    log("[bench] mixed (FP32 multigrid) ...")
    mixed = run_precision(prob, "mixed", a.steps, a.warmup, not a.no_timing, not a.no_tune, a.matrix_free)
    fp64 = None
    if not a.no_fp64:
        log("[bench] fp64 multigrid ...")
        fp64 = run_precision(prob, "fp64", a.steps, a.warmup, False, not a.no_tune, a.matrix_free)

    def summary(r):
        recs = r["recs"]
        solve_ms = statistics.median(x["solve_ms"] for x in recs)
        return dict(ms_per_step=1e3 * r["total_s"] / len(recs), solve_ms_median=solve_ms,
                    solve_dof_per_s=ndof / (solve_ms / 1e3),
                    system_ms_median=statistics.median(x["system_ms"] for x in recs),
                    fgmres_iterations=[x["its"] for x in recs],
                    rel_residual_max=max(x["rel_res"] for x in recs),
                    converged=all(x["converged"] for x in recs))

    ms = summary(mixed)
    ms["launch_shapes"] = mixed["shapes"]
    ms["matrix_free"] = mixed["matrix_free"]
    out = {
        "metric": METRIC,
        "value": ndof * a.steps / mixed["total_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{'patch' if prob.kind == 'patch' else 'spherical-cap'} indentation "
                               f"{prob.nx}x{prob.ny}x{prob.nz} Q1 hex, "
                               f"{ndof} dof, {prob.n_levels}-level GMG V(2,2), FGMRES(30) rtol 1e-8",
                   "nx": prob.nx, "ny": prob.ny, "nz": prob.nz, "levels": prob.n_levels,
                   "depth": prob.depth_increment, "seed": prob.seed, "precision": "mixed"},
        "mixed": ms,
    }
    if fp64 is not None:
        fs = summary(fp64)
        fs["launch_shapes"] = fp64["shapes"]
        out["fp64_gmg"] = fs
        out["fp64_gmg"]["value"] = ndof * a.steps / fp64["total_s"]
        out["speedup_solve_mixed_vs_fp64"] = fs["solve_ms_median"] / ms["solve_ms_median"]
        out["speedup_step_mixed_vs_fp64"] = fs["ms_per_step"] / ms["ms_per_step"]
        out["mixed_vs_fp64_solution_rel_diff"] = float(
            np.linalg.norm(mixed["x"] - fp64["x"]) / np.linalg.norm(fp64["x"]))
    k = mixed["kernels"].get("pbj_sweep")
    if k:
        mf = mixed["matrix_free"]
        out["roofline"] = {"bound": "hbm", "achieved": k["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": k["gbs"] / HBM_PEAK_GBS, "traffic": sweep_traffic(prob, mf),
                           "kernel": "finest-level FP32 smoother sweep "
                                     + ("(matrix-free: mf_element + mf_gather<2>)" if mf
                                        else "(defect_upper_split + pbj_lower)"),
                           "bytes_per_launch": k["bytes"], "avg_ms": k["avg_ms"], "launches": k["launches"]}
        out["kernels"] = mixed["kernels"]
    if not a.no_pade and a.workload in ("tiny", "medium"):
        log("[bench] assembly per Pade order ...")
        out["pade_assembly"] = pade_assembly(prob)
    if not a.no_cpu_baseline:
        log("[bench] oracle cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(prob=prob if a.workload == "tiny" else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
