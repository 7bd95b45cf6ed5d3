#!/usr/bin/env python3
"""Newton-step benchmark on one MI355X.

A step is one Newton iteration of a running indentation simulation: residual
and tangent reassembled on every multigrid level at the injected state, block
inverses and coarse factorisation, FGMRES + geometric-multigrid solve to a
1e-8 relative FP64 residual, state update and the Newton convergence test.
The simulation runs the workload's load steps in order (the state is never
reset): each load step's Newton iterations continue until the free-dof
residual is below 1e-9 of its first right-hand side, then the next load step
starts from the converged state.  The first W iterations are untimed
(warm-up); the next K are timed, so the timed systems are the later, harder
ones of the run, not a repeat of the first.

Default workload: the single-GPU scale limit, 256x256x128 hex elements on a
1x1x0.5 box (76,682,889 dof), 6 levels, spherical-cap indenter of radius 0.2
pushed 0.0025 per load step.  The headline value is the FP32-multigrid
(mixed) path; the all-FP64 multigrid path runs the same Newton sequence and
is timed beside it.  Also reported: the 64^3 patch workload's whole 5-step
run with every Newton solve, and the CPU oracle on the whole 8^3 workload and
on a bounded sample of the default workload, each with the GPU solutions'
error against the oracle's.

Prints one JSON line (see the README/DESIGN for the fields).
"""
import argparse
import dataclasses
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
# calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of the same kernels, per workload
COUNTERS = {
    "medium": os.path.join(ROOT, "profiles", "hbm_counters_patch64_mixed.txt"),
    "scale": os.path.join(ROOT, "profiles", "hbm_counters_cap256x256x128_mixed.txt"),
}

WORKLOADS = {
    "tiny": synth.tiny,
    "medium": synth.medium,
    "large": synth.large,
    "scale": synth.scale_limit,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class NewtonRun:
    """Newton iterations of one problem's load-step sequence through the
    C ABI, with the library's own step rule (Sec. 3.4, as mvpf_time_step):
    iterate newton_system / solve / newton_update until the free-dof
    residual is <= newton_rtol times the attempt's first right-hand side
    norm (a linear solve stopped at max_it still gives its update).  An
    attempt fails after newton_max solves without convergence, on a
    non-finite residual or on a singular 9x9 block / coarse operator; then
    the state of the attempt's start is restored and the depth increment
    halved (at most 8 times per load step).  The material's rho belongs to the whole load step; an
    attempt over a fraction f of it runs with rho / f (the time step is
    proportional to the increment).  An accepted attempt sets eta_n <- eta
    and, if it stopped short of the load step's depth, the next attempt goes
    on to it.  One call of iteration() is one Newton iteration (a failed
    attempt's restore is part of the iteration that ended it)."""

    def __init__(self, gp, prob, newton_rtol=1e-9, newton_max=12, tag=None):
        self.gp, self.prob, self.tag = gp, prob, tag
        self.rtol, self.nmax = newton_rtol, newton_max
        self.k, self.j, self.b0 = 1, 0, 0.0
        self.index = 0
        self.depth = 0.0                     # depth of the last accepted state
        self.trial = prob.depth_increment   # depth of the current attempt
        self.halvings = 0
        self.saved = None
        self.rho0 = prob.material.rho
        self.rho = self.rho0

    def _save(self):
        self.saved = [t.clone() for t in self.gp.get_state()[:3]]
        dd = abs(self.trial - self.depth)
        f = dd / self.prob.depth_increment
        rho = self.rho0 / f if 0 < f < 1 else self.rho0
        if rho != self.rho:
            self.gp.set_viscosity(rho)
            self.rho = rho

    def _fail(self):
        u, e, en = self.saved
        self.gp.set_state(u, e, en, self.depth)
        self.halvings += 1
        if self.halvings > 8:
            raise RuntimeError(f"load step {self.k}: Newton failed after 8 halvings")
        self.trial = self.depth + 0.5 * (self.trial - self.depth)
        self.j = 0

    def iteration(self):
        from paper_2011_08802_amd import mvpf
        gp = self.gp
        if self.j == 0:
            self._save()
        depth = self.trial
        rec = dict(index=self.index, load_step=self.k, depth=round(depth, 8), newton=self.j)
        t0 = time.perf_counter()
        try:
            gp.newton_system(depth)
        except mvpf.MvpfError as err:
            if err.code != -4:  # MVPF_ESINGULAR: the attempt fails
                raise
            self._fail()
            self.index += 1
            rec.update(system_ms=1e3 * (time.perf_counter() - t0), solve_ms=0.0, fgmres=0, rel_residual=float("nan"),
                       solve_converged=False, newton_rel_residual=float("nan"), attempt="singular block: halved",
                       iteration_ms=1e3 * (time.perf_counter() - t0))
            return rec
        t1 = time.perf_counter()
        if self.j == 0:
            self.b0 = float(torch.linalg.norm(gp.get_rhs()))
        _, st = gp.solve(want_x=False)
        gp.newton_update()
        _, rfree = gp.residual()
        t2 = time.perf_counter()
        rec.update(system_ms=1e3 * (t1 - t0), solve_ms=st.solve_ms, fgmres=st.iterations,
                   rel_residual=st.rel_residual, solve_converged=bool(st.converged),
                   newton_rel_residual=rfree / self.b0 if self.b0 else float("nan"))
        self.index += 1
        if np.isfinite(rfree) and rfree <= self.rtol * self.b0:
            _, e, _, _ = gp.get_state()
            gp.set_state(None, None, e, depth)
            self.depth = depth
            rec["attempt"] = "accepted"
            self.j = 0
            goal = self.k * self.prob.depth_increment
            if depth == goal:
                self.k += 1
                self.halvings = 0
                self.trial = self.k * self.prob.depth_increment
            else:
                self.trial = goal
        elif not np.isfinite(rfree) or self.j + 1 >= self.nmax:
            self._fail()
            rec["attempt"] = "failed: halved"
        else:
            self.j += 1
        rec["iteration_ms"] = 1e3 * (time.perf_counter() - t0)
        if self.tag:
            log(f"[{self.tag}] it {rec['index']}: load step {rec['load_step']} depth {rec['depth']:.5f} newton "
                f"{rec['newton']} fgmres {rec['fgmres']} solve {rec['solve_ms']:.1f} ms, newton residual "
                f"{rec['newton_rel_residual']:.2e} {rec.get('attempt', '')}")
        return rec


def run_sequence(prob, precision, warmup, steps, timing, tune=True, matrix_free=-1, snapshot_at=None, tag=None,
                 coarse="galerkin", **solver):
    """W untimed + K timed Newton iterations of the workload's load-step
    sequence from the seeded initial state.  Before it (untimed): launch
    shapes autotuned on the first Newton system and that system's solution
    kept for the error statement.  snapshot_at = n <= W keeps (u, eta) after
    the first n iterations (taken in the warm-up, outside the timed region)."""
    from paper_2011_08802_amd import mvpf
    gp = mvpf.Problem(prob, precision, rtol=1e-8, coarse=coarse, **solver)
    try:
        if matrix_free >= 0:
            gp.set_tuning("matrix_free", 0, matrix_free)
        gp.init_random(prob.seed)
        u0, e0, en0, _ = gp.get_state()
        u0, e0, en0 = u0.clone(), e0.clone(), en0.clone()
        gp.newton_system(prob.depth_increment)
        shapes = gp.autotune() if tune else None
        gp.newton_system(prob.depth_increment)
        x1, st1 = gp.solve()
        gp.set_state(u0, e0, en0, 0.0)
        del u0, e0, en0
        run = NewtonRun(gp, prob, tag=tag)
        recs, snap = [], None
        for _ in range(warmup):
            recs.append(run.iteration())
            if snapshot_at is not None and run.index == snapshot_at:
                snap = [t.clone() for t in gp.get_state()[:2]]
        if timing:
            gp.kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            recs.append(run.iteration())
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        kstats = {}
        if timing:
            for name in ("pbj_sweep", "residual", "spmv_outer"):
                n, ms, by = gp.kernel_stats(name)
                if n:
                    kstats[name] = dict(launches=n, avg_ms=ms / n, bytes=by, gbs=by / (ms / n) / 1e6)
            gp.kernel_timing(False)
        mf = gp.get_tuning("matrix_free")
    finally:
        gp.close()
    for r in recs[:warmup]:
        r["timed"] = False
    for r in recs[warmup:]:
        r["timed"] = True
    return dict(total_s=total, recs=recs, kernels=kstats, x1=x1, first_its=st1.iterations, shapes=shapes,
                matrix_free=mf, snapshot=snap)


def multistep(prob, precision, budget_s=120.0, coarse="galerkin"):
    """The workload's whole run: every load step to convergence, every Newton
    solve listed (untimed as a whole; each solve's own time is recorded).
    Stops after budget_s seconds of wall time (then 'completed' is false)."""
    from paper_2011_08802_amd import mvpf
    gp = mvpf.Problem(prob, precision, rtol=1e-8, coarse=coarse)
    try:
        gp.init_random(prob.seed)
        gp.newton_system(prob.depth_increment)
        gp.autotune()
        gp.init_random(prob.seed)
        run = NewtonRun(gp, prob, tag=f"64^3 {precision}")
        recs = []
        t0 = time.perf_counter()
        while run.k <= prob.steps and len(recs) < 400 and time.perf_counter() - t0 < budget_s:
            recs.append(run.iteration())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gp.close()
    keep = ("load_step", "depth", "newton", "fgmres", "solve_ms", "system_ms", "rel_residual", "newton_rel_residual")
    return dict(load_steps=prob.steps, completed=run.k > prob.steps, load_steps_done=run.k - 1,
                budget_s=budget_s, depth_increment=prob.depth_increment, newton_iterations=len(recs),
                fgmres_iterations=sum(r["fgmres"] for r in recs),
                solve_ms=sum(r["solve_ms"] for r in recs), wall_s=wall,
                failed_attempts=sum(1 for r in recs if r.get("attempt", "").startswith(("failed", "singular"))),
                solves=[{k: (round(r[k], 4) if isinstance(r[k], float) and k.endswith("ms") else r[k])
                         for k in keep} for r in recs])


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
    # once martensite forms the systems are much harder than the patch workload's.  Rediscretised
    # coarse levels: V(4,4) with damping 0.4 and FGMRES(60) take the whole run from 125 s (V(3,3),
    # 0.5, FGMRES(30)) to 80 s.  Galerkin coarse levels: the default V(2,2), 0.55, FGMRES(30) takes
    # 51 s, V(4,4), 0.4, FGMRES(60) 62 s.
    gal = a.coarse == "galerkin"
    nu = a.sweeps if a.sweeps > 0 else (2 if gal else 4)
    sweeps = dict(nu_pre=nu, nu_post=nu, omega=a.omega if a.omega > 0 else (0.55 if gal else 0.4),
                  restart=a.restart if a.restart > 0 else (30 if gal else 60))
    log(f"[bench] indentation workload: {prob.nx}x{prob.ny}x{prob.nz}, {ndof} dof, run {run}, smoother {sweeps}")
    res = {}
    for prec in ("mixed",) + (() if a.no_fp64 else ("fp64",)):
        gp = mvpf.Problem(prob, prec, rtol=1e-8, coarse=a.coarse, **sweeps)
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
                               f"V({nu},{nu}) damping {sweeps['omega']}, FGMRES({sweeps['restart']}) rtol 1e-8; "
                               f"a step = one whole "
                               f"run; value = dof x Newton iterations per second", "precision": "mixed",
                   "levels": prob.n_levels, "coarse": a.coarse, **run},
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


def sweep_traffic(workload, prob, matrix_free):
    """Measured HBM bytes of one finest-level smoother sweep from the committed
    counter summary of this workload (None if there is none).  Assembled:
    pass 1 on two wavefronts per tile + pass 2; matrix-free: the element
    kernel + the gather with the Jacobi update.  Rows are matched by kernel
    name and grid size (the finest level's launch)."""
    path = COUNTERS.get(workload)
    if path is None or not os.path.exists(path):
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
    with open(path) as f:
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_newton(p, threads, reference, coarse="galerkin"):
    """The oracle (test infrastructure) on one Newton iteration of problem p
    from its seeded initial state: autodiff assembly of the residual and
    tangent on every level + multigrid setup, then FGMRES+GMG to 1e-8 (timed).
    reference: 'direct' (the plain definition, sparse LU) or 'fgmres' (the
    oracle's own FGMRES+GMG at rtol 1e-12), untimed."""
    from oracle import solver as S
    from oracle.fem import Mesh, NDOF
    from oracle.material import Card
    torch.set_num_threads(threads)
    card = Card(p.material)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    mask, target = S.dirichlet(m, p.kind, p.patch, p.radius, depth=p.depth_increment)
    t0 = time.perf_counter()
    sysk = S.NewtonSystem(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, S.increment(mask, target, U),
                          p.depth_increment)
    mg = S.Multigrid(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, K_fine=sysk.K, depth=p.depth_increment,
                     coarse="galerkin" if coarse == "galerkin" else "reassemble")
    t1 = time.perf_counter()
    x, st = S.fgmres(sysk.A, sysk.b, mg.precondition, rtol=1e-8)
    t2 = time.perf_counter()
    if reference == "direct":
        xref = S.direct_solve(sysk.A, sysk.b)
    else:
        xref, _ = S.fgmres(sysk.A, sysk.b, mg.precondition, rtol=1e-12)
    return dict(assembly_s=t1 - t0, solve_s=t2 - t1, iterations=st.iterations, x=x, xref=xref)


def gpu_errors(p, xref, coarse="galerkin"):
    """GPU solves (mixed and FP64 multigrid, rtol 1e-8) of the same first
    Newton system; relative error of each against the oracle's reference."""
    from paper_2011_08802_amd import mvpf
    out = {}
    for prec in ("mixed", "fp64"):
        gp = mvpf.Problem(p, prec, rtol=1e-8, coarse=coarse)
        try:
            gp.init_random(p.seed)
            gp.newton_system(p.depth_increment)
            x, st = gp.solve()
            xg = x.cpu().numpy()
        finally:
            gp.close()
        out[prec] = dict(rel_error=float(np.linalg.norm(xg - xref) / np.linalg.norm(xref)),
                         fgmres_iterations=st.iterations)
    return out


def cpu_baseline(sample, coarse="galerkin"):
    """The oracle on the host cores: the whole 8^3 workload (all threads and
    one thread) and a bounded sample of the benchmarked workload; value = the
    sample's DOF per second of one Newton iteration (assembly + solve)."""
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or (os.cpu_count() or 1)
    tiny = synth.tiny()
    log(f"[bench] oracle: whole 8^3 workload, {threads} threads")
    a = oracle_newton(tiny, threads, "direct", coarse)
    log("[bench] oracle: whole 8^3 workload, 1 thread")
    a1 = oracle_newton(tiny, 1, "direct", coarse)
    err_tiny = gpu_errors(tiny, a["xref"], coarse)
    log(f"[bench] oracle: sample {sample.nx}x{sample.ny}x{sample.nz}, {threads} threads")
    b = oracle_newton(sample, threads, "fgmres", coarse)
    err_sample = gpu_errors(sample, b["xref"], coarse)
    torch.set_num_threads(threads)
    step_s = b["assembly_s"] + b["solve_s"]
    return dict(
        value=sample.n_dof / step_s, unit="DOF/s", cores=threads, kind="oracle",
        sample=(f"one Newton iteration (autodiff assembly on all {sample.n_levels} levels + multigrid setup "
                f"{b['assembly_s']:.1f} s, FGMRES+GMG to 1e-8 {b['solve_s']:.1f} s, {b['iterations']} its) "
                f"of the same {sample.kind} indentation at {sample.nx}x{sample.ny}x{sample.nz} elements "
                f"({sample.n_dof} dof): the benchmarked workload's geometry and loading on a coarser mesh"),
        solve_dof_per_s=sample.n_dof / b["solve_s"],
        os_cpu_count=os.cpu_count(), cpu_model=cpu_model(),
        threads_note="the box allots OMP_NUM_THREADS host threads per GPU; os_cpu_count is the host's total",
        whole_8cubed={"dof": tiny.n_dof, "threads": threads, "newton_step_s": a["assembly_s"] + a["solve_s"],
                      "solve_s": a["solve_s"], "iterations": a["iterations"],
                      "one_thread_newton_step_s": a1["assembly_s"] + a1["solve_s"],
                      "one_thread_solve_s": a1["solve_s"],
                      "gpu_error_vs_oracle_direct_solve": err_tiny},
        sample_gpu_error_vs_oracle_fgmres_rtol12=err_sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scale", choices=list(WORKLOADS) + ["batched", "indent"])
    ap.add_argument("--fp64-steps", type=int, default=5,
                    help="timed Newton iterations of the FP64-multigrid comparison (after the same warm-up)")
    ap.add_argument("--no-multistep", action="store_true", help="skip the whole 64^3 run")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-multigrid comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes (no autotuning)")
    ap.add_argument("--no-pade", action="store_true", help="skip the assembly cost per Pade order")
    ap.add_argument("--matrix-free", type=int, default=-1,
                    help="finest level applied from its Gauss-point Hessians (1) or assembled (0); -1: the default")
    ap.add_argument("--sweeps", type=int, default=0,
                    help="pre- and post-smoothing sweeps (default: 2; indentation workload 4)")
    ap.add_argument("--levels", type=int, default=0, help="multigrid levels (default: the workload's)")
    ap.add_argument("--pre", type=int, default=-1, help="pre-smoothing sweeps (overrides --sweeps)")
    ap.add_argument("--post", type=int, default=-1, help="post-smoothing sweeps (overrides --sweeps)")
    ap.add_argument("--omega", type=float, default=0.0, help="smoother damping (default 0.55)")
    ap.add_argument("--restart", type=int, default=0,
                    help="FGMRES restart length (default: 30; indentation workload 60)")
    ap.add_argument("--indent-depth", type=float, default=0.0,
                    help="indentation workload: maximum depth (default: the workload's 0.03)")
    ap.add_argument("--coarse", default="galerkin", choices=["galerkin", "rediscretise"],
                    help="coarse multigrid operators: Galerkin products of the finest tangent (default) or the "
                         "paper's rediscretisation at the injected state")
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
    single_main(a)


SAMPLES = {  # bounded samples of each workload for the oracle (about 10-20 s of oracle work)
    "tiny": lambda p: p,
    "medium": lambda p: synth.Problem(16, 16, 16, n_levels=3, patch=2, depth_increment=p.depth_increment),
    "large": lambda p: synth.Problem(16, 16, 16, n_levels=3, patch=2, depth_increment=p.depth_increment),
    "scale": lambda p: synth.Problem(24, 24, 12, lz=0.5, n_levels=3, kind="cap", radius=p.radius,
                                     depth_increment=p.depth_increment),
}


def single_main(a):
    prob = WORKLOADS[a.workload]()
    if a.levels > 0:
        prob = dataclasses.replace(prob, n_levels=a.levels)
    ndof = prob.n_dof
    W, K = a.warmup, a.steps
    log(f"[bench] workload {a.workload}: {prob.nx}x{prob.ny}x{prob.nz}, {ndof} dof, {prob.n_levels} levels; "
        f"{W} + {K} Newton iterations of the load-step sequence")
    log("[bench] mixed (FP32 multigrid) ...")
    solver = {}
    if a.sweeps > 0:
        solver.update(nu_pre=a.sweeps, nu_post=a.sweeps)
    if a.restart > 0:
        solver.update(restart=a.restart)
    if a.pre >= 0:
        solver.update(nu_pre=a.pre)
    if a.post >= 0:
        solver.update(nu_post=a.post)
    if a.omega > 0:
        solver.update(omega=a.omega)
    nu, nu2, restart = solver.get("nu_pre", 2), solver.get("nu_post", 2), solver.get("restart", 30)
    mixed = run_sequence(prob, "mixed", W, K, not a.no_timing, not a.no_tune, a.matrix_free, snapshot_at=W,
                         tag="mixed", coarse=a.coarse, **solver)
    x1m = mixed.pop("x1")
    log(f"[bench] mixed: {ndof * K / mixed['total_s']:.4g} DOF/s, {1e3 * mixed['total_s'] / K:.1f} ms per Newton "
        f"iteration; sweep {mixed['kernels'].get('pbj_sweep')}")
    fp64 = None
    if not a.no_fp64:
        kf = min(K, a.fp64_steps)
        log(f"[bench] fp64 multigrid: {W} + {kf} Newton iterations of the same sequence ...")
        fp64 = run_sequence(prob, "fp64", W, kf, False, not a.no_tune, a.matrix_free, snapshot_at=W, tag="fp64",
                            coarse=a.coarse, **solver)
        x1f = fp64.pop("x1")

    def summary(r):
        recs = [x for x in r["recs"] if x["timed"]]
        return dict(ms_per_step=1e3 * r["total_s"] / len(recs),
                    solve_ms_median=statistics.median(x["solve_ms"] for x in recs),
                    solve_dof_per_s=ndof * len(recs) / (1e-3 * sum(x["solve_ms"] for x in recs)),
                    system_ms_median=statistics.median(x["system_ms"] for x in recs),
                    fgmres_iterations=[x["fgmres"] for x in recs],
                    rel_residual_max=max(x["rel_residual"] for x in recs),
                    converged=all(x["solve_converged"] for x in recs),
                    load_steps_touched=sorted({x["load_step"] for x in recs}))

    ms = summary(mixed)
    ms["launch_shapes"] = mixed["shapes"]
    ms["matrix_free"] = mixed["matrix_free"]
    keep = ("index", "load_step", "depth", "newton", "fgmres", "solve_ms", "system_ms", "iteration_ms",
            "rel_residual", "newton_rel_residual", "timed")
    out = {
        "metric": METRIC,
        "value": ndof * K / mixed["total_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{'patch' if prob.kind == 'patch' else 'spherical-cap'} indentation "
                               f"{prob.nx}x{prob.ny}x{prob.nz} Q1 hex ({prob.lx:g}x{prob.ly:g}x{prob.lz:g}), "
                               f"{ndof} dof, {prob.n_levels}-level GMG V({nu},{nu2}) damping {solver.get('omega', 0.55)} "
                               f"({a.coarse} coarse operators), "
                               f"FGMRES({restart}) rtol 1e-8; "
                               f"{prob.steps} load steps of {prob.depth_increment}; a step = one Newton "
                               f"iteration of the running load-step sequence (Newton rtol 1e-9), iterations "
                               f"{W}..{W + K - 1} timed",
                   "nx": prob.nx, "ny": prob.ny, "nz": prob.nz, "levels": prob.n_levels,
                   "load": prob.kind, "depth_increment": prob.depth_increment, "load_steps": prob.steps,
                   "seed": prob.seed, "precision": "mixed", "coarse": a.coarse},
        "mixed": ms,
        "newton_iterations": [{k: (round(r[k], 4) if isinstance(r[k], float) and k.endswith("ms") else r[k])
                               for k in keep} for r in mixed["recs"]],
    }
    if fp64 is not None:
        fs = summary(fp64)
        fs["launch_shapes"] = fp64["shapes"]
        fs["value"] = ndof * len([x for x in fp64["recs"] if x["timed"]]) / fp64["total_s"]
        fs["fgmres_iterations_all"] = [x["fgmres"] for x in fp64["recs"]]
        out["fp64_gmg"] = fs
        # the same Newton systems (same position in the sequence), warm-up included but the first
        common = range(1, min(len(mixed["recs"]), len(fp64["recs"])))
        sm = [mixed["recs"][i]["solve_ms"] for i in common]
        sf = [fp64["recs"][i]["solve_ms"] for i in common]
        out["speedup_solve_mixed_vs_fp64"] = statistics.median(f / m for f, m in zip(sf, sm))
        out["speedup_solve_mixed_vs_fp64_basis"] = f"median over Newton iterations 1..{len(sm)} of the sequence"
        d1 = float(torch.linalg.norm(x1m - x1f) / torch.linalg.norm(x1f))
        err = {"first_newton_system_solution_rel_diff": d1}
        if mixed["snapshot"] is not None and fp64["snapshot"] is not None:
            (um, em), (uf, ef) = mixed["snapshot"], fp64["snapshot"]
            err[f"state_after_{W}_newton_iterations_rel_diff"] = {
                "u": float(torch.linalg.norm(um - uf) / torch.linalg.norm(uf)),
                "eta": float(torch.linalg.norm(em - ef) / torch.linalg.norm(ef))}
        out["error_vs_fp64_gpu"] = err
    del x1m
    if fp64 is not None:
        del x1f
    mixed["snapshot"] = None
    if fp64 is not None:
        fp64["snapshot"] = None
    torch.cuda.empty_cache()
    out["error_vs_oracle"] = ("not computed at this size (the oracle's autodiff assembly would take hours); "
                              "see cpu_baseline: GPU error vs the oracle on the whole 8^3 workload and on the "
                              "sample" if a.workload != "tiny" else "see cpu_baseline")
    k = mixed["kernels"].get("pbj_sweep")
    if k:
        mf = mixed["matrix_free"]
        out["roofline"] = {"bound": "hbm", "achieved": k["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": k["gbs"] / HBM_PEAK_GBS, "traffic": sweep_traffic(a.workload, prob, mf),
                           "kernel": "finest-level FP32 smoother sweep "
                                     + ("(matrix-free: mf_element + mf_gather<2>)" if mf
                                        else "(defect_upper_split + pbj_lower)"),
                           "bytes_per_launch": k["bytes"], "avg_ms": k["avg_ms"], "launches": k["launches"]}
        out["kernels"] = mixed["kernels"]
    if not a.no_multistep and a.workload != "medium":
        med = synth.medium()
        out["multistep_64cubed"] = {}
        for prec in ("fp64", "mixed"):
            log(f"[bench] whole 64^3 run ({med.steps} load steps of {med.depth_increment}), {prec} ...")
            try:
                out["multistep_64cubed"][prec] = multistep(med, prec, coarse=a.coarse)
            except Exception as err:  # reported, not fatal for the headline
                out["multistep_64cubed"][prec] = {"error": str(err)}
    if not a.no_pade and a.workload in ("tiny", "medium"):
        log("[bench] assembly per Pade order ...")
        out["pade_assembly"] = pade_assembly(prob)
    if not a.no_cpu_baseline:
        log("[bench] oracle cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(SAMPLES[a.workload](prob), a.coarse)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
