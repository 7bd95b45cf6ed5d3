"""GPU (HIP, through the C ABI) vs the CPU oracle, element by element.

Tolerances: FP64 operators (residual, right-hand side, K x on every level,
V-cycle) <= 1e-12 relative unless stated (double rounding of differently
ordered sums); FP32 operators <= 2e-6 relative; solves at rtol 1e-12 match
the oracle's direct solve to <= 1e-9 relative."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import OracleCase, abs_product, check_entries, gpu_problem, rel, rel_blocks, say, seeded_state
from oracle import solver as S
from oracle.fem import Discretisation, Mesh, NDOF
from oracle.material import Card

pytestmark = pytest.mark.gpu

CASES = {
    # 8^3 unit cube, 2x2 patch, 3 levels (the tiny workload), reference state
    "tiny": (synth.tiny(), 0.0),
    # ragged: 585 nodes (not a multiple of 64), non-cubic box, perturbed state
    "ragged": (synth.Problem(8, 12, 4, ly=1.5, lz=0.5, n_levels=3, patch=2, depth_increment=0.01), 2e-3),
    # smallest: 2^3 elements, 2 levels (coarsest is one element)
    "minimal": (synth.Problem(2, 2, 2, n_levels=2, patch=2, depth_increment=0.05), 1e-3),
    # spherical-cap indenter (R = 0.2) on a 1 x 1 x 0.5 box, the shape of the
    # 256x256x128 workload: 5 top nodes in contact
    "cap": (synth.Problem(16, 16, 8, lz=0.5, n_levels=3, kind="cap", radius=0.2, depth_increment=0.02), 1e-3),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    p, amp = CASES[request.param]
    U, En = seeded_state(p, amp)
    say(f"[case {request.param}] oracle setup nx={p.nx} ny={p.ny} nz={p.nz} L={p.n_levels}")
    oc = OracleCase(p, U, En, p.depth_increment)
    say(f"[case {request.param}] GPU setup")
    gp = gpu_problem(p, U, En, "fp64")
    # this handle exercises the large-grid row kernels on every level; the
    # mixed-precision handles below use the default small-grid kernels
    gp.set_tuning("small_grid_nodes", 0, 0)
    gp.newton_system(p.depth_increment)
    yield request.param, p, U, En, oc, gp
    gp.close()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def test_init_random_matches_generator():
    p = synth.tiny()
    from paper_2011_08802_amd import mvpf
    gp = mvpf.Problem(p)
    gp.init_random(p.seed)
    u, e, en, d = gp.get_state()
    assert torch.count_nonzero(u) == 0 and d == 0.0
    assert np.array_equal(e.cpu().numpy(), p.eta0())
    assert np.array_equal(en.cpu().numpy(), p.eta0())
    gp.close()


def test_residual_parity(case):
    name, p, U, En, oc, gp = case
    say(f"[{name}] residual")
    R, nf = gp.residual()
    Ro = oc.sys.R
    check_entries(R.cpu().numpy(), Ro, 1e-12, "residual", oc.abs_scales()[0])
    free = ~oc.mask.ravel()
    assert abs(nf - np.linalg.norm(Ro[free])) <= 1e-12 * np.linalg.norm(Ro[free])


def test_rhs_parity(case):
    name, p, U, En, oc, gp = case
    say(f"[{name}] rhs")
    b = gp.get_rhs().cpu().numpy()
    check_entries(b, oc.sys.b, 1e-12, "rhs", oc.abs_scales()[1])


def test_operator_parity_all_levels(case):
    name, p, U, En, oc, gp = case
    rng = np.random.default_rng(3)
    for l, lev in enumerate(oc.mg.levels):
        say(f"[{name}] K x level {l}")
        x = rng.standard_normal(lev.A.shape[0])
        y = gp.jacobian_apply(l, _dev(x)).cpu().numpy()
        check_entries(y, lev.A @ x, 1e-12, f"K x level {l}", abs_product(lev.A, x))


def test_preconditioner_parity_fp64(case):
    name, p, U, En, oc, gp = case
    say(f"[{name}] V-cycle")
    v = np.random.default_rng(4).standard_normal(oc.sys.b.shape[0])
    z = gp.precondition(_dev(v)).cpu().numpy()
    zo = oc.mg.precondition(v)
    assert rel(z, zo) < 1e-10, rel(z, zo)


def test_fgmres_iterations_match_oracle(case):
    name, p, U, En, oc, gp = case
    say(f"[{name}] FGMRES rtol 1e-8")
    x, st = gp.solve()
    xo, sto = S.fgmres(oc.sys.A, oc.sys.b, oc.mg.precondition, rtol=1e-8)
    assert st.converged and sto.converged
    assert abs(st.iterations - sto.iterations) <= 1, (st.iterations, sto.iterations)
    assert st.rel_residual <= 1e-8
    # true residual of the GPU solution, evaluated by the oracle
    xr = x.cpu().numpy()
    assert np.linalg.norm(oc.sys.b - oc.sys.A @ xr) <= 1.0001e-8 * np.linalg.norm(oc.sys.b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_matches_direct(case, precision):
    name, p, U, En, oc, _ = case
    say(f"[{name}] solve {precision} rtol 1e-12")
    gp = gpu_problem(p, U, En, precision, rtol=1e-12)
    gp.newton_system(p.depth_increment)
    x, st = gp.solve()
    gp.close()
    assert st.converged and st.rel_residual <= 1e-12
    assert rel(x.cpu().numpy(), oc.x) <= 1e-9, rel(x.cpu().numpy(), oc.x)


def test_mixed_operators_fp32(case):
    name, p, U, En, oc, _ = case
    say(f"[{name}] mixed operators")
    from paper_2011_08802_amd import mvpf
    gp = gpu_problem(p, U, En, "mixed")
    gp.newton_system(p.depth_increment)
    rng = np.random.default_rng(5)
    for l, lev in enumerate(oc.mg.levels[:-1]):
        x = rng.standard_normal(lev.A.shape[0])
        y = gp.jacobian_apply(l, _dev(x), mvpf.MIXED).cpu().numpy()
        check_entries(y, lev.A @ x, 2e-6, f"FP32 K x level {l}", abs_product(lev.A, x))
    # the FP64 copy of the finest operator is exact
    x = rng.standard_normal(oc.sys.b.shape[0])
    y = gp.jacobian_apply(0, _dev(x), mvpf.FP64).cpu().numpy()
    check_entries(y, oc.sys.A @ x, 1e-12, "FP64 K x finest", abs_product(oc.sys.A, x))
    v = rng.standard_normal(oc.sys.b.shape[0])
    z = gp.precondition(_dev(v)).cpu().numpy()
    assert rel(z, oc.mg.precondition(v)) < 1e-4
    gp.close()


def test_zero_rhs_gives_zero_solution(case):
    name, p, U, En, oc, gp = case
    b = torch.zeros(oc.sys.b.shape[0], dtype=torch.float64, device="cuda")
    x, st = gp.solve(b)
    assert st.converged and st.iterations == 0 and torch.count_nonzero(x) == 0


def test_assembly_and_solve_are_deterministic():
    p = synth.tiny()
    U, En = seeded_state(p, 1e-3)
    say("[determinism] two runs")
    out = []
    for _ in range(2):
        gp = gpu_problem(p, U, En, "mixed")
        gp.newton_system(p.depth_increment)
        b = gp.get_rhs()
        x, st = gp.solve()
        out.append((b.cpu().numpy(), x.cpu().numpy(), st.iterations))
        gp.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_newton_time_step_matches_oracle():
    """One implicit step with Newton to 1e-11: GPU (FGMRES+GMG at 1e-12) vs the
    oracle's Newton with direct solves."""
    p = synth.Problem(4, 4, 4, n_levels=2, patch=2, depth_increment=0.02)
    U, En = seeded_state(p)
    say("[newton] oracle")
    card = Card(p.material)
    m = Mesh.from_problem(p)
    mask, target = S.dirichlet(m, "patch", p.patch, depth=p.depth_increment)
    Uo, it, ok = S.newton_step(p, card, U.ravel(), En.ravel(), mask, S.increment(mask, target, U), rtol=1e-11)
    assert ok
    say("[newton] GPU time step")
    for prec in ("fp64", "mixed"):
        gp = gpu_problem(p, U, En, prec, rtol=1e-12, newton_rtol=1e-11)
        st = gp.time_step(p.depth_increment)
        assert st.converged and st.halvings == 0
        assert abs(st.newton_iterations - it) <= 1, (st.newton_iterations, it)
        u, e, en, d = gp.get_state()
        Ug = np.concatenate([u.cpu().numpy(), e.cpu().numpy()], 1)
        assert rel(Ug, Uo) <= 1e-9, rel(Ug, Uo)
        assert np.array_equal(e.cpu().numpy(), en.cpu().numpy()) and d == p.depth_increment
        gp.close()


def test_launch_shape_does_not_change_results():
    """Persistent launch shapes of the operator kernels (tuning knobs and the
    autotuner) leave every result bitwise unchanged."""
    p = synth.tiny()
    U, En = seeded_state(p, 1e-3)
    say("[launch shape] default vs minimal grids vs small matrix-free workgroups vs autotuned")
    outs = []
    for mode in ("default", "minimal", "mf8", "autotune"):
        gp = gpu_problem(p, U, En, "mixed")
        gp.newton_system(p.depth_increment)
        if mode == "minimal":
            for l in range(p.n_levels):
                gp.set_tuning("row_blocks", l, 8)
            gp.set_tuning("outer_blocks", 0, 8)
            assert gp.get_tuning("row_blocks", 0) == 8
        elif mode == "mf8":
            gp.set_tuning("mf_elements_per_block", 0, 8)
            assert gp.get_tuning("mf_elements_per_block") == 8
        elif mode == "autotune":
            shapes = gp.autotune()
            assert len(shapes) == p.n_levels
        x, st = gp.solve()
        outs.append((x.cpu().numpy(), st.iterations))
        gp.close()
    for x, its in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and its == outs[0][1]


def test_sixteen_cubed_coarse_1125():
    """16^3 with 3 levels: the coarsest level has 1125 unknowns, as in the
    64^3 workload (panel factorisation with 3 rows per thread).  Operators on
    every level, V-cycle (both row-kernel families) and FGMRES."""
    p = synth.Problem(16, 16, 16, n_levels=3, patch=4, depth_increment=0.01)
    U, En = seeded_state(p, 5e-4)
    say("[16^3] oracle")
    oc = OracleCase(p, U, En, p.depth_increment, direct=False)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(oc.sys.b.shape[0])
    zo = oc.mg.precondition(v)
    xo, sto = S.fgmres(oc.sys.A, oc.sys.b, oc.mg.precondition, rtol=1e-12)
    for small in (0, 40000):
        say(f"[16^3] GPU small_grid_nodes={small}")
        gp = gpu_problem(p, U, En, "fp64", rtol=1e-12)
        gp.set_tuning("small_grid_nodes", 0, small)
        gp.newton_system(p.depth_increment)
        b = gp.get_rhs().cpu().numpy()
        check_entries(b, oc.sys.b, 1e-12, "rhs", oc.abs_scales()[1])
        for l, lev in enumerate(oc.mg.levels):
            x = rng.standard_normal(lev.A.shape[0])
            check_entries(gp.jacobian_apply(l, _dev(x)).cpu().numpy(), lev.A @ x, 1e-12, f"K x level {l}",
                          abs_product(lev.A, x))
        z = gp.precondition(_dev(v)).cpu().numpy()
        assert rel(z, zo) < 1e-10, rel(z, zo)
        x, st = gp.solve()
        assert st.converged and abs(st.iterations - sto.iterations) <= 1, (st.iterations, sto.iterations)
        assert rel(x.cpu().numpy(), xo) < 1e-9
        gp.close()


@pytest.mark.parametrize("n,levels,coarse_dof", [(12, 2, 3087), (16, 2, 6561)])
def test_large_coarse_inverse(n, levels, coarse_dof):
    """Two-level hierarchies whose coarsest level is large (6^3 and 8^3
    elements, the latter the size of the 128^3 workload's coarsest level):
    blocked Gauss-Jordan with several outer panels and narrow sub-panels.
    Coarse operator, V-cycle and FGMRES solve vs the oracle."""
    p = synth.Problem(n, n, n, n_levels=levels, patch=4, depth_increment=0.01)
    _coarse_case(p, levels, coarse_dof, f"{n}^3 L{levels}")


@pytest.mark.parametrize("nx,ny,nz,coarse_dof", [(6, 8, 10, 1080), (6, 10, 10, 1296)])
def test_coarse_panel_variants(nx, ny, nz, coarse_dof):
    """Two-level hierarchies on box meshes whose coarsest level has 1 080
    unknowns (sub-panels factored by 256 threads holding 5 rows each, the
    variant for 1 025 to 1 280 unknowns) or 1 296 unknowns (512 threads
    holding 3 rows each): coarse operator, V-cycle and FGMRES solve vs the
    oracle."""
    h = 1.0 / max(nx, ny, nz)
    p = synth.Problem(nx, ny, nz, lx=nx * h, ly=ny * h, lz=nz * h, n_levels=2, patch=4, depth_increment=0.01)
    _coarse_case(p, 2, coarse_dof, f"{nx}x{ny}x{nz} L2")


def _coarse_case(p, levels, coarse_dof, tag):
    U, En = seeded_state(p, 5e-4)
    say(f"[{tag}] oracle (coarse {coarse_dof} dof)")
    oc = OracleCase(p, U, En, p.depth_increment, direct=False)
    assert oc.mg.levels[-1].A.shape[0] == coarse_dof
    rng = np.random.default_rng(7)
    v = rng.standard_normal(oc.sys.b.shape[0])
    zo = oc.mg.precondition(v)
    xo, sto = S.fgmres(oc.sys.A, oc.sys.b, oc.mg.precondition, rtol=1e-12)
    say(f"[{tag}] GPU")
    gp = gpu_problem(p, U, En, "fp64", rtol=1e-12)
    gp.newton_system(p.depth_increment)
    x = rng.standard_normal(coarse_dof)
    yc = gp.jacobian_apply(levels - 1, _dev(x)).cpu().numpy()
    Ac = oc.mg.levels[-1].A
    check_entries(yc, Ac @ x, 1e-12, "coarse K x", abs_product(Ac, x))
    z = gp.precondition(_dev(v)).cpu().numpy()
    assert rel(z, zo) < 1e-10, rel(z, zo)
    xs, st = gp.solve()
    assert st.converged and abs(st.iterations - sto.iterations) <= 1, (st.iterations, sto.iterations)
    assert rel(xs.cpu().numpy(), xo) < 1e-9
    gp.close()


def test_assembly_slabs_bitwise():
    """Assembly in slabs of element layers (one halo layer recomputed per
    slab) gives bitwise the same residual, Newton system and solution as the
    whole-level assembly."""
    p = synth.tiny()
    U, En = seeded_state(p, 1e-3)
    rng = np.random.default_rng(8)
    xs = None
    outs = []
    for slab in (0, 192, 256):  # whole level; 1 and 2 node layers per slab on 8^3
        say(f"[slabs] assembly_slab_elements={slab}")
        gp = gpu_problem(p, U, En, "mixed")
        if slab:
            gp.set_tuning("assembly_slab_elements", 0, slab)
            assert gp.get_tuning("assembly_slab_elements") == slab
        R, nf = gp.residual()
        gp.newton_system(p.depth_increment)
        b = gp.get_rhs()
        info = gp.info()
        if xs is None:
            xs = [rng.standard_normal(9 * info.n_nodes[l]) for l in range(p.n_levels)]
        from paper_2011_08802_amd import mvpf
        ys = [gp.jacobian_apply(l, _dev(xs[l]), mvpf.FP64 if l in (0, p.n_levels - 1) else mvpf.MIXED).cpu().numpy()
              for l in range(p.n_levels)]
        x, st = gp.solve()
        outs.append((R.cpu().numpy(), nf, b.cpu().numpy(), ys, x.cpu().numpy(), st.iterations))
        gp.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1] == outs[0][1]
        assert np.array_equal(o[2], outs[0][2])
        for y, y0 in zip(o[3], outs[0][3]):
            assert np.array_equal(y, y0)
        assert np.array_equal(o[4], outs[0][4]) and o[5] == outs[0][5]


def test_time_step_failure_restores_state():
    """Newton failure handling, forced from the host through the options (one
    Newton iteration allowed, unreachable tolerance): every attempt fails, the
    increment is halved 8 times, the call reports non-convergence and the
    state and depth are exactly those before the call."""
    from paper_2011_08802_amd import mvpf
    p = synth.tiny()
    U, En = seeded_state(p, 1e-3)
    gp = gpu_problem(p, U, En, "mixed", newton_max=1, newton_rtol=1e-30)
    before = gp.get_state()
    st = gp.time_step(p.depth_increment)
    after = gp.get_state()
    assert not st.converged and st.halvings == 9 and st.newton_iterations == 9
    for a, b in zip(before[:3], after[:3]):
        assert torch.equal(a, b)
    assert after[3] == before[3] == 0.0
    # the problem stays usable: a normal step from the restored state converges
    gp.set_opts(newton_max=12, newton_rtol=1e-9)
    st = gp.time_step(p.depth_increment)
    assert st.converged and st.halvings == 0
    gp.close()


def test_set_viscosity_and_time_step_restores_it():
    """mvpf_set_viscosity: the residual with another rho = 1/(m tau) (Sec. 2.3)
    matches the oracle's with that rho entry by entry, and setting the
    material's rho back reproduces the first residual bitwise.  A time step
    whose attempts all fail (forced from the host: one Newton iteration,
    unreachable tolerance) runs its halved attempts with 2^k rho and returns
    with the state, the depth and the material's rho exactly as before."""
    from dataclasses import replace
    p = synth.tiny()
    U, En = seeded_state(p, 1e-3)
    En = 0.5 * En  # eta_hat != eta_hat_n: the viscous term is not zero
    say("[viscosity] tiny, rho 3.7 vs the oracle")
    gp = gpu_problem(p, U, En, "mixed")
    R0, nf0 = gp.residual()
    R0 = R0.cpu().numpy()
    gp.set_viscosity(3.7)
    R1, _ = gp.residual()
    p1 = replace(p, material=replace(p.material, rho=3.7))
    oc = OracleCase(p1, U, En, 0.0, build_mg=False, direct=False)
    check_entries(R1.cpu().numpy(), oc.sys.R, 1e-12, "residual at rho 3.7", oc.abs_scales()[0])
    assert not np.array_equal(R1.cpu().numpy(), R0)
    gp.set_viscosity(p.material.rho)
    R2, nf2 = gp.residual()
    assert np.array_equal(R2.cpu().numpy(), R0) and nf2 == nf0
    with pytest.raises(RuntimeError, match="rho must be finite"):
        gp.set_viscosity(float("nan"))
    say("[viscosity] failing time step")
    gp.set_opts(newton_max=1, newton_rtol=1e-30)
    before = gp.get_state()
    st = gp.time_step(p.depth_increment)
    after = gp.get_state()
    assert not st.converged and st.halvings == 9 and st.newton_iterations == 9
    for a, b in zip(before[:3], after[:3]):
        assert torch.equal(a, b)
    assert after[3] == before[3] == 0.0
    R3, nf3 = gp.residual()
    assert np.array_equal(R3.cpu().numpy(), R0) and nf3 == nf0
    gp.close()


def test_time_step_singular_setup_restores_state():
    """A singular 9x9 diagonal block ends a Newton attempt like a failed one
    (Sec. 3.4: the increment is halved), and the state is restored.  The
    singular blocks are forced from the host by a material card with zero
    stiffness: the displacement rows of every free node's diagonal block are
    then exactly zero.  Every attempt fails at its first solver setup, the
    increment is halved 8 times, the call reports non-convergence, and the
    state and depth are bitwise those before the call."""
    from dataclasses import replace
    from paper_2011_08802_amd import mvpf
    p = synth.tiny()
    p = replace(p, material=replace(p.material, cubic=(0.0, 0.0, 0.0), ortho=(0.0,) * 9))
    U, En = seeded_state(p, 1e-3)
    say("[singular setup] zero-stiffness card, time step")
    gp = gpu_problem(p, U, En, "mixed")
    before = gp.get_state()
    st = gp.time_step(p.depth_increment)
    after = gp.get_state()
    assert not st.converged and st.halvings == 9 and st.newton_iterations == 0
    for a, b in zip(before[:3], after[:3]):
        assert torch.equal(a, b)
    assert after[3] == before[3] == 0.0
    # the newton-system call itself reports the singular block
    with pytest.raises(RuntimeError, match="singular"):
        gp.newton_system(p.depth_increment)
    gp.close()


def test_newton_step_and_tuning_cache():
    """mvpf_newton_step is mvpf_newton_system + mvpf_solve + mvpf_newton_update
    (bitwise the same state afterwards); a second problem of the same shape
    takes its launch shapes from the tuning cache (the same values)."""
    p = synth.Problem(16, 16, 16, n_levels=3, patch=4, depth_increment=0.01)
    U, En = seeded_state(p, 1e-3)
    say("[newton_step] 16^3 mixed")
    a = gpu_problem(p, U, En, "mixed")
    b = gpu_problem(p, U, En, "mixed")
    try:
        a.newton_system(p.depth_increment)
        shapes_a = a.autotune()
        _, sa = a.solve(want_x=False)
        a.newton_update()
        b.newton_system(p.depth_increment)
        assert b.get_tuning("autotune_cache") == 1
        shapes_b = b.autotune()
        assert list(shapes_a) == list(shapes_b)
        b.set_state(U[:, :3], U[:, 3:], En, 0.0)
        sb = b.newton_step(p.depth_increment)
        assert sa.iterations == sb.iterations and sa.converged and sb.converged
        for x, y in zip(a.get_state()[:3], b.get_state()[:3]):
            assert torch.equal(x, y)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("order", [11, 22, 33])
def test_pade_orders_match_oracle(order):
    """Hencky strain by the (1,1), (2,2) or (3,3) Pade approximant (Eqs.
    pade11, pade22, pade33): residual, right-hand side and finest-level K x
    at <= 1e-12 against the oracle of the same order (AD of its own matrix
    polynomials), and a solve at rtol 1e-12 within 1e-9 of the oracle's
    direct solve.  The strains are large enough (random displacements of
    amplitude 5e-3 on h = 1/8) that the orders' residuals differ by far more
    than the tolerance, so a kernel of the wrong order cannot pass."""
    p = synth.Problem(8, 8, 6, lz=0.75, n_levels=2, patch=2, depth_increment=0.01,
                      material=synth.config_material(pade=order))
    U, En = seeded_state(p, 5e-3)
    say(f"[pade {order}] oracle")
    oc = OracleCase(p, U, En, p.depth_increment, build_mg=False)
    if order != 22:
        p22 = synth.Problem(8, 8, 6, lz=0.75, n_levels=2, patch=2, depth_increment=0.01)
        o22 = OracleCase(p22, U, En, p22.depth_increment, build_mg=False, direct=False)
        assert rel(o22.sys.R, oc.sys.R) > 1e-7, rel(o22.sys.R, oc.sys.R)
    say(f"[pade {order}] GPU")
    gp = gpu_problem(p, U, En, "fp64", rtol=1e-12)
    gp.newton_system(p.depth_increment)
    R, _ = gp.residual()
    check_entries(R.cpu().numpy(), oc.sys.R, 1e-12, "residual", oc.abs_scales()[0])
    check_entries(gp.get_rhs().cpu().numpy(), oc.sys.b, 1e-12, "rhs", oc.abs_scales()[1])
    x = np.random.default_rng(5).standard_normal(oc.sys.A.shape[0])
    check_entries(gp.jacobian_apply(0, _dev(x)).cpu().numpy(), oc.sys.A @ x, 1e-12, "K x",
                  abs_product(oc.sys.A, x))
    dx, st = gp.solve()
    gp.close()
    assert st.converged and st.rel_residual <= 1e-12
    assert rel(dx.cpu().numpy(), oc.x) <= 1e-9, rel(dx.cpu().numpy(), oc.x)
