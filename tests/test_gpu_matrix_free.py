"""Matrix-free finest level (tuning key "matrix_free"): the tangent applied
from its stored Gauss-point Hessians, never assembled into blocks, vs the
oracle's assembled tangent (Sec. 3.4).

Tolerances as for the assembled operators: FP64 K x <= 1e-12 relative, FP32
<= 2e-6, V-cycle (FP64 mode) <= 1e-10, solves at rtol 1e-12 within 1e-9 of
the oracle's direct solve.  Cases: the patch cases of the parity tests, a
spherical-cap case and a sphere-contact case (the contact stiffness is
applied matrix-free as well)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import OracleCase, abs_product, check_entries, gpu_problem, rel, say, seeded_state

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": (synth.tiny(), 0.0, 0.02),
    "ragged": (synth.Problem(8, 12, 4, ly=1.5, lz=0.5, n_levels=3, patch=2, depth_increment=0.01), 2e-3, 0.01),
    "minimal": (synth.Problem(2, 2, 2, n_levels=2, patch=2, depth_increment=0.05), 1e-3, 0.05),
    "sphere": (synth.Problem(8, 8, 4, lz=0.5, n_levels=3, kind="sphere", radius=0.5), 1e-3, 0.03),
}


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


@pytest.fixture(scope="module", params=list(CASES))
def mf_case(request):
    p, amp, d = CASES[request.param]
    U, En = seeded_state(p, amp)
    say(f"[mf {request.param}] oracle")
    oc = OracleCase(p, U, En, d)
    yield request.param, p, U, En, d, oc


def _mf_problem(p, U, En, d, precision, **opts):
    gp = gpu_problem(p, U, En, precision, depth=d, **opts)
    gp.set_tuning("matrix_free", 0, 1)
    assert gp.get_tuning("matrix_free") == 1
    gp.newton_system(d)
    return gp


def test_mf_fp64_operator_vcycle_solve(mf_case):
    name, p, U, En, d, oc = mf_case
    from paper_2011_08802_amd import mvpf
    say(f"[mf {name}] fp64")
    gp = _mf_problem(p, U, En, d, "fp64", rtol=1e-12)
    rng = np.random.default_rng(21)
    x = rng.standard_normal(oc.sys.b.shape[0])
    check_entries(gp.jacobian_apply(0, _dev(x), mvpf.FP64).cpu().numpy(), oc.sys.A @ x, 1e-12, "FP64 K x",
                  abs_product(oc.sys.A, x))
    v = rng.standard_normal(oc.sys.b.shape[0])
    assert rel(gp.precondition(_dev(v)).cpu().numpy(), oc.mg.precondition(v)) < 1e-10
    check_entries(gp.get_rhs().cpu().numpy(), oc.sys.b, 1e-12, "rhs", oc.abs_scales()[1])
    dx, st = gp.solve()
    gp.close()
    assert st.converged and st.rel_residual <= 1e-12
    assert rel(dx.cpu().numpy(), oc.x) <= 1e-9, rel(dx.cpu().numpy(), oc.x)


def test_mf_mixed_operator_and_solve(mf_case):
    name, p, U, En, d, oc = mf_case
    from paper_2011_08802_amd import mvpf
    say(f"[mf {name}] mixed")
    gp = _mf_problem(p, U, En, d, "mixed", rtol=1e-12)
    rng = np.random.default_rng(22)
    x = rng.standard_normal(oc.sys.b.shape[0])
    ax = abs_product(oc.sys.A, x)
    check_entries(gp.jacobian_apply(0, _dev(x), mvpf.MIXED).cpu().numpy(), oc.sys.A @ x, 2e-6, "FP32 K x", ax)
    check_entries(gp.jacobian_apply(0, _dev(x), mvpf.FP64).cpu().numpy(), oc.sys.A @ x, 1e-12, "FP64 K x", ax)
    dx, st = gp.solve()
    gp.close()
    assert st.converged and st.rel_residual <= 1e-12
    assert rel(dx.cpu().numpy(), oc.x) <= 1e-9, rel(dx.cpu().numpy(), oc.x)


def test_mf_iterations_match_assembled():
    """Same preconditioner up to rounding: FGMRES at rtol 1e-8 takes the same
    number of iterations (+-1) with and without the matrix-free finest level,
    and both results are deterministic."""
    p = synth.Problem(16, 16, 16, n_levels=3, patch=4, depth_increment=0.01)
    U, En = seeded_state(p, 1e-3)
    its = []
    for mf in (0, 1, 1):
        say(f"[mf 16^3] matrix_free={mf}")
        gp = gpu_problem(p, U, En, "mixed")
        gp.set_tuning("matrix_free", 0, mf)
        gp.newton_system(p.depth_increment)
        x, st = gp.solve()
        its.append((st.iterations, x.cpu().numpy()))
        gp.close()
    assert abs(its[0][0] - its[1][0]) <= 1 and its[1][0] == its[2][0]
    assert np.array_equal(its[1][1], its[2][1])
    assert rel(its[1][1], its[0][1]) < 1e-6


MERGE_CASES = {
    # 20 elements per row: workgroups of 8, 16 and 32 elements end inside rows
    # and take several row ends; the sphere case adds the contact face outputs
    "rows20": synth.Problem(20, 6, 4, ly=0.3, lz=0.2, n_levels=2, patch=2, depth_increment=0.01),
    "rows20_sphere": synth.Problem(20, 6, 4, ly=0.3, lz=0.2, n_levels=2, kind="sphere", radius=0.5,
                                   depth_increment=0.03),
}


@pytest.mark.parametrize("name", list(MERGE_CASES))
def test_mf_merged_outputs_independent_of_workgroup_size(name):
    """Element outputs merged along x inside a workgroup (its last element's
    right corners and row ends through separate streams): for 8, 16 and 32
    elements per workgroup the FP32 and FP64 products and the V-cycle are
    bitwise the same (a node's two parts always meet in one addition), and
    the products match the oracle's tangent entry by entry."""
    from paper_2011_08802_amd import mvpf
    p = MERGE_CASES[name]
    U, En = seeded_state(p, 1e-3)
    d = p.depth_increment
    say(f"[mf merge {name}] oracle")
    oc = OracleCase(p, U, En, d, build_mg=False, direct=False)
    rng = np.random.default_rng(31)
    x = rng.standard_normal(oc.sys.b.shape[0])
    v = rng.standard_normal(oc.sys.b.shape[0])
    ya = abs_product(oc.sys.A, x)
    outs = []
    for epw in (8, 16, 32):
        say(f"[mf merge {name}] {epw} elements per workgroup")
        gp = gpu_problem(p, U, En, "mixed", depth=d)
        try:
            gp.set_tuning("matrix_free", 0, 1)
            gp.set_tuning("mf_elements_per_block", 0, epw)
            gp.newton_system(d)
            y64 = gp.jacobian_apply(0, _dev(x), mvpf.FP64).cpu().numpy()
            y32 = gp.jacobian_apply(0, _dev(x), mvpf.MIXED).cpu().numpy()
            z = gp.precondition(_dev(v)).cpu().numpy()
        finally:
            gp.close()
        check_entries(y64, oc.sys.A @ x, 1e-12, f"FP64 K x ({epw})", ya)
        check_entries(y32, oc.sys.A @ x, 2e-6, f"FP32 K x ({epw})", ya)
        outs.append((y64, y32, z))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
