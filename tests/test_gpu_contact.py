"""Penalty contact with a rigid sphere (Sec. 2.4, Eqs. Ngap and PenPot) and
the indentation driver with adaptive time steps (Sec. 3.4), GPU vs oracle.

Tolerances as in the other parity tests: FP64 operators <= 1e-12 relative,
V-cycle <= 1e-10, solves at rtol 1e-12 within 1e-9 of the oracle's direct
solve.  The driver's step sizes are decided by Newton iteration counts (FP64
on both sides): the accepted depths must agree exactly, the loads and final
states within 1e-8 relative."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import OracleCase, abs_product, check_entries, gpu_problem, rel, say, seeded_state
from oracle import solver as S
from oracle.contact import SphereContact
from oracle.fem import Mesh, NDOF
from oracle.material import Card

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


# 8x8x4 on a 1x1x0.5 box, sphere R = 0.5 pressed 0.03: ~12 top faces in
# contact on the finest level, 3 levels (the coarsest 2x2x1 still in contact)
def sphere_problem(n_levels=3, radius=0.5):
    return synth.Problem(8, 8, 4, lz=0.5, n_levels=n_levels, kind="sphere", radius=radius)


@pytest.fixture(scope="module")
def contact_case():
    p = sphere_problem()
    U, En = seeded_state(p, 1e-3)
    d = 0.03
    say("[contact] oracle system")
    oc = OracleCase(p, U, En, d)
    say("[contact] GPU system")
    gp = gpu_problem(p, U, En, "fp64", depth=d, rtol=1e-12)
    gp.newton_system(d)
    yield p, U, En, d, oc, gp
    gp.close()


def test_contact_is_active(contact_case):
    p, U, En, d, oc, gp = contact_case
    c = SphereContact(Mesh.from_problem(p), p.radius, p.eps_n)
    assert np.count_nonzero(c.residual(U.ravel(), d)) >= 30


def test_contact_residual_rhs_parity(contact_case):
    p, U, En, d, oc, gp = contact_case
    say("[contact] residual, rhs")
    R, nf = gp.residual()
    check_entries(R.cpu().numpy(), oc.sys.R, 1e-12, "residual", oc.abs_scales()[0])
    check_entries(gp.get_rhs().cpu().numpy(), oc.sys.b, 1e-12, "rhs", oc.abs_scales()[1])


def test_contact_operator_parity_all_levels(contact_case):
    p, U, En, d, oc, gp = contact_case
    rng = np.random.default_rng(11)
    for l, lev in enumerate(oc.mg.levels):
        say(f"[contact] K x level {l}")
        x = rng.standard_normal(lev.A.shape[0])
        check_entries(gp.jacobian_apply(l, _dev(x)).cpu().numpy(), lev.A @ x, 1e-12, f"K x level {l}",
                      abs_product(lev.A, x))


def test_contact_vcycle_and_solve(contact_case):
    p, U, En, d, oc, gp = contact_case
    say("[contact] V-cycle, solve")
    v = np.random.default_rng(12).standard_normal(oc.sys.b.shape[0])
    assert rel(gp.precondition(_dev(v)).cpu().numpy(), oc.mg.precondition(v)) < 1e-10
    x, st = gp.solve()
    assert st.converged and st.rel_residual <= 1e-12
    assert rel(x.cpu().numpy(), oc.x) <= 1e-9, rel(x.cpu().numpy(), oc.x)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_contact_load_parity(contact_case, precision):
    """mvpf_contact_load vs the oracle's AD derivative of the contact energy
    with respect to the depth, at the state and depth set on the problem."""
    p, U, En, d, oc, _ = contact_case
    gp = gpu_problem(p, U, En, precision, depth=d)
    P = gp.contact_load()
    gp.close()
    Po = SphereContact(Mesh.from_problem(p), p.radius, p.eps_n).load(U.ravel(), d)
    assert Po > 0 and abs(P - Po) <= 1e-12 * abs(Po), (P, Po)


def test_contact_time_step_matches_oracle():
    """One implicit step with contact from the seeded state: Newton iteration
    count and end state vs the oracle's Newton with direct solves."""
    p = sphere_problem(n_levels=2)
    U, En = seeded_state(p, 0.0)
    d = 0.02
    card = Card(p.material)
    m = Mesh.from_problem(p)
    mask, _ = S.dirichlet(m, "sphere")
    say("[contact step] oracle Newton")
    Uo, it, ok = S.newton_step(p, card, U.ravel(), En.ravel(), mask, np.zeros(mask.shape), rtol=1e-11, depth=d)
    assert ok
    say("[contact step] GPU time step")
    gp = gpu_problem(p, U, En, "fp64", rtol=1e-12, newton_rtol=1e-11)
    st = gp.time_step(d)
    u, e, en, dd = gp.get_state()
    gp.close()
    assert st.converged and st.halvings == 0 and st.newton_iterations == it, (st.newton_iterations, it)
    got = np.concatenate([u.cpu().numpy(), e.cpu().numpy()], 1)
    assert dd == d and rel(got, Uo.reshape(-1, NDOF)) <= 1e-9


def test_indentation_run_matches_oracle():
    """Load to 0.01 and unload on a 4x4x2 mesh (sphere R = 1): the accepted
    depths (decided by Newton iteration counts), the iteration counts, the
    loads and the final state agree with the oracle's driver."""
    p = synth.Problem(4, 4, 2, lz=0.5, n_levels=2, kind="sphere", radius=1.0)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    kw = dict(depth_max=0.01, dd_init=0.0025, dd_min=1e-5, dd_max=0.005, visc_depth=0.05)
    say("[indent] oracle driver")
    recs, Uo, ok = S.indent(p, U.ravel(), U[:, 3:].ravel().copy(), S.IndentOptions(**kw))
    assert ok
    say("[indent] GPU driver")
    gp = gpu_problem(p, U, U[:, 3:], "fp64", rtol=1e-12)
    grecs, rc = gp.indent(max_steps=100, **kw)
    u, e, en, dd = gp.get_state()
    gp.close()
    assert rc == 0 and len(grecs) == len(recs)
    assert [r.depth for r in grecs] == [r.depth for r in recs]
    assert [r.newton_iterations for r in grecs] == [r.newton_iterations for r in recs]
    assert [r.rejected for r in grecs] == [r.rejected for r in recs]
    Pg = np.array([r.load for r in grecs])
    Po = np.array([r.load for r in recs])
    assert np.abs(Pg - Po).max() <= 1e-8 * np.abs(Po).max()
    got = np.concatenate([u.cpu().numpy(), e.cpu().numpy()], 1)
    assert dd == 0.0 and rel(got, Uo.reshape(-1, NDOF)) <= 1e-8
