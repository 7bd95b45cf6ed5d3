"""Pins of the oracle's penalty contact with a rigid sphere (Sec. 2.4, Eqs.
Ngap and PenPot) and of its indentation driver with adaptive time steps
(Sec. 3.4)."""
import numpy as np
import pytest

import synth
from oracle import solver as S
from oracle.contact import SphereContact
from oracle.fem import Mesh, NDOF

R, EPS = 0.2, 3.5e4


def flat_energy(d, r=R, eps=EPS):
    """Closed form for an undeformed flat surface and a contact disk inside
    the face: with s = |x - c| the gap is s - R on the disk and s ds = rho
    d rho, so Pi_c = pi eps int_{R-d}^{R} (s - R)^2 s ds."""
    def F(s):
        return s ** 4 / 4.0 - 2.0 * r * s ** 3 / 3.0 + r * r * s * s / 2.0
    return np.pi * eps * (F(r) - F(r - d))


def flat_load(d, r=R, eps=EPS):
    """d/dd of the closed form: pi eps d^2 (R - d) (pi eps R d^2 for d << R,
    the integral of eps times the parabolic penetration d - rho^2 / 2R)."""
    return np.pi * eps * d * d * (r - d)


@pytest.mark.parametrize("n, tol_e, tol_p", [(64, 1e-4, 3e-3), (128, 1e-5, 1e-4)])
def test_flat_surface_closed_form(n, tol_e, tol_p):
    """Energy and load of the 2x2 Gauss face quadrature converge to the
    closed forms (the gap's sign, the sphere's centre, the face weights and
    the factor 1/2 all enter)."""
    m = Mesh(n, n, 1, 1.0 / n)
    c = SphereContact(m, R, EPS)
    U = np.zeros(m.n_nodes * NDOF)
    d = 0.02
    assert abs(c.energy(U, d) / flat_energy(d) - 1.0) < tol_e
    assert abs(c.load(U, d) / flat_load(d) - 1.0) < tol_p


def test_rigid_lift_is_a_deeper_indenter():
    """x = X + u: lifting the whole surface by t is the same as pushing the
    indenter t deeper."""
    m = Mesh(32, 32, 1, 1.0 / 32)
    c = SphereContact(m, R, EPS)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 2] = 0.004
    assert np.isclose(c.energy(U.ravel(), 0.01), c.energy(np.zeros(U.size), 0.014), rtol=1e-13)
    assert np.isclose(c.load(U.ravel(), 0.01), c.load(np.zeros(U.size), 0.014), rtol=1e-12)


def _deformed(m, amp=2e-3, seed=3):
    U = np.zeros((m.n_nodes, NDOF))
    U[:, :3] = amp * np.random.default_rng(seed).standard_normal((m.n_nodes, 3))
    U[:, 3:] = 0.01
    return U.ravel()


def test_residual_tangent_load_are_derivatives():
    """Central differences of the energy (residual, load) and of the residual
    (tangent) on a deformed surface with a partial contact zone; the tangent
    is symmetric; only top-face displacement dofs carry contact terms."""
    m = Mesh(6, 6, 2, 1.0 / 6)
    c = SphereContact(m, 0.6, EPS)
    U = _deformed(m)
    d = 0.03
    Rv = c.residual(U, d)
    r, cc, v = c.tangent_coo(U, d)
    n = m.n_nodes * NDOF
    import scipy.sparse as sp
    K = sp.coo_matrix((v, (r, cc)), shape=(n, n)).toarray()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    _, _, k = m.node_ijk(np.arange(m.n_nodes))
    nz = np.nonzero(Rv)[0]
    assert len(nz) > 0 and np.all(k[nz // NDOF] == m.nz) and np.all(nz % NDOF < 3)
    hstep = 1e-7
    dofs = nz[np.argsort(-np.abs(Rv[nz]))[:6]]
    for q in dofs:
        e = np.zeros(n)
        e[q] = hstep
        fd = (c.energy(U + e, d) - c.energy(U - e, d)) / (2 * hstep)
        assert abs(fd - Rv[q]) <= 1e-6 * np.abs(Rv).max(), (q, fd, Rv[q])
        col = (c.residual(U + e, d) - c.residual(U - e, d)) / (2 * hstep)
        assert np.abs(col - K[:, q]).max() <= 1e-5 * np.abs(K).max()
    fdP = (c.energy(U, d + hstep) - c.energy(U, d - hstep)) / (2 * hstep)
    assert abs(fdP - c.load(U, d)) <= 1e-6 * abs(fdP)
    assert c.load(U, d) > 0.0


def test_separated_indenter_contributes_nothing():
    m = Mesh(6, 6, 2, 1.0 / 6)
    c = SphereContact(m, 0.6, EPS)
    U = _deformed(m, amp=1e-4)
    d = -0.01
    assert c.energy(U, d) == 0.0 and c.load(U, d) == 0.0
    assert not np.any(c.residual(U, d))
    assert not np.any(c.tangent_coo(U, d)[2])


def test_sphere_loading_constrains_only_the_bottom():
    m = Mesh(4, 4, 4, 0.25)
    mask, target = S.dirichlet(m, "sphere")
    _, _, k = m.node_ijk(np.arange(m.n_nodes))
    assert mask[k == 0][:, :3].all() and mask.sum() == 3 * np.count_nonzero(k == 0)
    assert not np.any(target)


def test_step_control_rule(monkeypatch):
    """The adaptive rule with fake Newton results: grow below 7 iterations,
    shrink above, halve and retry on failure, never overshoot, unload to 0,
    and rho = visc_depth / |dd| for every attempted step."""
    p = synth.Problem(4, 4, 2, lz=0.5, n_levels=2, kind="sphere", radius=0.5)
    U = np.zeros(p.n_nodes * NDOF)
    En = np.zeros(p.n_nodes * 6)
    script = iter([(3, True), (9, True), (12, False), (7, True), (3, True), (5, True),
                   (8, True)] + [(4, True)] * 20)
    seen = []

    def fake(problem, card, U, Eta_n, mask, g, rtol, max_iter, depth):
        it, ok = next(script)
        seen.append((depth, card.rho))
        return U, it, ok

    monkeypatch.setattr(S, "newton_step", fake)
    monkeypatch.setattr(SphereContact, "load", lambda self, U, d: d)
    o = S.IndentOptions(depth_max=0.03, dd_init=0.01, dd_min=1e-4, dd_max=0.02, visc_depth=1e-3)
    recs, _, ok = S.indent(p, U, En, o)
    assert ok
    # steps 0.01 (3 its: x1.25), 0.0125 (9 its: x0.8), then the last 0.0075
    # of the loading fails and is retried with half of it (7 its: kept),
    # and the remaining 0.00375 lands on 0.03 exactly
    assert [r.depth for r in recs[:4]] == pytest.approx([0.01, 0.0225, 0.02625, 0.03])
    assert recs[3].depth == 0.03
    assert recs[2].rejected == 1
    # rho of every attempt = visc_depth / step
    assert seen[0][1] == pytest.approx(1e-3 / 0.01)
    assert seen[1][1] == pytest.approx(1e-3 / 0.0125)
    assert seen[2][1] == pytest.approx(1e-3 / 0.0075)
    assert seen[3][1] == pytest.approx(1e-3 / 0.00375)
    # the loading phase ends exactly at depth_max, the unloading one at 0
    ds = [r.depth for r in recs]
    assert 0.03 in ds and ds[-1] == 0.0
    i = ds.index(0.03)
    assert all(a < b for a, b in zip(ds[:i], ds[1:i + 1]))
    assert all(a > b for a, b in zip(ds[i:], ds[i + 1:]))


def test_small_indentation_run():
    """A whole load-unload run on a 4x4x2 mesh: the load rises with depth
    while loading, falls while unloading and vanishes at depth 0 (the surface
    springs back: no contact left)."""
    p = synth.Problem(4, 4, 2, lz=0.5, n_levels=2, kind="sphere", radius=1.0,
                      material=synth.config_material())
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    o = S.IndentOptions(depth_max=0.01, dd_init=0.0025, dd_min=1e-5, dd_max=0.005, visc_depth=0.05)
    recs, U1, ok = S.indent(p, U.ravel(), U[:, 3:].ravel().copy(), o)
    assert ok
    ds = np.array([r.depth for r in recs])
    Ps = np.array([r.load for r in recs])
    i = int(np.argmax(ds))
    assert ds[i] == 0.01 and ds[-1] == 0.0 and len(recs) > 3
    assert np.all(np.diff(Ps[:i + 1]) > 0) and np.all(np.diff(Ps[i:]) <= 0)
    assert Ps[i] > 0 and Ps[-1] <= 1e-6 * Ps[i]
