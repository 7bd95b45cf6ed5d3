"""Pins of the oracle for cards with N variants generated from one stretch
tensor by the cubic symmetry (N = 12 here, 15 unknowns per node; the paper's
footnote in Sec. 4.4) and for the logarithmic mixing rule of the
transformation stretch (Sec. 2.1).  The 12-variant card is synthetic."""
import numpy as np
import pytest
import torch
from torch.func import grad, hessian

import synth
from oracle import energy as E
from oracle import material as M
from oracle import solver as S
from oracle.fem import Discretisation, Mesh
from oracle.material import Card

DT = torch.float64
CARDS = {
    "cualni-linear": lambda: synth.config_material(),
    "cualni-log": lambda: synth.config_material(mixing="log"),
    "n12-linear": lambda: synth.twelve_variant_material(),
    "n12-log": lambda: synth.twelve_variant_material(mixing="log"),
}


def test_cubic_rotations():
    R = M.cubic_rotations()
    assert len(R) == 24
    for Q in R:
        assert np.allclose(Q @ Q.T, np.eye(3)) and np.isclose(np.linalg.det(Q), 1.0)
    # a group: closed under products, all distinct
    keys = {tuple(Q.ravel()) for Q in R}
    assert len(keys) == 24
    for A in R:
        for B in R:
            assert tuple((A @ B).ravel()) in keys


def test_orbit_of_the_six_variant_stretch_is_sec41():
    """The cubic orbit of U_1 of Sec. 4.1 is exactly the six printed
    variants (as a set): the orbit construction reproduces the paper's card."""
    a, b, g = 1.0424, 0.9178, 1.0619
    U = M.stretch_tensors(a, b, g)
    orb, _ = M.orbit_variants(U[1])
    assert len(orb) == 6
    for V in orb:
        assert any(np.allclose(V, U[k], atol=1e-15) for k in range(1, 7))


def test_twelve_variant_card():
    """12 distinct symmetric variants, each with the eigenvalues and the
    determinant of U1; the set is closed under the cubic rotations; variant
    k's stiffness is L1 rotated by the rotation that made U_k (checked in
    the sample frame through (n n) : L_k : (n n) = L1_iiii for n = Q R_k e_i)."""
    om = synth.twelve_variant_material()
    card = Card(om)
    U1 = np.asarray(om.U1).reshape(3, 3)
    lam = np.linalg.eigvalsh(U1)
    assert card.n_var == 12 and card.U.shape == (13, 3, 3) and card.L.shape == (13, 3, 3, 3, 3)
    Q = np.asarray(om.Q).reshape(3, 3)
    cub = [Q.T @ card.U[k] @ Q for k in range(1, 13)]  # back in cubic axes
    for V in cub:
        assert np.allclose(V, V.T)
        assert np.allclose(np.linalg.eigvalsh(V), lam, atol=1e-14)
    for i in range(12):
        for j in range(i):
            assert np.max(np.abs(cub[i] - cub[j])) > 1e-3
    for R in M.cubic_rotations():
        for V in cub:
            assert any(np.allclose(R @ V @ R.T, W, atol=1e-14) for W in cub)
    _, Rs = M.orbit_variants(U1)
    L1 = np.asarray(om.L1).reshape(6, 6)
    for k in range(1, 13):
        for i in range(3):
            n = Q @ Rs[k - 1][:, i]
            nn = np.outer(n, n)
            assert np.isclose(np.einsum("ij,ijkl,kl->", nn, card.L[k], nn), L1[i, i], rtol=1e-12)
    assert card.W.shape == (13, 13) and card.W[0, 5] == om.w_am and card.W[3, 7] == om.w_mm


@pytest.mark.parametrize("name", ["cualni-log", "n12-log"])
def test_log_mixing_closed_forms(name):
    """F^t = exp(sum eta_i log U_i): F^t = U_k for a pure variant, I for the
    austenite, U_k^t on the austenite-variant edge (eigenvalues lambda^t),
    and det F^t = prod_k det(U_k)^eta_k = (det U)^(1 - eta_0) since every
    variant has the same determinant; so exchanging two variants' fractions
    at fixed eta_0 leaves det F^t unchanged.  Under linear mixing the
    determinant does not follow that power law."""
    card = Card(CARDS[name]())
    tc = E.TorchCard(card)
    n = card.n_var
    detU = np.linalg.det(card.U[1])
    eta = torch.zeros(n + 1, dtype=DT)
    eta[0] = 1.0
    assert np.allclose(E.transformation_gradient(eta, tc).numpy(), np.eye(3), atol=1e-15)
    for k in range(1, n + 1):
        eta = torch.zeros(n + 1, dtype=DT)
        eta[k] = 1.0
        assert np.allclose(E.transformation_gradient(eta, tc).numpy(), card.U[k], atol=1e-14)
        for t in (0.3, 0.8):
            eta = torch.zeros(n + 1, dtype=DT)
            eta[0], eta[k] = 1.0 - t, t
            Ft = E.transformation_gradient(eta, tc).numpy()
            w, V = np.linalg.eigh(card.U[k])
            assert np.allclose(Ft, V @ np.diag(w ** t) @ V.T, atol=1e-14)
    rng = np.random.default_rng(4)
    for _ in range(3):
        eh = rng.uniform(0.0, 0.15, n)
        eta = torch.as_tensor(np.concatenate([[1 - eh.sum()], eh]), dtype=DT)
        d = float(torch.linalg.det(E.transformation_gradient(eta, tc)))
        assert abs(d - detU ** eh.sum()) <= 1e-14
        i, j = 1, 1 + n // 2
        sw = eta.clone()
        sw[i], sw[j] = eta[j], eta[i]
        d2 = float(torch.linalg.det(E.transformation_gradient(sw, tc)))
        assert abs(d2 - d) <= 1e-14
    if name == "cualni-log":  # the power law of det F^t is not that of linear mixing
        tl = E.TorchCard(Card(synth.config_material()))
        eta = torch.as_tensor(np.concatenate([[0.5], [0.5, 0, 0, 0, 0, 0]]), dtype=DT)
        assert abs(float(torch.linalg.det(E.transformation_gradient(eta, tl))) - detU ** 0.5) > 1e-3


@pytest.mark.parametrize("name", list(CARDS))
def test_stress_free_and_small_strain(name):
    """F = R F^t(eta): the elastic energy and P vanish (any mixing rule, any
    N); at F = I, eta = austenite, d^2 psi / dF^2 = L_0."""
    card = Card(CARDS[name]())
    tc = E.TorchCard(card)
    n = card.n_var
    rng = np.random.default_rng(11)
    eh = torch.as_tensor(rng.uniform(0.0, 0.15, n), dtype=DT)
    eta = E.full_eta(eh)
    R = torch.as_tensor(synth.random_rotation(3), dtype=DT)
    F = R @ E.transformation_gradient(eta, tc)
    P = grad(lambda F: E.elastic_energy(F, eta, tc))(F)
    assert float(P.abs().max()) < 1e-11
    eta0 = E.full_eta(torch.zeros(n, dtype=DT))
    Hs = hessian(lambda F: E.elastic_energy(F, eta0, tc))(torch.eye(3, dtype=DT))
    assert np.allclose(Hs.numpy(), card.L[0], atol=1e-10)


@pytest.mark.parametrize("name", ["cualni-log", "n12-linear"])
def test_log_and_n12_ad_matches_central_differences(name):
    card = Card(CARDS[name]())
    tc = E.TorchCard(card)
    n = card.n_var
    rng = np.random.default_rng(5)
    F = torch.as_tensor(np.eye(3) + 0.03 * rng.standard_normal((3, 3)), dtype=DT)
    eh = torch.as_tensor(rng.uniform(0.02, 0.1, n), dtype=DT)
    geh = torch.as_tensor(0.1 * rng.standard_normal((n, 3)), dtype=DT)
    ehn = torch.as_tensor(rng.uniform(0.0, 0.1, n), dtype=DT)

    def f(x):
        return E.density(x[:9].reshape(3, 3), x[9:9 + n], x[9 + n:].reshape(n, 3), ehn, tc)

    x0 = torch.cat([F.ravel(), eh, geh.ravel()])
    g = grad(f)(x0).numpy()
    h = 1e-5
    for i in range(9 + n):
        e = torch.zeros_like(x0)
        e[i] = h
        fd = (float(f(x0 + e)) - float(f(x0 - e))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i]))


def test_elastic_prefactor_log_mixing():
    """Along F = lam F^t(eta) with logarithmic mixing, psi_el =
    1/2 (det U)^(1 - eta_0) r(lam^2)^2 sum_i eta_i I:L_i:I (Eq. elasticEn;
    I:L:I = 1182 for the austenite, 1104 for every CuAlNi variant)."""
    mp = synth.config_material(mixing="log")
    tc = E.TorchCard(Card(mp))
    detU = mp.alpha * mp.beta * mp.gamma
    lam = 1.02
    c = lam * lam
    r = 1.5 * (c * c - 1.0) / (c * c + 4.0 * c + 1.0)
    eh = torch.zeros(6, dtype=DT)
    eh[0], eh[3], eh[5] = 0.2, 0.15, 0.1
    eta = E.full_eta(eh)
    got = float(E.elastic_energy(lam * E.transformation_gradient(eta, tc), eta, tc))
    want = 0.5 * detU ** 0.45 * r * r * (0.55 * 1182.0 + 0.45 * 1104.0)
    assert abs(got - want) <= 1e-12 * abs(want)


def test_n12_patch_test_and_tangent():
    """15 unknowns per node: an affine displacement with uniform order
    parameters leaves zero mechanical residual at interior nodes (patch
    test), and the tangent is the central difference of the residual."""
    om = synth.twelve_variant_material()
    card = Card(om)
    p = synth.Problem(3, 3, 3, n_levels=2, patch=2, material=om)
    m = Mesh.from_problem(p)
    disc = Discretisation(m, card)
    assert disc.ndof == 15
    rng = np.random.default_rng(2)
    G = 0.01 * rng.standard_normal((3, 3))
    X = np.stack(m.node_xyz(np.arange(m.n_nodes)), axis=1) if hasattr(m, "node_xyz") else \
        np.stack([v * m.h for v in m.node_ijk(np.arange(m.n_nodes))], axis=1)
    U = np.zeros((m.n_nodes, 15))
    U[:, :3] = X @ G.T
    U[:, 3:] = rng.uniform(0.0, 0.1, 12)
    R = disc.residual(U.ravel(), U[:, 3:].ravel().copy()).reshape(-1, 15)
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    inner = (i > 0) & (i < m.nx) & (j > 0) & (j < m.ny) & (k > 0) & (k < m.nz)
    assert inner.sum() == 8
    assert np.abs(R[inner, :3]).max() < 1e-12 * max(1.0, np.abs(R[:, :3]).max())
    # tangent vs central differences of the residual (a few columns)
    U[:, 3:] = p.eta0()
    U[:, :3] = 1e-3 * rng.standard_normal((m.n_nodes, 3))
    En = U[:, 3:].ravel().copy()
    r, c, v = disc.tangent_coo(U.ravel(), En)
    import scipy.sparse as sp
    K = sp.coo_matrix((v, (r, c)), shape=(U.size, U.size)).tocsr()
    assert abs(K - K.T).max() < 1e-9 * abs(K).max()
    for col in (0, 20, 4 * 15 + 7, 40 * 15 + 14):
        e = np.zeros(U.size)
        e[col] = 1e-6
        fd = (disc.residual(U.ravel() + e, En) - disc.residual(U.ravel() - e, En)) / 2e-6
        assert np.allclose(K[:, col].toarray().ravel(), fd, rtol=1e-6, atol=1e-5)


def test_n12_solver_reaches_direct_solution():
    """Newton system with 15 unknowns per node: FGMRES + GMG (point-block
    Jacobi with 15x15 blocks) reaches the direct solution; the initial order
    parameters use the counters (3 + N) a + 3 + i."""
    om = synth.twelve_variant_material()
    p = synth.Problem(4, 4, 4, n_levels=2, patch=2, depth_increment=0.02, material=om)
    e = p.eta0()
    assert e.shape == (p.n_nodes, 12) and p.n_dof == 15 * p.n_nodes
    assert np.array_equal(e[1, 0:1], synth.uniform01(p.seed, np.array([15 + 3], dtype=np.uint64)) * 0.05)
    card = Card(om)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, 15))
    U[:, 3:] = e
    mask, target = S.dirichlet(m, "patch", p.patch, depth=p.depth_increment, ndof=15)
    g = S.increment(mask, target, U)
    sy = S.NewtonSystem(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, g)
    mg = S.Multigrid(p, card, U.ravel(), U[:, 3:].ravel().copy(), mask, K_fine=sy.K)
    assert mg.bs == 15 and mg.levels[0].Dinv.shape[1:] == (15, 15)
    x, st = S.fgmres(sy.A, sy.b, mg.precondition, rtol=1e-12)
    xd = S.direct_solve(sy.A, sy.b)
    assert st.converged and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
