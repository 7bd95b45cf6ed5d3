"""Pins of the oracle's discretisation (Sec. 3.3-3.4) on small Q1 meshes."""
import numpy as np
import pytest
import torch

import synth
from oracle import energy as E
from oracle.fem import Discretisation, Mesh, NDOF
from oracle.material import Card

ZERO_ELASTIC = dict(cubic=(0.0, 0.0, 0.0), ortho=(0.0,) * 9)


def _card(**over):
    base = dict(F0=(0.0,) * 7, w_am=0.0, w_mm=0.0, ell=0.0, rho=0.0, eps_eta=0.0)
    base.update(ZERO_ELASTIC)
    base.update(over)
    return Card(synth.config_material(**base))


def _kron_forms(h):
    Km = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    Mm = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    # local node a = ax + 2 ay + 4 az  <->  kron order (az, ay, ax)
    M3 = np.kron(np.kron(Mm, Mm), Mm)
    L3 = np.kron(np.kron(Mm, Mm), Km) + np.kron(np.kron(Mm, Km), Mm) + np.kron(np.kron(Km, Mm), Mm)
    return M3, L3


def _one_element_tangent(card, h=0.3, seed=0):
    m = Mesh(1, 1, 1, h)
    d = Discretisation(m, card)
    rng = np.random.default_rng(seed)
    U = np.zeros((8, NDOF))
    U[:, 3:] = rng.uniform(0.0, 0.05, (8, 6))
    _, K = d.element_tangents(U.ravel(), U[:, 3:].ravel(), np.array([0]))
    return K[0].reshape(8, NDOF, 8, NDOF)


def test_element_mass_matrix():
    """Viscous term only: K_eta,eta = M_e (x) rho (I + 1 1^T), M_e the textbook
    Q1 mass matrix (exact under 2x2x2 Gauss)."""
    h = 0.3
    K = _one_element_tangent(_card(rho=2.0), h)
    M3, _ = _kron_forms(h)
    S = 2.0 * (np.eye(6) + np.ones((6, 6)))
    assert np.allclose(K[:, 3:, :, 3:], np.einsum("ab,kl->akbl", M3, S), atol=1e-14)
    assert np.allclose(M3.sum(), h ** 3) and np.allclose(M3.sum(1), h ** 3 / 8)
    assert np.abs(K[:, :3]).max() == 0 and np.abs(K[:, :, :, :3]).max() == 0


def test_element_double_obstacle_matrix():
    """Interface term only: K_eta,eta = S (x) (M_e - l^2 L_e), with the hand-
    derived condensed species matrix S_kk = -2 w_am, S_kl = w_mm - 2 w_am."""
    h, wam, wmm, ell = 0.3, 0.7, 0.2, 0.11
    K = _one_element_tangent(_card(w_am=wam, w_mm=wmm, ell=ell), h)
    M3, L3 = _kron_forms(h)
    S = np.full((6, 6), wmm - 2 * wam)
    np.fill_diagonal(S, -2 * wam)
    expect = np.einsum("ab,kl->akbl", M3 - ell ** 2 * L3, S)
    assert np.allclose(K[:, 3:, :, 3:], expect, atol=1e-13)
    assert np.allclose(L3.sum(1), 0.0, atol=1e-14)


def _affine_state(m, A, eta_hat):
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    X = np.stack([i, j, k], 1) * m.h
    U = np.zeros((m.n_nodes, NDOF))
    U[:, :3] = X @ A.T
    U[:, 3:] = eta_hat
    return U


def _interior(m):
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    return (i > 0) & (i < m.nx) & (j > 0) & (j < m.ny) & (k > 0) & (k < m.nz)


def test_patch_affine_displacement_uniform_eta():
    """Homogeneous F and uniform eta_hat: interior mechanical residual is zero
    and the interior eta residual equals h^3 dpsi/deta_hat (sum of the 8
    element integrals of N_a is h^3)."""
    card = Card(synth.config_material())
    m = Mesh(3, 3, 3, 0.2)
    d = Discretisation(m, card)
    rng = np.random.default_rng(11)
    A = 0.02 * rng.standard_normal((3, 3))
    eh = rng.uniform(0.0, 0.05, 6)
    ehn = rng.uniform(0.0, 0.05, 6)
    U = _affine_state(m, A, eh)
    En = np.tile(ehn, (m.n_nodes, 1))
    R = d.residual(U.ravel(), En.ravel()).reshape(-1, NDOF)
    inn = _interior(m)
    scale = np.abs(R[:, :3]).max()
    assert scale > 1e-6
    assert np.abs(R[inn, :3]).max() < 1e-12 * scale
    tc = E.TorchCard(card)
    F = torch.as_tensor(np.eye(3) + A, dtype=torch.float64)
    g = torch.func.grad(lambda e: E.density(F, e, torch.zeros(6, 3, dtype=torch.float64),
                                            torch.as_tensor(ehn), tc))(torch.as_tensor(eh)).numpy()
    assert np.allclose(R[inn, 3:], m.h ** 3 * g, rtol=1e-11, atol=1e-16)


def test_patch_stress_free_state_all_nodes():
    """F = F^t(eta*) everywhere: the mechanical residual vanishes at every
    node, boundary nodes included (P = 0 pointwise)."""
    card = Card(synth.config_material())
    m = Mesh(2, 3, 2, 0.25)
    d = Discretisation(m, card)
    eh = np.array([0.3, 0.05, 0.1, 0.0, 0.2, 0.15])
    Ft = np.einsum("i,ijk->jk", np.concatenate([[1 - eh.sum()], eh]), card.U)
    U = _affine_state(m, Ft - np.eye(3), eh)
    R = d.residual(U.ravel(), U[:, 3:].ravel()).reshape(-1, NDOF)
    assert np.abs(R[:, :3]).max() < 1e-13


def test_interface_energy_of_sine_profile():
    """The 1D double-obstacle profile eta = (1 + sin(x/l))/2 across a width
    pi*l carries energy gamma = w pi l / 4 per unit area (Eq. IntEnergy with
    w = 4 gamma/(pi l)); the Q1 value converges to it at second order."""
    w, ell = 1.0, 0.08
    gamma = w * np.pi * ell / 4
    card = _card(w_am=w, w_mm=0.0, ell=ell)
    errs = []
    for nx in (16, 32, 64):
        h = 1.0 / nx
        m = Mesh(nx, 1, 1, h)
        i, _, _ = m.node_ijk(np.arange(m.n_nodes))
        s = np.clip((i * h - 0.5) / ell, -np.pi / 2, np.pi / 2)
        eta1 = 0.5 * (1 + np.sin(s))
        U = np.zeros((m.n_nodes, NDOF))
        U[:, 3] = eta1
        d = Discretisation(m, card)
        errs.append(abs(d.potential(U.ravel(), U[:, 3:].ravel()) / h ** 2 - gamma))
    assert errs[-1] < 0.01 * gamma
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_tangent_is_symmetric_and_matches_fd_of_residual():
    card = Card(synth.config_material())
    m = Mesh(2, 2, 2, 0.5)
    d = Discretisation(m, card)
    rng = np.random.default_rng(3)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, :3] = 0.01 * rng.standard_normal((m.n_nodes, 3))
    U[:, 3:] = rng.uniform(0.01, 0.05, (m.n_nodes, 6))
    En = rng.uniform(0.0, 0.05, (m.n_nodes, 6)).ravel()
    from oracle.solver import assemble
    K = assemble(d, U.ravel(), En).toarray()
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())
    v = rng.standard_normal(K.shape[0])
    eps = 1e-6
    fd = (d.residual(U.ravel() + eps * v, En) - d.residual(U.ravel() - eps * v, En)) / (2 * eps)
    assert np.linalg.norm(fd - K @ v) <= 1e-7 * np.linalg.norm(K @ v)


def test_sampled_residual_equals_full_residual_rows():
    card = Card(synth.config_material())
    m = Mesh(4, 4, 4, 0.25)
    d = Discretisation(m, card)
    rng = np.random.default_rng(4)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, :3] = 0.01 * rng.standard_normal((m.n_nodes, 3))
    U[:, 3:] = synth.initial_eta(7, m.n_nodes)
    En = U[:, 3:].ravel().copy()
    R = d.residual(U.ravel(), En).reshape(-1, NDOF)
    nodes = np.array([0, 17, 62, m.n_nodes - 1])
    Rs = d.residual(U.ravel(), En, elems=m.elements_of_nodes(nodes)).reshape(-1, NDOF)
    assert np.array_equal(R[nodes], Rs[nodes])
