"""Pins of the oracle's material card (Sec. 4.1, Table 1)."""
import numpy as np
import pytest

import synth
from oracle import material as M


@pytest.mark.parametrize("abg", [(1.0424, 0.9178, 1.0619), (1.0619, 0.9178, 1.0230)])
def test_stretch_eigenvalues_and_det(abg):
    a, b, g = abg
    U = M.stretch_tensors(a, b, g)
    assert np.allclose(U[0], np.eye(3))
    for k in range(1, 7):
        assert np.allclose(U[k], U[k].T)
        assert np.allclose(np.sort(np.linalg.eigvalsh(U[k])), np.sort([a, b, g]), atol=1e-14)
        assert np.isclose(np.linalg.det(U[k]), a * b * g, rtol=1e-14)


def test_variant_axes_are_principal_axes():
    a, b, g = 1.0424, 0.9178, 1.0619
    U = M.stretch_tensors(a, b, g)
    R = M.variant_axes()
    for k in range(1, 7):
        assert np.allclose(R[k].T @ R[k], np.eye(3), atol=1e-15)
        assert np.allclose(U[k] @ R[k], R[k] @ np.diag([a, b, g]), atol=1e-14)


def test_paper_matrices_with_identity_rotation():
    """Q = I reproduces the printed U_1 (Sec. 4.1) entry by entry."""
    mp = synth.MaterialParams(**synth.PAPER_STRETCHES)
    card = M.Card(mp)
    a, b, g = 1.0619, 0.9178, 1.0230
    U1 = np.array([[(a + g) / 2, 0, (a - g) / 2], [0, b, 0], [(a - g) / 2, 0, (a + g) / 2]])
    U6 = np.array([[b, 0, 0], [0, (a + g) / 2, -(a - g) / 2], [0, -(a - g) / 2, (a + g) / 2]])
    assert np.allclose(card.U[1], U1, atol=1e-15)
    assert np.allclose(card.U[6], U6, atol=1e-15)


def _symmetries(L):
    assert np.allclose(L, L.transpose(1, 0, 2, 3))
    assert np.allclose(L, L.transpose(0, 1, 3, 2))
    assert np.allclose(L, L.transpose(2, 3, 0, 1))


def test_stiffness_symmetries_and_table_values():
    mp = synth.config_material()
    card = M.Card(mp)
    for k in range(7):
        _symmetries(card.L[k])
    L0 = M.cubic_stiffness(142.0, 126.0, 96.0)
    assert L0[0, 0, 0, 0] == 142.0 and L0[0, 0, 1, 1] == 126.0 and L0[1, 2, 1, 2] == 96.0
    Lm = M.orthorhombic_stiffness(*mp.ortho)
    assert Lm[2, 2, 2, 2] == 205.0 and Lm[0, 2, 0, 2] == 19.7 and Lm[1, 1, 2, 2] == 115.0


def test_orthorhombic_invariant_under_axis_flips():
    Lm = M.orthorhombic_stiffness(*synth.MaterialParams().ortho)
    for s in ([-1, 1, 1], [1, -1, 1], [1, 1, -1]):
        assert np.allclose(M.rotate4(Lm, np.diag(s)), Lm)


def test_isotropic_stiffness_rotation_invariant():
    lam, mu = 70.0, 30.0
    Liso = M.cubic_stiffness(lam + 2 * mu, lam, mu)
    Q = synth.random_rotation(12345)
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-14)
    assert np.isclose(np.linalg.det(Q), 1.0)
    assert np.allclose(M.rotate4(Liso, Q), Liso, atol=1e-12)


def test_voigt_round_trip():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 6))
    C6 = A + A.T
    L = M.voigt_to_tensor(C6)
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    back = np.array([[L[idx[p][0], idx[p][1], idx[q][0], idx[q][1]] for q in range(6)]
                     for p in range(6)])
    assert np.array_equal(back, C6)


def test_sample_frame_rotation():
    """With [011] along z, the rotated card equals R * card_cubic."""
    mp = synth.config_material()
    Q = np.asarray(mp.Q).reshape(3, 3)
    assert np.allclose(Q @ Q.T, np.eye(3)) and np.isclose(np.linalg.det(Q), 1.0)
    assert np.allclose(Q @ (np.array([0, 1, 1]) / np.sqrt(2)), [0, 0, 1])
    card = M.Card(mp)
    cub = M.Card(synth.MaterialParams())
    for k in range(7):
        assert np.allclose(card.U[k], Q @ cub.U[k] @ Q.T)
        assert np.allclose(card.L[k], M.rotate4(cub.L[k], Q))


def test_splitmix64_published_sequence():
    """splitmix64 seeded with 0 yields e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f; its state advances by the golden-ratio increment."""
    gold = 0x9E3779B97F4A7C15
    xs = np.array([0, gold, (2 * gold) % 2 ** 64], dtype=np.uint64)
    out = [int(v) for v in synth.splitmix64(xs)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    e = synth.initial_eta(synth.BASE_SEED, 1000)
    assert e.shape == (1000, 6) and e.min() >= 0.0 and e.max() < 0.05
    assert abs(e.mean() - 0.025) < 0.002


def test_variant_stiffness_axes_in_sample_frame():
    """Reading of Table 1: variant k's orthorhombic axes 1, 2, 3 are the
    eigenvectors of its stretch tensor for alpha, beta, gamma.  In the sample
    frame (with [011] along z) the normal stiffness along each axis n,
    (n n) : L_k : (n n), is c11 = 189, c22 = 141, c33 = 205 GPa, the mixed
    normal terms are c12, c13, c23, and the shear stiffness of each axis pair
    (sym(a b) : L_k : sym(b a) with sym(a b) = (a b + b a)/2) is c66 (alpha-beta),
    c55 (alpha-gamma), c44 (beta-gamma).  The axes come from the eigenvectors
    of the sample-frame U_k, so a transposed rotation of the stiffness fails."""
    mp = synth.config_material()
    card = M.Card(mp)
    c11, c22, c33, c44, c55, c66, c12, c13, c23 = mp.ortho
    for k in range(1, 7):
        w, v = np.linalg.eigh(card.U[k])
        axis = {s: v[:, int(np.argmin(np.abs(w - s)))] for s in (mp.alpha, mp.beta, mp.gamma)}
        na, nb, ng = axis[mp.alpha], axis[mp.beta], axis[mp.gamma]
        L = card.L[k]

        def q(A, B):
            return float(np.einsum("ij,ijkl,kl->", A, L, B))

        def nn(n):
            return np.outer(n, n)

        def sym(x, y):
            return 0.5 * (np.outer(x, y) + np.outer(y, x))

        assert np.isclose(q(nn(na), nn(na)), c11, rtol=1e-12)
        assert np.isclose(q(nn(nb), nn(nb)), c22, rtol=1e-12)
        assert np.isclose(q(nn(ng), nn(ng)), c33, rtol=1e-12)
        assert np.isclose(q(nn(na), nn(nb)), c12, rtol=1e-12)
        assert np.isclose(q(nn(na), nn(ng)), c13, rtol=1e-12)
        assert np.isclose(q(nn(nb), nn(ng)), c23, rtol=1e-12)
        assert np.isclose(q(sym(na, nb), sym(na, nb)), c66, rtol=1e-12)
        assert np.isclose(q(sym(na, ng), sym(na, ng)), c55, rtol=1e-12)
        assert np.isclose(q(sym(nb, ng), sym(nb, ng)), c44, rtol=1e-12)
    # the austenite keeps its cubic constants along the crystal axes
    Qm = np.asarray(mp.Q).reshape(3, 3)
    e1 = Qm @ np.array([1.0, 0.0, 0.0])
    assert np.isclose(np.einsum("i,j,ijkl,k,l->", e1, e1, card.L[0], e1, e1), mp.cubic[0], rtol=1e-12)
