"""Pins of the oracle's local density (Sec. 2.2-2.3, 3.1-3.2)."""
import numpy as np
import pytest
import torch
from torch.func import grad, hessian

import synth
from oracle import energy as E
from oracle.material import Card

DT = torch.float64


def _tc(**over):
    return E.TorchCard(Card(synth.config_material(**over)))


def _rand_spd(rng, lo, hi):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    lam = rng.uniform(lo, hi, 3)
    return Q @ np.diag(lam) @ Q.T, lam, Q


def _r(order, c):
    I = torch.eye(3, dtype=DT)
    return float(E.pade_half_log(torch.as_tensor(c, dtype=DT) * I, order)[0, 0])


@pytest.mark.parametrize("order,power,const,xs", [
    (11, 3, 1 / 24, (1e-2, 2e-2)),
    (22, 5, 1 / 360, (1e-2, 2e-2)),
    (33, 7, 1 / 5600, (3e-2, 5e-2))])
def test_pade_taylor_order(order, power, const, xs):
    """The (k,k) approximant matches 1/2 ln c through (c-1)^(2k); the leading
    error term is const*(c-1)^(2k+1), const = (k!)^4 / (2 (2k)! (2k+1)!)
    (Pade table of ln(1+x), halved).  Averaging x and -x cancels the next,
    even-power term."""
    for x in xs:
        ratios = [(0.5 * np.log1p(t) - _r(order, 1.0 + t)) / t ** power for t in (x, -x)]
        assert abs(0.5 * sum(ratios) - const) < 0.05 * const


def test_pade22_error_table():
    cs = np.linspace(0.9, 1.1, 41)
    assert max(abs(_r(22, c) - 0.5 * np.log(c)) for c in cs) < 3.7e-8
    assert abs(_r(22, 0.5) - 0.5 * np.log(0.5)) < 4.3e-4
    assert abs(_r(22, 2.0) - 0.5 * np.log(2.0)) < 4.3e-4


@pytest.mark.parametrize("order", [11, 22, 33])
def test_pade_matrix_identities(order):
    rng = np.random.default_rng(1)
    I = torch.eye(3, dtype=DT)
    assert torch.count_nonzero(E.pade_half_log(I, order)) == 0
    C, lam, Qe = _rand_spd(rng, 0.7, 1.4)
    Ct = torch.as_tensor(C, dtype=DT)
    H = E.pade_half_log(Ct, order).numpy()
    Hinv = E.pade_half_log(torch.linalg.inv(Ct), order).numpy()
    assert np.allclose(H, -Hinv, atol=1e-14)
    R = synth.random_rotation(77)
    HR = E.pade_half_log(torch.as_tensor(R @ C @ R.T, dtype=DT), order).numpy()
    assert np.allclose(HR, R @ H @ R.T, atol=1e-14)
    # isotropic matrix function: same eigenvectors, scalar map on eigenvalues
    rl = np.array([_r(order, l) for l in lam])
    assert np.allclose(H, Qe @ np.diag(rl) @ Qe.T, atol=1e-14)


def test_pade22_vs_spectral_log():
    rng = np.random.default_rng(2)
    for _ in range(5):
        C, lam, Qe = _rand_spd(rng, 0.9, 1.1)
        H = E.pade_half_log(torch.as_tensor(C, dtype=DT), 22).numpy()
        Hex = Qe @ np.diag(0.5 * np.log(lam)) @ Qe.T
        bound = max(abs(_r(22, l) - 0.5 * np.log(l)) for l in lam)
        assert np.max(np.abs(np.linalg.eigvalsh(H - Hex))) <= bound * 1.0001 + 1e-15


def _state(rng, amp=0.03):
    F = torch.as_tensor(np.eye(3) + amp * rng.standard_normal((3, 3)), dtype=DT)
    eh = torch.as_tensor(rng.uniform(0.02, 0.1, 6), dtype=DT)
    geh = torch.as_tensor(0.1 * rng.standard_normal((6, 3)), dtype=DT)
    ehn = torch.as_tensor(rng.uniform(0.0, 0.1, 6), dtype=DT)
    return F, eh, geh, ehn


def test_pure_rotation_zero_hencky_and_stress():
    tc = _tc()
    R = torch.as_tensor(synth.random_rotation(5), dtype=DT)
    eta = E.full_eta(torch.zeros(6, dtype=DT))
    He = E.hencky_elastic_strain(R, eta, tc)
    assert float(He.abs().max()) < 1e-14
    P = grad(lambda F: E.elastic_energy(F, eta, tc))(R)
    assert float(P.abs().max()) < 1e-12


def test_stress_free_transformed_state():
    """F = R F^t(eta): elastic part vanishes, so P = dpsi/dF = 0."""
    tc = _tc()
    rng = np.random.default_rng(3)
    eh = torch.as_tensor(rng.uniform(0.0, 0.2, 6), dtype=DT)
    eta = E.full_eta(eh)
    R = torch.as_tensor(synth.random_rotation(6), dtype=DT)
    F = R @ E.transformation_gradient(eta, tc)
    P = grad(lambda F: E.elastic_energy(F, eta, tc))(F)
    assert float(P.abs().max()) < 1e-11
    assert abs(float(E.elastic_energy(F, eta, tc))) < 1e-25


def test_objectivity():
    tc = _tc()
    rng = np.random.default_rng(4)
    F, eh, geh, ehn = _state(rng, 0.05)
    R = torch.as_tensor(synth.random_rotation(9), dtype=DT)
    a = float(E.density(F, eh, geh, ehn, tc))
    b = float(E.density(R @ F, eh, geh, ehn, tc))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_small_strain_limit():
    """At F = I, eta = austenite: d^2 psi / dF dF = L_0 (linear elasticity)."""
    tc = _tc()
    eta = E.full_eta(torch.zeros(6, dtype=DT))
    Hs = hessian(lambda F: E.elastic_energy(F, eta, tc))(torch.eye(3, dtype=DT))
    assert np.allclose(Hs.numpy(), tc.L[0].numpy(), atol=1e-10)


def test_ad_matches_central_differences():
    tc = _tc()
    rng = np.random.default_rng(5)
    F, eh, geh, ehn = _state(rng)

    def f(x):
        return E.density(x[:9].reshape(3, 3), x[9:15], x[15:].reshape(6, 3), ehn, tc)

    x0 = torch.cat([F.ravel(), eh, geh.ravel()])
    g = grad(f)(x0).numpy()
    H = hessian(f)(x0).numpy()
    assert np.allclose(H, H.T, atol=1e-10)
    h = 1e-5
    for i in range(len(x0)):
        e = torch.zeros_like(x0)
        e[i] = h
        fd = (float(f(x0 + e)) - float(f(x0 - e))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i]))
        gd = (grad(f)(x0 + e) - grad(f)(x0 - e)).numpy() / (2 * h)
        assert np.allclose(gd, H[i], rtol=1e-6, atol=1e-6)


def test_order_parameter_driving_force_closed_form():
    """Stress-free state F = F^t(eta): the eta_hat-gradient of psi, derived by
    hand from the condensation eta_0 = 1 - sum eta_i (Sec. 3.1):
      F_k - F_0 + sum_j (w_kj - w_0j) eta_j + rho (d_k - d_0)
        + eps (<eta_k>_- - <eta_0>_-) ,   d_i = eta_i - eta_{i,n}."""
    mp = synth.config_material()
    tc = _tc()
    rng = np.random.default_rng(8)
    eh = rng.uniform(-0.02, 0.3, 6)
    ehn = rng.uniform(0.0, 0.1, 6)
    eta = np.concatenate([[1 - eh.sum()], eh])
    etan = np.concatenate([[1 - ehn.sum()], ehn])
    W = np.full((7, 7), mp.w_mm)
    W[0, :] = W[:, 0] = mp.w_am
    np.fill_diagonal(W, 0)
    neg = np.minimum(eta, 0)
    d = eta - etan
    expect = np.array([mp.F0[k] - mp.F0[0] + (W[k] - W[0]) @ eta + mp.rho * (d[k] - d[0])
                       + mp.eps_eta * (neg[k] - neg[0]) for k in range(1, 7)])
    Ft = E.transformation_gradient(E.full_eta(torch.as_tensor(eh, dtype=DT)), tc)

    def f(e):
        return E.density(Ft, e, torch.zeros(6, 3, dtype=DT), torch.as_tensor(ehn, dtype=DT), tc) \
            - E.elastic_energy(Ft, E.full_eta(e), tc)

    g = grad(f)(torch.as_tensor(eh, dtype=DT)).numpy()
    assert np.allclose(g, expect, rtol=1e-12, atol=1e-12)
    assert eta[0] < 0 or eh.min() < 0


def test_penalty_kink_has_zero_curvature_at_zero():
    x = torch.tensor([0.0, -1e-3, 1e-3], dtype=DT)
    f = lambda t: 0.5 * (E.neg_part(t) ** 2).sum()
    Hd = torch.diagonal(hessian(f)(x)).numpy()
    assert list(Hd) == [0.0, 1.0, 0.0]


def _scalar_pade(order, c):
    """Scalar forms of the Pade approximants of 1/2 ln c (Eqs. pade11, pade22,
    pade33 evaluated on c I)."""
    if order == 11:
        return (c - 1.0) / (c + 1.0)
    if order == 22:
        return 1.5 * (c * c - 1.0) / (c * c + 4.0 * c + 1.0)
    return (11 * c ** 3 + 27 * c * c - 27 * c - 11) / (6.0 * (c ** 3 + 9 * c * c + 9 * c + 1))


@pytest.mark.parametrize("order", [11, 22, 33])
def test_elastic_prefactor_and_stiffness_mixing(order):
    """Eq. elasticEn with the mixed stiffness L(eta) = sum eta_i L_i.  Along
    F = lam F^t(eta) the elastic stretch is lam I, so C^e = lam^2 I, H^e = r I
    with r the scalar approximant at lam^2, and
        psi_el = 1/2 det(F^t) r^2 sum_i eta_i (I : L_i : I).
    I : L : I is 3 c11 + 6 c12 = 1182 GPa for the cubic austenite and
    c11 + c22 + c33 + 2 (c12 + c13 + c23) = 1104 GPa for every martensite
    variant (Table 1; invariant under rotation).  On the edge between the
    austenite and variant k, F^t = I + t (U_k - I) has the eigenvalues
    1 + t (s - 1), s in {alpha, beta, gamma}, so det F^t is their product.
    Dropping det F^t, taking det F instead, or freezing L at L_0 all fail."""
    mp = synth.config_material(pade=order)
    tc = E.TorchCard(Card(mp))
    a, b, g = mp.alpha, mp.beta, mp.gamma
    lam = 1.03
    r = _scalar_pade(order, lam * lam)
    for k in (1, 4, 6):
        for t in (0.0, 0.37, 1.0):
            eh = torch.zeros(6, dtype=DT)
            eh[k - 1] = t
            eta = E.full_eta(eh)
            Jt = np.prod([1.0 + t * (s - 1.0) for s in (a, b, g)])
            F = lam * E.transformation_gradient(eta, tc)
            got = float(E.elastic_energy(F, eta, tc))
            want = 0.5 * Jt * r * r * ((1.0 - t) * 1182.0 + t * 1104.0)
            assert abs(got - want) <= 1e-12 * abs(want), (k, t, got, want)
    # an interior point of the simplex: two variants and the austenite
    eh = torch.zeros(6, dtype=DT)
    eh[1], eh[4] = 0.3, 0.25
    eta = E.full_eta(eh)
    Ft = E.transformation_gradient(eta, tc)
    Jt = float(np.prod(np.linalg.eigvalsh(Ft.numpy())))
    got = float(E.elastic_energy(lam * Ft, eta, tc))
    want = 0.5 * Jt * r * r * (0.45 * 1182.0 + 0.55 * 1104.0)
    assert abs(got - want) <= 1e-12 * abs(want)
