"""Local density of the penalised incremental potential.

Oracle (test infrastructure only; see the package docstring).

psi(F, eta_hat, grad eta_hat; eta_hat_n) is the integrand of the penalised
global incremental potential (Eq. PenPot, Sec. 3.1) without its contact term
(the external-load potential is zero, Sec. 2.3):

  chemical      sum_i eta_i F_i^0                               (Sec. 2.2)
  elastic       1/2 det(F^t) H^e : L(eta) H^e                   (Eq. elasticEn)
                F^t = sum_i eta_i U_i                           (Eq. LinMix)
                or F^t = exp(sum_i eta_i log U_i)   (logarithmic mixing, Sec. 2.1)
                F^e = F (F^t)^-1,  C^e = (F^e)^T F^e
                H^e = Pade approximant of 1/2 log C^e           (Eqs. pade11/22/33)
                L(eta) = sum_i eta_i L_i
  interface     sum_{i<j} w_ij (eta_i eta_j - l_ij^2 grad eta_i . grad eta_j)
                with w_ij = 4 gamma_ij / (pi l_ij)              (Eq. IntEnergy)
  dissipation   sum_i (rho_i/2) (eta_i - eta_{i,n})^2, rho_i = 1/(m_i tau)
                (backward-Euler incremental dissipation, Sec. 2.3)
  penalty       sum_i (eps/2) <eta_i>_-^2, <x>_- = min(x, 0)    (Eq. PenPot)

with eta_0 = 1 - sum_{i>=1} eta_i and grad eta_0 = -sum grad eta_i
(condensation, Sec. 3.1).  The constant -E_n of Eq. GlobIncPot is dropped: it
does not change the residual or the tangent.

All functions take batched PyTorch float64 tensors and are differentiable to
second order, so residual and tangent follow by automatic differentiation as in
the paper (Sec. 3.4).
"""
from __future__ import annotations

import torch

DT = torch.float64


def _eye(like: torch.Tensor) -> torch.Tensor:
    return torch.eye(3, dtype=like.dtype, device=like.device).expand(like.shape)


def pade_half_log(C: torch.Tensor, order: int = 22) -> torch.Tensor:
    """Pade approximant of 1/2 log C for a batch of SPD 3x3 matrices.

    (1,1): (C - I)(C + I)^-1                                    Eq. pade11
    (2,2): 3/2 (C^2 - I)(C^2 + 4C + I)^-1                       Eq. pade22
    (3,3): 1/6 (11C^3 + 27C^2 - 27C - 11I)(C^3 + 9C^2 + 9C + I)^-1   Eq. pade33
    """
    I = _eye(C)
    if order == 11:
        return (C - I) @ torch.linalg.inv(C + I)
    C2 = C @ C
    if order == 22:
        return 1.5 * (C2 - I) @ torch.linalg.inv(C2 + 4.0 * C + I)
    if order == 33:
        C3 = C2 @ C
        num = 11.0 * C3 + 27.0 * C2 - 27.0 * C - 11.0 * I
        den = C3 + 9.0 * C2 + 9.0 * C + I
        return num @ torch.linalg.inv(den) / 6.0
    raise ValueError(f"unknown Pade order {order}")


def full_eta(eta_hat: torch.Tensor) -> torch.Tensor:
    """(eta_0, eta_1..eta_N) from the condensed vector (Sec. 3.1)."""
    return torch.cat([1.0 - eta_hat.sum(-1, keepdim=True), eta_hat], dim=-1)


def full_grad_eta(grad_eta_hat: torch.Tensor) -> torch.Tensor:
    """Gradients (..., N+1, 3) with grad eta_0 = -sum grad eta_i."""
    return torch.cat([-grad_eta_hat.sum(-2, keepdim=True), grad_eta_hat], dim=-2)


class TorchCard:
    """The material card as float64 tensors."""

    def __init__(self, card):
        self.U = torch.as_tensor(card.U, dtype=DT)
        self.L = torch.as_tensor(card.L, dtype=DT)
        self.F0 = torch.as_tensor(card.F0, dtype=DT)
        self.W = torch.as_tensor(card.W, dtype=DT)
        self.ell2 = torch.as_tensor(card.ell2, dtype=DT)
        self.rho = torch.as_tensor(card.rho, dtype=DT)
        self.eps = float(card.eps)
        self.pade = int(card.pade)
        self.mixing = getattr(card, "mixing", "linear")
        self.logU = torch.as_tensor(card.logU, dtype=DT) if self.mixing == "log" else None


EXP_TERMS = 30


def expm_series(M: torch.Tensor) -> torch.Tensor:
    """exp(M) by its defining power series sum_{n <= 30} M^n / n!.  For
    ||M||_F <= 1 the omitted tail is below 1/31! ~ 1e-34, so the result is
    exact up to rounding (callers check the range: check_log_range)."""
    term = torch.eye(3, dtype=M.dtype).expand(M.shape)
    out = term
    for n in range(1, EXP_TERMS + 1):
        term = term @ M / n
        out = out + term
    return out


def check_log_range(eta_hat_nodal, tc: TorchCard) -> None:
    """The logarithmic mixing argument M = sum_k eta_k log U_k stays within
    expm_series' range ||M||_F <= 1 at every Gauss point if it does at the
    nodes: Q1 interpolation takes convex combinations of nodal values, so
    sum_k |eta_k| ||log U_k||_F at a Gauss point is at most its largest
    nodal value (eta_0 carries log U_0 = 0)."""
    if tc.mixing != "log":
        return
    import numpy as np
    norms = torch.linalg.matrix_norm(tc.logU[1:]).numpy()
    bound = float(np.max(np.abs(np.asarray(eta_hat_nodal)) @ norms)) if np.size(eta_hat_nodal) else 0.0
    if bound > 1.0:
        raise ValueError(f"log mixing: sum |eta| ||log U|| reaches {bound:.3f} > 1, outside the oracle's range")


def transformation_gradient(eta: torch.Tensor, tc: TorchCard) -> torch.Tensor:
    """F^t = sum_i eta_i U_i (Eq. LinMix), or with logarithmic mixing
    F^t = exp(sum_i eta_i log U_i) (Sec. 2.1)."""
    if tc.mixing == "log":
        return expm_series(torch.einsum("...i,ijk->...jk", eta, tc.logU))
    return torch.einsum("...i,ijk->...jk", eta, tc.U)


def hencky_elastic_strain(F: torch.Tensor, eta: torch.Tensor, tc: TorchCard) -> torch.Tensor:
    Ft = transformation_gradient(eta, tc)
    Fe = F @ torch.linalg.inv(Ft)
    Ce = Fe.transpose(-1, -2) @ Fe
    return pade_half_log(Ce, tc.pade)


def elastic_energy(F: torch.Tensor, eta: torch.Tensor, tc: TorchCard) -> torch.Tensor:
    """1/2 det(F^t) H^e : L(eta) H^e (Eq. elasticEn)."""
    Ft = transformation_gradient(eta, tc)
    Jt = torch.linalg.det(Ft)
    He = hencky_elastic_strain(F, eta, tc)
    L = torch.einsum("...i,iabcd->...abcd", eta, tc.L)
    return 0.5 * Jt * torch.einsum("...ab,...abcd,...cd->...", He, L, He)


def neg_part(x: torch.Tensor) -> torch.Tensor:
    """<x>_- = x if x < 0 else 0 (strict test: zero slope at x = 0)."""
    return torch.where(x < 0, x, torch.zeros_like(x))


def density(F, eta_hat, grad_eta_hat, eta_hat_n, tc: TorchCard) -> torch.Tensor:
    """psi for batches: F (...,3,3), eta_hat (...,N), grad_eta_hat (...,N,3),
    eta_hat_n (...,N).  Returns (...)."""
    eta = full_eta(eta_hat)
    eta_n = full_eta(eta_hat_n)
    geta = full_grad_eta(grad_eta_hat)
    chem = (eta * tc.F0).sum(-1)
    el = elastic_energy(F, eta, tc)
    # sum_{i<j} = 1/2 sum_{i != j}; W has a zero diagonal.
    inter = 0.5 * torch.einsum("...i,ij,...j->...", eta, tc.W, eta) \
        - 0.5 * torch.einsum("...ia,ij,...ja->...", geta, tc.W * tc.ell2, geta)
    diss = 0.5 * (tc.rho * (eta - eta_n) ** 2).sum(-1)
    pen = 0.5 * tc.eps * (neg_part(eta) ** 2).sum(-1)
    return chem + el + inter + diss + pen
