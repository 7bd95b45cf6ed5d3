"""Frictionless penalty contact with a rigid spherical indenter.

Oracle (test infrastructure only; see the package docstring).

What is computed (Sec. 2.4, Eqs. Ngap and PenPot; Sec. 4.1 for the indenter):
the potential contact surface is the top face z = nz h of the reference
configuration; the indenter is a rigid sphere of radius R centred above the
centre of the top face, pushed to depth d:

    c = (nx h / 2, ny h / 2, nz h + R - d).

For a surface point X with current position x = X + u(X), the closest-point
projection onto the sphere gives the normal gap and the sphere's normal

    g_N = |x - c| - R,      n = (x - c) / |x - c|            (Eq. Ngap)

and the penalty regularisation of the impenetrability condition adds

    Pi_c = int_{Gamma_c} 1/2 eps_N <g_N>_-^2 dS              (Eq. PenPot)

to the global potential, <x>_- = min(x, 0).  On each top face u is the
bilinear interpolation of its four nodes' displacements and the integral is
taken by 2x2 Gauss-Legendre points (weights h^2 / 4).  The contact residual
and tangent are the first and second derivatives of Pi_c with respect to the
nodal displacements, by automatic differentiation as for the bulk terms.

The indentation load is the force conjugate to the depth,

    P = dPi_c / dd  (at fixed u),

also by automatic differentiation (with dg_N/dd = n_z it is
int eps_N <g_N>_- n_z dS, non-negative under a pressing indenter).
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import grad, hessian, vmap

from .energy import DT
from .fem import Mesh


def face_gauss():
    """Bilinear shape values N[g, a] at the 2x2 Gauss points of the unit
    square (a = ax + 2 ay) and the unit-square weights (1/4 each)."""
    q = [0.5 * (1.0 - 1.0 / np.sqrt(3.0)), 0.5 * (1.0 + 1.0 / np.sqrt(3.0))]
    N = np.zeros((4, 4))
    for g in range(4):
        xi, et = q[g & 1], q[(g >> 1) & 1]
        for a in range(4):
            N[g, a] = (xi if a & 1 else 1.0 - xi) * (et if a & 2 else 1.0 - et)
    return N, np.full(4, 0.25)


class SphereContact:
    """Penalty contact of the top face with a rigid sphere on one mesh."""

    def __init__(self, mesh: Mesh, radius: float, eps_n: float):
        self.mesh = mesh
        self.R = float(radius)
        self.eps = float(eps_n)
        N, w = face_gauss()
        self.N = torch.as_tensor(N, dtype=DT)
        self.w = torch.as_tensor(w * mesh.h * mesh.h, dtype=DT)
        m = mesh
        fi, fj = np.meshgrid(np.arange(m.nx), np.arange(m.ny), indexing="ij")
        fi, fj = fi.T.ravel(), fj.T.ravel()  # faces in x-fastest order
        nodes = np.empty((len(fi), 4), dtype=np.int64)
        for a in range(4):
            nodes[:, a] = m.node_id(fi + (a & 1), fj + ((a >> 1) & 1), m.nz)
        self.face_nodes = nodes
        X = np.stack([(fi[:, None] + (np.arange(4) & 1)[None, :]) * m.h,
                      (fj[:, None] + ((np.arange(4) >> 1) & 1)[None, :]) * m.h,
                      np.full((len(fi), 4), m.nz * m.h)], axis=2)
        self.X = torch.as_tensor(X, dtype=DT)  # (faces, 4, 3)

    def centre(self, depth):
        m = self.mesh
        return torch.stack([torch.as_tensor(0.5 * m.nx * m.h, dtype=DT),
                            torch.as_tensor(0.5 * m.ny * m.h, dtype=DT),
                            m.nz * m.h + self.R - depth])

    def face_energy(self, u: torch.Tensor, X: torch.Tensor, depth: torch.Tensor) -> torch.Tensor:
        """Pi_c of one face: u, X (4, 3) nodal displacements and positions."""
        x = self.N @ (X + u)                     # (4 Gauss points, 3)
        gN = torch.linalg.norm(x - self.centre(depth), dim=1) - self.R
        neg = torch.clamp(gN, max=0.0)
        return (self.w * 0.5 * self.eps * neg * neg).sum()

    def _u_faces(self, U: np.ndarray) -> torch.Tensor:
        return torch.as_tensor(U.reshape(self.mesh.n_nodes, -1)[self.face_nodes][:, :, :3], dtype=DT)

    def energy(self, U: np.ndarray, depth: float) -> float:
        d = torch.as_tensor(depth, dtype=DT)
        e = vmap(self.face_energy, in_dims=(0, 0, None))(self._u_faces(U), self.X, d)
        return float(e.sum())

    def residual(self, U: np.ndarray, depth: float) -> np.ndarray:
        """dPi_c/dU, node-interleaved (only top-face u components nonzero)."""
        d = torch.as_tensor(depth, dtype=DT)
        Gf = vmap(grad(self.face_energy), in_dims=(0, 0, None))(self._u_faces(U), self.X, d).numpy()
        nd = U.size // self.mesh.n_nodes
        R = np.zeros(self.mesh.n_nodes * nd)
        dofs = self.face_nodes[:, :, None] * nd + np.arange(3)
        np.add.at(R, dofs.ravel(), Gf.ravel())
        return R

    def tangent_coo(self, U: np.ndarray, depth: float):
        """COO triplets of d^2 Pi_c / dU^2."""
        d = torch.as_tensor(depth, dtype=DT)
        Hf = vmap(hessian(self.face_energy), in_dims=(0, 0, None))(self._u_faces(U), self.X, d)
        Hf = Hf.reshape(len(self.face_nodes), 12, 12).numpy()
        nd = U.size // self.mesh.n_nodes
        dofs = (self.face_nodes[:, :, None] * nd + np.arange(3)).reshape(-1, 12)
        rows = np.repeat(dofs, 12, axis=1).ravel()
        cols = np.tile(dofs, (1, 12)).ravel()
        return rows, cols, Hf.ravel()

    def load(self, U: np.ndarray, depth: float) -> float:
        """Indentation load P = dPi_c/dd at fixed displacements."""
        d = torch.as_tensor(depth, dtype=DT)
        uf = self._u_faces(U)
        dfun = grad(lambda dd: vmap(self.face_energy, in_dims=(0, 0, None))(uf, self.X, dd).sum())
        return float(dfun(d))

