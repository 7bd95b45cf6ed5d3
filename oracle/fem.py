"""Structured Q1 hexahedral discretisation and the discrete potential.

Oracle (test infrastructure only; see the package docstring).

Discretisation (Sec. 3.3, Eq. FEapprox): equal-order interpolation of the
displacement u = phi - X and of the condensed order parameters eta_hat, with
the same nodal basis for both.  The paper uses linear tetrahedra; the workloads
here use trilinear (Q1) hexahedra on a uniform grid of cubes of side h, with
2x2x2 Gauss-Legendre quadrature for every term of the potential.

Degrees of freedom are node-interleaved, 9 per node:
  [u_x, u_y, u_z, eta_1, ..., eta_6]
and nodes are numbered lexicographically with x fastest:
  node(i, j, k) = i + (nx+1) * (j + (ny+1) * k).
Element (ei, ej, ek) has local node a = ax + 2 ay + 4 az at
(ei+ax, ej+ay, ek+az).

Residual and tangent (Sec. 3.4): with the discrete potential
Pi(U) = sum_e Pi_e(U_e), R = dPi/dU and K = d^2 Pi / dU^2, both obtained here
by automatic differentiation of the element potential, as the paper obtains
them from UFL.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import grad, hessian, vmap

from . import energy
from .energy import DT

# unknowns per node and variants of the six-variant card; a card of N
# variants has 3 + N unknowns per node (Discretisation.ndof)
NDOF = 9
NETA = 6


class Mesh:
    """nx*ny*nz cubes of side h; node and element index helpers."""

    def __init__(self, nx: int, ny: int, nz: int, h: float):
        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h)
        self.nnx, self.nny, self.nnz = self.nx + 1, self.ny + 1, self.nz + 1
        self.n_nodes = self.nnx * self.nny * self.nnz
        self.n_elem = self.nx * self.ny * self.nz

    @classmethod
    def from_problem(cls, p, level: int = 0) -> "Mesh":
        f = 2 ** level
        if p.nx % f or p.ny % f or p.nz % f:
            raise ValueError("mesh not divisible for the requested level")
        hx, hy, hz = p.lx / p.nx, p.ly / p.ny, p.lz / p.nz
        if not (np.isclose(hx, hy) and np.isclose(hx, hz)):
            raise ValueError("elements must be cubes")
        return cls(p.nx // f, p.ny // f, p.nz // f, hx * f)

    def node_id(self, i, j, k):
        return i + self.nnx * (j + self.nny * k)

    def node_ijk(self, n):
        n = np.asarray(n)
        return n % self.nnx, (n // self.nnx) % self.nny, n // (self.nnx * self.nny)

    def element_ijk(self, e):
        e = np.asarray(e)
        return e % self.nx, (e // self.nx) % self.ny, e // (self.nx * self.ny)

    def element_nodes(self, elems=None) -> np.ndarray:
        """(n_sel, 8) global node ids of the selected (default: all) elements."""
        if elems is None:
            elems = np.arange(self.n_elem)
        ei, ej, ek = self.element_ijk(elems)
        out = np.empty((len(elems), 8), dtype=np.int64)
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            out[:, a] = self.node_id(ei + ax, ej + ay, ek + az)
        return out

    def elements_of_nodes(self, nodes) -> np.ndarray:
        """Sorted ids of all elements touching any of ``nodes``."""
        i, j, k = self.node_ijk(np.asarray(nodes))
        sel = []
        for dz in (-1, 0):
            for dy in (-1, 0):
                for dx in (-1, 0):
                    ei, ej, ek = i + dx, j + dy, k + dz
                    ok = (ei >= 0) & (ei < self.nx) & (ej >= 0) & (ej < self.ny) \
                        & (ek >= 0) & (ek < self.nz)
                    sel.append((ei + self.nx * (ej + self.ny * ek))[ok])
        return np.unique(np.concatenate(sel))


def gauss_tables(h: float):
    """Shape values N[g,a], physical gradients dN[g,a,d] and weights w[g]
    for 2x2x2 Gauss-Legendre points on a cube of side h.

    Reference cube [0,1]^3: N_a = prod_d (xi_d if a_d else 1 - xi_d);
    Gauss abscissae (1 -+ 1/sqrt3)/2, weights 1/8 each (times h^3).
    """
    q = [0.5 * (1.0 - 1.0 / np.sqrt(3.0)), 0.5 * (1.0 + 1.0 / np.sqrt(3.0))]
    N = np.zeros((8, 8))
    dN = np.zeros((8, 8, 3))
    for g in range(8):
        xi = (q[g & 1], q[(g >> 1) & 1], q[(g >> 2) & 1])
        for a in range(8):
            bits = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
            f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(3)]
            df = [1.0 if bits[d] else -1.0 for d in range(3)]
            N[g, a] = f[0] * f[1] * f[2]
            dN[g, a, 0] = df[0] * f[1] * f[2] / h
            dN[g, a, 1] = f[0] * df[1] * f[2] / h
            dN[g, a, 2] = f[0] * f[1] * df[2] / h
    w = np.full(8, h ** 3 / 8.0)
    return N, dN, w


class Discretisation:
    """Element potential, residual and tangent on one mesh."""

    def __init__(self, mesh: Mesh, card, chunk: int = 1024):
        self.mesh = mesh
        self.tc = energy.TorchCard(card)
        self.nv = int(card.U.shape[0]) - 1   # variants N
        self.ndof = 3 + self.nv              # unknowns per node
        N, dN, w = gauss_tables(mesh.h)
        self.N = torch.as_tensor(N, dtype=DT)
        self.dN = torch.as_tensor(dN, dtype=DT)
        self.w = torch.as_tensor(w, dtype=DT)
        self.chunk = int(chunk)

    def element_potential(self, d: torch.Tensor, eta_n: torch.Tensor) -> torch.Tensor:
        """Pi_e for one element: d (8, 9) nodal unknowns, eta_n (8, 6) previous
        order parameters.  Sum over Gauss points of w_g * psi(x_g)."""
        u = d[:, :3]
        eh = d[:, 3:]
        I = torch.eye(3, dtype=DT)
        F = I + torch.einsum("ai,gaj->gij", u, self.dN)
        eta_g = self.N @ eh
        geta_g = torch.einsum("ak,gaj->gkj", eh, self.dN)
        etan_g = self.N @ eta_n
        psi = energy.density(F, eta_g, geta_g, etan_g, self.tc)
        return (self.w * psi).sum()

    def _gather(self, U: np.ndarray, Eta_n: np.ndarray, elems):
        energy.check_log_range(U.reshape(-1, self.ndof)[:, 3:], self.tc)
        en = self.mesh.element_nodes(elems)
        d = torch.as_tensor(U.reshape(-1, self.ndof)[en], dtype=DT)
        dn = torch.as_tensor(Eta_n.reshape(-1, self.nv)[en], dtype=DT)
        return en, d, dn

    def element_residuals(self, U, Eta_n, elems):
        en, d, dn = self._gather(U, Eta_n, elems)
        return en, vmap(grad(self.element_potential))(d, dn).reshape(len(en), 8 * self.ndof).numpy()

    def element_tangents(self, U, Eta_n, elems):
        en, d, dn = self._gather(U, Eta_n, elems)
        K = vmap(hessian(self.element_potential))(d, dn)
        m = 8 * self.ndof
        return en, K.reshape(len(en), m, m).numpy()

    def potential(self, U, Eta_n) -> float:
        en, d, dn = self._gather(U, Eta_n, np.arange(self.mesh.n_elem))
        return float(vmap(self.element_potential)(d, dn).sum())

    def residual(self, U: np.ndarray, Eta_n: np.ndarray, elems=None) -> np.ndarray:
        """Global R = dPi/dU (unconstrained), node-interleaved, length 9*n_nodes.
        With ``elems`` only those elements' contributions are summed."""
        if elems is None:
            elems = np.arange(self.mesh.n_elem)
        nd, m = self.ndof, 8 * self.ndof
        R = np.zeros(self.mesh.n_nodes * nd)
        for s in range(0, len(elems), self.chunk):
            en, Re = self.element_residuals(U, Eta_n, elems[s:s + self.chunk])
            dofs = (en[:, :, None] * nd + np.arange(nd)).reshape(len(en), m)
            np.add.at(R, dofs.ravel(), Re.ravel())
        return R

    def tangent_coo(self, U: np.ndarray, Eta_n: np.ndarray, elems=None):
        """COO triplets of K = d^2 Pi / dU^2 (unconstrained)."""
        if elems is None:
            elems = np.arange(self.mesh.n_elem)
        rows, cols, vals = [], [], []
        nd, m = self.ndof, 8 * self.ndof
        for s in range(0, len(elems), self.chunk):
            en, Ke = self.element_tangents(U, Eta_n, elems[s:s + self.chunk])
            dofs = (en[:, :, None] * nd + np.arange(nd)).reshape(len(en), m)
            rows.append(np.repeat(dofs, m, axis=1).ravel())
            cols.append(np.tile(dofs, (1, m)).ravel())
            vals.append(Ke.ravel())
        return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
