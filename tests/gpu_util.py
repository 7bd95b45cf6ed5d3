"""Shared setup for the GPU parity tests: seeded states and the oracle's
counterparts (oracle = CPU reference, test infrastructure only)."""
import os
import sys

import numpy as np

import synth
from oracle import solver as S
from oracle.fem import Discretisation, Mesh, NDOF
from oracle.material import Card


def say(msg):
    """Progress line naming the case, flushed before the GPU work starts."""
    print(msg, flush=True)
    sys.stdout.flush()


def seeded_state(p, u_amp=0.0, seed=7):
    """(U (n, 3 + N), Eta_n (n, N)): eta_hat from the problem seed
    (splitmix64), optional small random displacement field (numpy PCG64 with
    ``seed``)."""
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, 3 + p.n_var))
    U[:, 3:] = p.eta0()
    if u_amp:
        U[:, :3] = u_amp * np.random.default_rng(seed).standard_normal((m.n_nodes, 3))
    return U, U[:, 3:].copy()


def residual_abs(disc, U, En, elems=None):
    """Per-entry sum of the absolute element contributions to the residual,
    sum_e |R_e| (the rounding scale of the assembled sum: a node's element
    contributions cancel at equilibrium, so |R| alone understates it)."""
    if elems is None:
        elems = np.arange(disc.mesh.n_elem)
    nd = disc.ndof
    out = np.zeros(disc.mesh.n_nodes * nd)
    for s in range(0, len(elems), 4096):
        en, Re = disc.element_residuals(np.ravel(U), np.ravel(En), elems[s:s + 4096])
        dofs = (en[:, :, None] * nd + np.arange(nd)).reshape(len(en), 8 * nd)
        np.add.at(out, dofs.ravel(), np.abs(Re).ravel())
    return out


class OracleCase:
    """Oracle Newton system + multigrid for one problem/state/depth."""

    def __init__(self, p, U, En, depth, build_mg=True, direct=True, coarse="reassemble"):
        self.p = p
        self.card = Card(p.material)
        self.mesh = Mesh.from_problem(p)
        self.U, self.En = U, En
        self.mask, self.target = S.dirichlet(self.mesh, p.kind, p.patch, p.radius, depth=depth, ndof=3 + p.n_var)
        self.g = S.increment(self.mask, self.target, U)
        self.sys = S.NewtonSystem(p, self.card, U.ravel(), En.ravel(), self.mask, self.g, depth)
        self.mg = S.Multigrid(p, self.card, U.ravel(), En.ravel(), self.mask, K_fine=self.sys.K,
                              depth=depth, coarse=coarse) if build_mg else None
        self.x = S.direct_solve(self.sys.A, self.sys.b) if direct else None
        self.depth = depth
        self._scales = None

    def abs_scales(self):
        """(R_abs, b_abs): per-entry rounding scales of the residual and the
        right-hand side, sum_e |R_e| (+ |contact part|) and R_abs + |K| |g|
        (|g| on constrained dofs, where b = g exactly)."""
        if self._scales is None:
            sy = self.sys
            R_abs = residual_abs(sy.disc, self.U, self.En)
            if sy.contact is not None:
                R_abs = R_abs + np.abs(sy.contact.residual(self.U.ravel(), self.depth))
            m = self.mask.ravel()
            gv = np.where(m, self.g.ravel(), 0.0)
            b_abs = R_abs + abs(sy.K) @ np.abs(gv)
            b_abs[m] = np.abs(gv[m])
            self._scales = (R_abs, b_abs)
        return self._scales


def gpu_problem(p, U, En, precision="fp64", depth=0.0, **opts):
    from paper_2011_08802_amd import mvpf
    gp = mvpf.Problem(p, precision, **opts)
    gp.set_state(U[:, :3], U[:, 3:], En, depth)
    return gp


def rel(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_blocks(a, b, ndof=NDOF):
    """Relative errors of the displacement and order-parameter parts."""
    a = np.asarray(a).reshape(-1, ndof)
    b = np.asarray(b).reshape(-1, ndof)
    return rel(a[:, :3], b[:, :3]), rel(a[:, 3:], b[:, 3:])


def entry_errors(a, b, scale=None, ndof=NDOF):
    """Per-entry error ratios |a_i - b_i| / (|b_i| + s_i (+ c_i)), where s_i is
    the largest |b| among the 9 unknowns of entry i's node and c (optional)
    the entry's rounding scale: the sum of the absolute values of the terms
    that make it up, (|A| |x|)_i for a product A x, sum_e |R_e| for an
    assembled residual.  A computed sum of terms t_k differs from the exact
    one by at most (n eps) sum_k |t_k| (standard error analysis of summation,
    e.g. Higham, Accuracy and Stability of Numerical Algorithms, Sec. 4.2), so
    two correct evaluations in different orders agree to that scale."""
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    s = np.repeat(np.abs(b).reshape(-1, ndof).max(axis=1), ndof)
    den = np.abs(b) + s
    if scale is not None:
        den = den + np.abs(np.asarray(scale, dtype=float).ravel())
    return np.abs(a - b) / np.maximum(den, 1e-300)


def check_entries(a, b, tol, what, scale=None, ndof=NDOF):
    """Element-wise parity gate (see entry_errors): every entry within tol of
    the oracle's, relative to its node's scale.  On failure the worst entry
    (node, unknown, both values) is reported; the norm-wise relative errors of
    the displacement and order-parameter parts are printed as diagnostics."""
    e = entry_errors(a, b, scale, ndof)
    i = int(np.argmax(e))
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    ru, re = rel_blocks(a, b, ndof)
    say(f"    {what}: worst entry ratio {e[i]:.2e} (node {i // ndof}, unknown {i % ndof}); "
        f"norm-wise u {ru:.2e}, eta {re:.2e}")
    assert e[i] <= tol, (f"{what}: entry {i} (node {i // ndof}, unknown {i % ndof}) "
                         f"gpu {a[i]!r} oracle {b[i]!r}, ratio {e[i]:.3e} > {tol:g}")
    return float(e[i])


def abs_product(A, x):
    """(|A| |x|): the per-entry rounding scale of the product A x."""
    return abs(A) @ np.abs(np.asarray(x, dtype=float).ravel())


def prolong_nodal(xc, shape_c):
    """Trilinear prolongation of node-interleaved values (n_nodes_c, ndof) on
    a structured grid of shape_c = (nzc, nyc, nxc) elements to the grid twice
    as fine (the V-cycle's P; coarse node (I, J, K) = fine node (2I, 2J, 2K))."""
    nzc, nyc, nxc = shape_c
    c = np.asarray(xc, dtype=float).reshape(nzc + 1, nyc + 1, nxc + 1, -1)
    for ax in range(3):
        n = c.shape[ax]
        f = np.empty(c.shape[:ax] + (2 * n - 1,) + c.shape[ax + 1:])
        sl = [slice(None)] * 4
        sl[ax] = slice(0, None, 2)
        f[tuple(sl)] = c
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax], hi[ax] = slice(0, n - 1), slice(1, n)
        sl[ax] = slice(1, None, 2)
        f[tuple(sl)] = 0.5 * (c[tuple(lo)] + c[tuple(hi)])
        c = f
    return c.reshape(-1, c.shape[-1])


def restrict_nodal(yf, shape_c):
    """The transpose of prolong_nodal (fine grid of 2 shape_c elements)."""
    nzc, nyc, nxc = shape_c
    f = np.asarray(yf, dtype=float).reshape(2 * nzc + 1, 2 * nyc + 1, 2 * nxc + 1, -1)
    for ax in range(3):
        sl = [slice(None)] * 4
        sl[ax] = slice(0, None, 2)
        c = f[tuple(sl)].copy()
        sl[ax] = slice(1, None, 2)
        odd = 0.5 * f[tuple(sl)]
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax], hi[ax] = slice(0, -1), slice(1, None)
        c[tuple(lo)] += odd
        c[tuple(hi)] += odd
        f = c
    return f.reshape(-1, f.shape[-1])


def galerkin_apply(apply_fine, xc, shape_c, mask_f, mask_c):
    """A_c x_c of the eliminated Galerkin operator A_c = P~^T A_f P~ (P~ = P
    with the rows of constrained fine dofs zeroed) from a product with the
    eliminated fine operator (apply_fine: flat fine vector -> flat product):
    free coarse rows (P~^T A_f P~ x~)_free with x~ = x_c zeroed on the
    constrained coarse dofs; constrained rows x_c."""
    ndof = mask_c.shape[1]
    x = np.where(mask_c, 0.0, np.asarray(xc, dtype=float).reshape(-1, ndof))
    xf = np.where(mask_f, 0.0, prolong_nodal(x, shape_c))
    yf = np.asarray(apply_fine(xf.ravel()), dtype=float).reshape(-1, ndof)
    yc = restrict_nodal(np.where(mask_f, 0.0, yf), shape_c)
    return np.where(mask_c, np.asarray(xc, dtype=float).reshape(-1, ndof), yc).ravel()


def coarse_masks(mask0, shape0, n_levels):
    """Constrained-dof masks of every level: a coarse dof is constrained iff
    its coincident finest dof is."""
    nz, ny, nx = shape0
    m3 = np.asarray(mask0).reshape(nz + 1, ny + 1, nx + 1, -1)
    return [m3[::2 ** l, ::2 ** l, ::2 ** l].reshape(-1, m3.shape[-1]) for l in range(n_levels)]
