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
