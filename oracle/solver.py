"""Newton step, FGMRES and geometric multigrid with point-block Jacobi.

Oracle (test infrastructure only; see the package docstring).

What the method computes (Sec. 3.4, Eqs. FinalRes and linAlgEq): at each Newton
iteration the increment Delta solves K Delta = -R, then U <- U + Delta.  The
plain definition of that increment is a direct sparse solve (``direct_solve``);
GMRES with a geometric-multigrid preconditioner reaches it approximately.  The
preconditioner (Sec. 3.4): operators rebuilt on every level by reassembly (not
Galerkin projection), V-cycle of pre-smoothing, coarse correction, direct
solve on the coarsest level, prolongation and post-smoothing, with point-block
Jacobi relaxation whose 9x9 blocks gather all unknowns of a node and are
inverted by LU with partial pivoting.

Readings where the paper is silent:
* Dirichlet conditions: symmetric elimination (constrained rows and columns of
  K replaced by the identity); a prescribed increment g enters the first
  Newton system by lifting: b_free = -R_free - (K g)_free, b_con = g.
* Coarse-level state is the injection (coincident-node values) of the fine
  state; a coarse dof is constrained iff its coincident fine dof is.
* Besides the paper's reassembly, coarse operators can be the Galerkin
  products A_c = P~^T A P~ (P~ = P with the rows of constrained fine dofs
  zeroed, matching the transfers below).  For nested Q1 spaces and a state
  that is uniform over each coarse element the two coincide (the 2x2x2
  Gauss rule integrates both exactly); they differ where the penalty of
  Eq. IntEnergy is active on a pattern finer than the coarse mesh, which the
  injected coarse state cannot represent.
* Prolongation P = trilinear interpolation, restriction = P^T; restricted
  residuals are zeroed at constrained coarse dofs, prolongated corrections are
  not added at constrained fine dofs; the preconditioner is the identity on
  the constrained dofs of the finest level.
* Smoother: x <- x + omega D^-1 (b - A x), omega = 0.55, nu1 = nu2 = 2, zero
  initial guess on every level.  (The spectral radius of D^-1 A measured on
  these operators is about 3.37 on every level, so the damped-Jacobi
  stability limit 2/lambda_max is about 0.59 and the textbook 2/3 diverges;
  below that limit 0.55 needs one FGMRES iteration fewer than 0.5 on every
  workload.)
* Outer Krylov method: flexible GMRES(m), right preconditioned, x0 = 0,
  classical Gram-Schmidt applied twice, Givens rotations, stop when the
  recurrence residual drops to rtol * ||b||, then a true-residual check.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .contact import SphereContact
from .fem import NDOF, NETA, Discretisation, Mesh
from .material import Card


# ---------------------------------------------------------------------------
# boundary conditions
# ---------------------------------------------------------------------------

def dirichlet(mesh: Mesh, kind: str = "patch", patch: int = 2, radius: float = 0.2,
              depth: float = 0.0, ndof: int = NDOF):
    """Constrained-dof mask (n_nodes, ndof) bool and target values (n_nodes, ndof)
    (ndof = 3 + N unknowns per node, N variants).

    Bottom face z = 0: all three displacement components fixed at 0.  Top
    face: kind 'patch' -- nodes of the centred patch x patch element square
    have u_z = -depth; kind 'cap' -- nodes under a rigid sphere of radius R
    at total depth d, r^2 < 2 R d - d^2 (r measured from the top-face
    centre), have u_z = -(d - (R - sqrt(R^2 - r^2))); kind 'sphere' -- none
    (the indenter acts through penalty contact, module ``contact``).  Order
    parameters are never constrained (natural boundary conditions).
    """
    nn = mesh.n_nodes
    mask = np.zeros((nn, ndof), dtype=bool)
    target = np.zeros((nn, ndof))
    i, j, k = mesh.node_ijk(np.arange(nn))
    mask[k == 0, 0:3] = True
    top = k == mesh.nz
    if kind == "patch":
        if patch % 2 or mesh.nx % 2 or mesh.ny % 2:
            raise ValueError("patch and mesh must be even to centre the patch on a node")
        cx, cy, hp = mesh.nx // 2, mesh.ny // 2, patch // 2
        sel = top & (np.abs(i - cx) <= hp) & (np.abs(j - cy) <= hp)
        mask[sel, 2] = True
        target[sel, 2] = -depth
    elif kind == "cap":
        x = i * mesh.h - 0.5 * mesh.nx * mesh.h
        y = j * mesh.h - 0.5 * mesh.ny * mesh.h
        r2 = x * x + y * y
        sel = top & (r2 < 2.0 * radius * depth - depth * depth)
        mask[sel, 2] = True
        target[sel, 2] = -(depth - (radius - np.sqrt(radius * radius - r2[sel])))
    elif kind != "sphere":
        raise ValueError(kind)
    return mask, target


def increment(mask: np.ndarray, target: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Prescribed Newton increment g = target - current on constrained dofs."""
    return np.where(mask, target - U.reshape(mask.shape), 0.0)


def coarse_mask(fine_mesh: Mesh, fine_mask: np.ndarray, coarse_mesh: Mesh) -> np.ndarray:
    """A coarse dof is constrained iff the coincident fine dof is."""
    I, J, K = coarse_mesh.node_ijk(np.arange(coarse_mesh.n_nodes))
    return fine_mask[fine_mesh.node_id(2 * I, 2 * J, 2 * K)]


def inject(fine_mesh: Mesh, fine_nodal: np.ndarray, coarse_mesh: Mesh) -> np.ndarray:
    """Coarse nodal values = fine values at coincident nodes."""
    I, J, K = coarse_mesh.node_ijk(np.arange(coarse_mesh.n_nodes))
    return fine_nodal.reshape(fine_mesh.n_nodes, -1)[fine_mesh.node_id(2 * I, 2 * J, 2 * K)]


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

def assemble(disc: Discretisation, U: np.ndarray, Eta_n: np.ndarray,
             contact: Optional[SphereContact] = None, depth: float = 0.0) -> sp.csr_matrix:
    """Unconstrained tangent K as CSR (duplicates summed by scipy), with the
    contact tangent at indenter depth ``depth`` when ``contact`` is given."""
    n = disc.mesh.n_nodes * disc.ndof
    r, c, v = disc.tangent_coo(U, Eta_n)
    if contact is not None:
        rc, cc, vc = contact.tangent_coo(U, depth)
        r, c, v = np.concatenate([r, rc]), np.concatenate([c, cc]), np.concatenate([v, vc])
    return sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()


def contact_of(problem, mesh: Mesh) -> Optional[SphereContact]:
    """The indenter's penalty contact on ``mesh`` for kind 'sphere', else None."""
    if getattr(problem, "kind", "patch") != "sphere":
        return None
    return SphereContact(mesh, problem.radius, problem.eps_n)


def eliminate(K: sp.csr_matrix, mask: np.ndarray) -> sp.csr_matrix:
    """Replace constrained rows and columns by those of the identity."""
    m = mask.ravel()
    keep = sp.diags((~m).astype(float))
    return (keep @ K @ keep + sp.diags(m.astype(float))).tocsr()


def prolongation(coarse: Mesh, fine: Mesh, bs: int = NDOF) -> sp.csr_matrix:
    """Trilinear interpolation, node-interleaved with bs components:
    P = P_node (x) I_bs.  Fine node (i,j,k) takes weight prod_d w_d from coarse
    node (I,J,K), w_d = 1 if i_d = 2 I_d and 1/2 if |i_d - 2 I_d| = 1."""
    rows, cols, vals = [], [], []
    fi, fj, fk = fine.node_ijk(np.arange(fine.n_nodes))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # candidate coarse parent of each fine node
                ci, cj, ck = (fi + dx), (fj + dy), (fk + dz)
                ok = (ci % 2 == 0) & (cj % 2 == 0) & (ck % 2 == 0)
                ci, cj, ck = ci // 2, cj // 2, ck // 2
                ok &= (ci >= 0) & (ci <= coarse.nx) & (cj >= 0) & (cj <= coarse.ny) \
                    & (ck >= 0) & (ck <= coarse.nz)
                w = (0.5 ** abs(dx)) * (0.5 ** abs(dy)) * (0.5 ** abs(dz))
                rows.append(np.nonzero(ok)[0])
                cols.append(coarse.node_id(ci[ok], cj[ok], ck[ok]))
                vals.append(np.full(ok.sum(), w))
    Pn = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(fine.n_nodes, coarse.n_nodes)).tocsr()
    return sp.kron(Pn, sp.eye(bs), format="csr")


def block_diagonal_inverse(A: sp.csr_matrix, bs: int = NDOF) -> np.ndarray:
    """Inverses of the bs x bs diagonal blocks, (n_nodes, bs, bs).
    numpy.linalg.inv factors each block by LU with partial pivoting (LAPACK
    getrf/getri)."""
    n = A.shape[0] // bs
    Ab = A.tobsr(blocksize=(bs, bs))
    D = np.zeros((n, bs, bs))
    for row in range(n):
        for p in range(Ab.indptr[row], Ab.indptr[row + 1]):
            if Ab.indices[p] == row:
                D[row] = Ab.data[p]
    return np.linalg.inv(D)


@dataclass
class Level:
    mesh: Mesh
    mask: np.ndarray           # (n_nodes, 9) bool
    A: sp.csr_matrix           # eliminated operator
    Dinv: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None     # prolongation from the next coarser level
    lu: Optional[tuple] = None            # dense LU of the coarsest operator


@dataclass
class MGOptions:
    nu1: int = 2
    nu2: int = 2
    omega: float = 0.55


def galerkin_coarse(A: sp.csr_matrix, fine_mask: np.ndarray, P: sp.csr_matrix,
                    coarse_mask_: np.ndarray) -> sp.csr_matrix:
    """Galerkin coarse operator of an eliminated fine operator A: with P~ = P
    whose rows of constrained fine dofs are zero (a correction never touches
    them), A_c = P~^T A P~, then the constrained coarse dofs eliminated."""
    keep = sp.diags((~fine_mask.ravel()).astype(float))
    Pt = (keep @ P).tocsr()
    return eliminate((Pt.T @ A @ Pt).tocsr(), coarse_mask_)


class Multigrid:
    """Geometric multigrid hierarchy.  coarse = 'reassemble': every coarse
    operator is the discretisation on its own mesh at the injected state
    (Sec. 3.4); coarse = 'galerkin': A_l = P~^T A_{l-1} P~ (galerkin_coarse)
    from the finest operator down."""

    def __init__(self, problem, card: Card, U: np.ndarray, Eta_n: np.ndarray,
                 fine_mask: np.ndarray, n_levels: Optional[int] = None,
                 opts: MGOptions = MGOptions(), K_fine: Optional[sp.csr_matrix] = None,
                 depth: float = 0.0, coarse: str = "reassemble"):
        if coarse not in ("reassemble", "galerkin"):
            raise ValueError(f"coarse operators: 'reassemble' or 'galerkin', not {coarse!r}")
        self.opts = opts
        self.bs = 3 + card.n_var
        L = problem.n_levels if n_levels is None else n_levels
        self.levels: List[Level] = []
        mesh = Mesh.from_problem(problem, 0)
        Ul, En, mask = U.reshape(-1, self.bs), Eta_n.reshape(-1, self.bs - 3), fine_mask
        for l in range(L):
            if l > 0:
                cm = Mesh.from_problem(problem, l)
                Ul = inject(mesh, Ul, cm)
                En = inject(mesh, En, cm)
                fmask = mask
                mask = coarse_mask(mesh, mask, cm)
                prev = self.levels[-1]
                prev.P = prolongation(cm, mesh, self.bs)
                mesh = cm
                if coarse == "galerkin":
                    self.levels.append(Level(mesh=mesh, mask=mask, A=galerkin_coarse(prev.A, fmask, prev.P, mask)))
                    continue
            disc = Discretisation(mesh, card)
            K = K_fine if (l == 0 and K_fine is not None) else \
                assemble(disc, Ul.ravel(), En.ravel(), contact_of(problem, mesh), depth)
            A = eliminate(K, mask)
            self.levels.append(Level(mesh=mesh, mask=mask, A=A))
        self._finish()

    @classmethod
    def from_levels(cls, levels: List[Level], bs: int, opts: MGOptions = MGOptions()):
        """Hierarchy from given operators/masks/prolongations (finest first)."""
        mg = cls.__new__(cls)
        mg.opts, mg.bs, mg.levels = opts, bs, levels
        mg._finish()
        return mg

    def _finish(self):
        for lev in self.levels[:-1]:
            lev.Dinv = block_diagonal_inverse(lev.A, self.bs)
        self.levels[-1].lu = scipy.linalg.lu_factor(self.levels[-1].A.toarray())

    def smooth(self, lev: Level, x: np.ndarray, b: np.ndarray, sweeps: int) -> np.ndarray:
        """Damped point-block Jacobi: x <- x + omega D^-1 (b - A x)."""
        for _ in range(sweeps):
            r = (b - lev.A @ x).reshape(-1, self.bs)
            x = x + self.opts.omega * np.einsum("nij,nj->ni", lev.Dinv, r).ravel()
        return x

    def vcycle(self, l: int, b: np.ndarray) -> np.ndarray:
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            return scipy.linalg.lu_solve(lev.lu, b)
        x = self.smooth(lev, np.zeros_like(b), b, self.opts.nu1)
        r = b - lev.A @ x
        nxt = self.levels[l + 1]
        bc = lev.P.T @ r
        bc[nxt.mask.ravel()] = 0.0
        e = self.vcycle(l + 1, bc)
        corr = lev.P @ e
        corr[lev.mask.ravel()] = 0.0
        x = x + corr
        return self.smooth(lev, x, b, self.opts.nu2)

    def precondition(self, v: np.ndarray) -> np.ndarray:
        m = self.levels[0].mask.ravel()
        b = v.copy()
        b[m] = 0.0
        z = self.vcycle(0, b)
        z[m] = v[m]
        return z


# ---------------------------------------------------------------------------
# Krylov solver
# ---------------------------------------------------------------------------

@dataclass
class SolveStats:
    iterations: int = 0
    restarts: int = 0
    rel_residual: float = 0.0       # true ||b - A x|| / ||b||
    history: list = field(default_factory=list)   # recurrence residual / ||b||
    converged: bool = False


def fgmres(A, b: np.ndarray, precond, rtol: float = 1e-8, restart: int = 30,
           max_it: int = 500):
    """Flexible GMRES(m), right preconditioning, x0 = 0 (Saad 1993)."""
    n = b.shape[0]
    st = SolveStats()
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        st.converged = True
        return x, st
    r = b.copy()
    beta = bnorm
    while True:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            H[:j + 1, j] = h + h2
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            st.iterations += 1
            k = j + 1
            st.history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or st.iterations >= max_it:
                break
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        st.rel_residual = beta / bnorm
        if st.rel_residual <= rtol:
            st.converged = True
            return x, st
        if st.iterations >= max_it:
            return x, st
        st.restarts += 1


def poisson_levels(n: int, n_levels: int) -> List[Level]:
    """Scalar (block size 1) Q1 Laplacian on the unit cube with u = 0 on z = 0,
    rediscretised on n, n/2, ... (textbook tensor-product element matrix
    K_e = Km(x)Mm(x)Mm + Mm(x)Km(x)Mm + Mm(x)Mm(x)Km with the 1D forms
    Km = [[1,-1],[-1,1]]/h and Mm = h/6 [[2,1],[1,2]]).  Used to check the
    h-independence of the V-cycle."""
    levels = []
    prev = None
    for l in range(n_levels):
        m = Mesh(n >> l, n >> l, n >> l, 1.0 / (n >> l))
        h = m.h
        Km = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
        Mm = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
        # local node a = ax + 2 ay + 4 az  <->  kron order (az, ay, ax)
        Ke = np.kron(np.kron(Mm, Mm), Km) + np.kron(np.kron(Mm, Km), Mm) \
            + np.kron(np.kron(Km, Mm), Mm)
        en = m.element_nodes()
        r = np.repeat(en, 8, axis=1).ravel()
        c = np.tile(en, (1, 8)).ravel()
        v = np.tile(Ke.ravel(), m.n_elem)
        K = sp.coo_matrix((v, (r, c)), shape=(m.n_nodes, m.n_nodes)).tocsr()
        _, _, k = m.node_ijk(np.arange(m.n_nodes))
        mask = (k == 0)[:, None]
        lev = Level(mesh=m, mask=mask, A=eliminate(K, mask))
        if prev is not None:
            levels[-1].P = prolongation(m, prev, bs=1)
        levels.append(lev)
        prev = m
    return levels


def direct_solve(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """The plain definition of the Newton increment: x = A^-1 b (SuperLU)."""
    return spla.spsolve(A.tocsc(), b)


# ---------------------------------------------------------------------------
# Newton
# ---------------------------------------------------------------------------

class NewtonSystem:
    """Linear system of one Newton iteration (Eq. linAlgEq) with Dirichlet
    lifting: A = K with constrained rows/cols eliminated, b as described in the
    module docstring.  For an indenter in contact (kind 'sphere') R and K
    include the penalty contact terms at indenter depth ``depth``."""

    def __init__(self, problem, card: Card, U: np.ndarray, Eta_n: np.ndarray,
                 mask: np.ndarray, g: np.ndarray, depth: float = 0.0):
        self.mesh = Mesh.from_problem(problem, 0)
        self.disc = Discretisation(self.mesh, card)
        self.contact = contact_of(problem, self.mesh)
        self.R = self.disc.residual(U, Eta_n)
        if self.contact is not None:
            self.R = self.R + self.contact.residual(U, depth)
        self.K = assemble(self.disc, U, Eta_n, self.contact, depth)
        m = mask.ravel()
        gv = np.where(m, g.ravel(), 0.0)
        b = -self.R - self.K @ gv
        b[m] = gv[m]
        self.b = b
        self.A = eliminate(self.K, mask)
        self.mask = mask


def newton_step(problem, card: Card, U: np.ndarray, Eta_n: np.ndarray, mask: np.ndarray,
                g: np.ndarray, rtol: float = 1e-9, max_iter: int = 12, linear: str = "direct",
                lin_rtol: float = 1e-12, log: Optional[list] = None, depth: float = 0.0):
    """Newton iterations of one implicit step.  The first system carries the
    prescribed increment g; later ones are homogeneous on constrained dofs.
    Converged when ||R_free|| <= rtol * ||b_0|| (b_0 = first right-hand side).
    Returns (U, iterations, converged)."""
    U = U.copy()
    b0 = None
    gk = g
    for it in range(max_iter):
        sysk = NewtonSystem(problem, card, U, Eta_n, mask, gk, depth)
        if b0 is None:
            b0 = float(np.linalg.norm(sysk.b))
        rfree = float(np.linalg.norm(np.where(mask.ravel(), 0.0, sysk.R)))
        if log is not None:
            log.append(rfree)
        if it > 0 and rfree <= rtol * b0:
            return U, it, True
        if linear == "direct":
            dx = direct_solve(sysk.A, sysk.b)
        else:
            mg = Multigrid(problem, card, U, Eta_n, mask, K_fine=sysk.K, depth=depth)
            dx, _ = fgmres(sysk.A, sysk.b, mg.precondition, rtol=lin_rtol)
        U = U + dx
        if not np.all(np.isfinite(U)):  # diverged: the step fails
            return U, max_iter, False
        gk = np.zeros_like(g)
    sysk = NewtonSystem(problem, card, U, Eta_n, mask, gk, depth)
    rfree = float(np.linalg.norm(np.where(mask.ravel(), 0.0, sysk.R)))
    return U, max_iter, rfree <= rtol * b0


# ---------------------------------------------------------------------------
# indentation driver with adaptive time steps
# ---------------------------------------------------------------------------

@dataclass
class IndentOptions:
    """Loading to ``depth_max`` (then unloading to 0 when ``unload``) by a
    rigid spherical indenter moving at constant speed v.  The time step
    enters through the viscous coefficient rho = 1/(m tau) with tau = dd / v,
    i.e. rho = visc_depth / |dd| with visc_depth = v / m.  Step control
    (Sec. 3.4): after an accepted step with n Newton iterations the next
    depth increment is multiplied by ``grow`` if n < newton_desired and by
    ``shrink`` if n > newton_desired (kept within [dd_min, dd_max]); a step
    whose Newton iterations exceed newton_max is rejected and retried with
    half the increment.  Steps never overshoot the end of a phase: when at
    most dd + dd_min is left, the step goes exactly to the phase's end."""
    depth_max: float
    dd_init: float
    dd_min: float
    dd_max: float
    visc_depth: float
    grow: float = 1.25
    shrink: float = 0.8
    newton_desired: int = 7
    newton_max: int = 12
    unload: bool = True
    max_steps: int = 1000


@dataclass
class IndentRecord:
    depth: float
    load: float
    newton_iterations: int
    rejected: int


def indent(problem, U: np.ndarray, Eta_n: np.ndarray, opts: IndentOptions,
           newton_rtol: float = 1e-9):
    """Quasi-static indentation run (kind 'sphere') from depth 0 with the
    state (U, Eta_n).  Returns (records of the accepted steps, U, ok)."""
    from dataclasses import replace
    mesh = Mesh.from_problem(problem, 0)
    contact = contact_of(problem, mesh)
    if contact is None:
        raise ValueError("indentation needs the 'sphere' loading")
    mask, _ = dirichlet(mesh, "sphere", ndof=U.size // mesh.n_nodes)
    zero = np.zeros(mask.shape)
    U, Eta_n = U.copy(), Eta_n.copy()
    depth, dd = 0.0, opts.dd_init
    targets = [opts.depth_max] + ([0.0] if opts.unload else [])
    records: List[IndentRecord] = []
    rejected = 0
    for goal in targets:
        sign = 1.0 if goal > depth else -1.0
        while depth != goal:
            if len(records) >= opts.max_steps:
                return records, U, False
            rem = abs(goal - depth)
            if rem <= dd + opts.dd_min:  # the phase's last step: land on the goal
                step, trial = rem, goal
            else:
                step, trial = dd, depth + sign * dd
            card = Card(replace(problem.material, rho=opts.visc_depth / step))
            U1, it, ok = newton_step(problem, card, U, Eta_n, mask, zero, rtol=newton_rtol,
                                     max_iter=opts.newton_max, depth=trial)
            if not ok:
                rejected += 1
                dd = 0.5 * step
                if dd < opts.dd_min:
                    return records, U, False
                continue
            U, depth = U1, trial
            Eta_n = U.reshape(-1, mask.shape[1])[:, 3:].ravel().copy()
            records.append(IndentRecord(depth, contact.load(U, depth), it, rejected))
            rejected = 0
            if it < opts.newton_desired:
                dd = min(dd * opts.grow, opts.dd_max)
            elif it > opts.newton_desired:
                dd = max(dd * opts.shrink, opts.dd_min)
    return records, U, True
