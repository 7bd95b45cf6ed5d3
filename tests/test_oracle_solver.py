"""Pins of the oracle's linear and nonlinear solvers (Sec. 3.4)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import solver as S
from oracle.fem import Mesh, NDOF
from oracle.material import Card


def _tiny(n=4, levels=2, patch=2, depth=0.02, eta_offset=0.0):
    p = synth.Problem(n, n, n, n_levels=levels, patch=patch, depth_increment=depth)
    card = Card(p.material)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = eta_offset + p.eta0()
    En = U[:, 3:].ravel().copy()
    mask, target = S.dirichlet(m, "patch", p.patch, depth=p.depth_increment)
    g = S.increment(mask, target, U)
    return p, card, m, U.ravel(), En, mask, g


def test_dirichlet_sets():
    m = Mesh(8, 8, 8, 0.125)
    mask, g = S.dirichlet(m, "patch", 2, depth=0.02)
    assert np.array_equal(S.increment(mask, g, np.zeros((m.n_nodes, NDOF))), g)
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    assert mask[k == 0][:, :3].all() and not mask[k == 0][:, 3:].any()
    top = np.nonzero(mask[:, 2] & (k == 8))[0]
    assert len(top) == 9 and set(i[top]) == {3, 4, 5} and set(j[top]) == {3, 4, 5}
    assert np.all(g[top, 2] == -0.02) and np.count_nonzero(g) == 9
    cm = Mesh(4, 4, 4, 0.25)
    cmask = S.coarse_mask(m, mask, cm)
    ci, cj, ck = cm.node_ijk(np.arange(cm.n_nodes))
    assert np.nonzero(cmask[:, 2] & (ck == 4))[0].tolist() == [cm.node_id(2, 2, 4)]


def test_cap_profile():
    """Spherical cap: contact radius sqrt(2Rd - d^2); the centre node sits at
    -d and the profile follows the sphere R - sqrt(R^2 - r^2) - d."""
    m = Mesh(16, 16, 8, 1.0 / 16)
    R, d = 0.2, 0.02
    mask, t = S.dirichlet(m, "cap", radius=R, depth=d)
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    top = np.nonzero(mask[:, 2] & (k == 8))[0]
    r = np.hypot(i[top] / 16 - 0.5, j[top] / 16 - 0.5)
    assert r.max() < np.sqrt(2 * R * d - d * d)
    assert np.isclose(t[m.node_id(8, 8, 8), 2], -d)
    x, z = r, t[top, 2] + d            # indenter surface height above its tip
    assert np.allclose((R - z) ** 2 + x ** 2, R * R)
    # contact radius 0.0872 > h = 0.0625 but < h*sqrt2: centre + 4 edge neighbours
    assert len(top) == 5


def test_prolongation_exact_on_trilinear_fields():
    fine, coarse = Mesh(4, 6, 2, 0.1), Mesh(2, 3, 1, 0.2)
    P = S.prolongation(coarse, fine, bs=1)

    def f(m):
        i, j, k = m.node_ijk(np.arange(m.n_nodes))
        x, y, z = i * m.h, j * m.h, k * m.h
        return 1.5 - 2 * x + 0.5 * y + 3 * z + x * y - 2 * x * z + 0.7 * y * z + 4 * x * y * z

    assert np.allclose(P @ f(coarse), f(fine), atol=1e-14)
    assert np.allclose(np.asarray(P.sum(1)).ravel(), 1.0)


def test_direct_solve_matches_dense_library_solve():
    p, card, m, U, En, mask, g = _tiny(4)
    sysk = S.NewtonSystem(p, card, U, En, mask, g)
    x = S.direct_solve(sysk.A, sysk.b)
    y = np.linalg.solve(sysk.A.toarray(), sysk.b)
    # both are backward stable: forward error <= ~ cond(A) * eps
    kappa = np.linalg.cond(sysk.A.toarray())
    assert np.linalg.norm(x - y) <= 10 * kappa * 2.2e-16 * np.linalg.norm(y)
    assert np.allclose(x[mask.ravel()], g.ravel()[mask.ravel()], rtol=0, atol=1e-15)
    A = sysk.A.toarray()
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())


def test_lifting_equals_constrained_solve():
    """Lifting + elimination gives the same increment as solving the full
    system with the constrained rows replaced by Delta_c = g."""
    p, card, m, U, En, mask, g = _tiny(4)
    sysk = S.NewtonSystem(p, card, U, En, mask, g)
    x = S.direct_solve(sysk.A, sysk.b)
    K = sysk.K.toarray()
    mv = mask.ravel()
    rhs = -sysk.R.copy()
    K[mv, :] = 0.0
    K[mv, mv] = 1.0
    rhs[mv] = g.ravel()[mv]
    y = np.linalg.solve(K, rhs)
    assert np.linalg.norm(x - y) <= 1e-11 * np.linalg.norm(y)


@pytest.mark.slow
def test_fgmres_multigrid_reaches_direct_solution():
    p, card, m, U, En, mask, g = _tiny(8, levels=3)
    sysk = S.NewtonSystem(p, card, U, En, mask, g)
    x = S.direct_solve(sysk.A, sysk.b)
    mg = S.Multigrid(p, card, U, En, mask, K_fine=sysk.K)
    y, st = S.fgmres(sysk.A, sysk.b, mg.precondition, rtol=1e-12)
    assert st.converged and st.rel_residual <= 1e-12
    assert np.linalg.norm(y - x) <= 1e-9 * np.linalg.norm(x)
    y8, st8 = S.fgmres(sysk.A, sysk.b, mg.precondition, rtol=1e-8)
    assert st8.converged and st8.iterations < 40


def test_fgmres_without_preconditioner_is_gmres_on_spd_system():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((40, 40))
    A = sp.csr_matrix(B @ B.T + 40 * np.eye(40))
    b = rng.standard_normal(40)
    x, st = S.fgmres(A, b, lambda v: v, rtol=1e-13, restart=10)
    assert np.linalg.norm(x - np.linalg.solve(A.toarray(), b)) < 1e-11 * np.linalg.norm(x)
    assert st.restarts >= 1


@pytest.mark.slow
def test_poisson_vcycle_h_independent():
    its = []
    for n in (8, 16, 32):
        levs = S.poisson_levels(n, int(np.log2(n)) - 1)
        mg = S.Multigrid.from_levels(levs, 1)
        A = levs[0].A
        b = np.ones(A.shape[0])
        b[levs[0].mask.ravel()] = 0
        _, st = S.fgmres(A, b, mg.precondition, rtol=1e-8)
        assert st.converged
        its.append(st.iterations)
    assert max(its) - min(its) <= 2 and max(its) <= 12


def test_newton_converges_quadratically():
    """Order parameters away from zero (no penalty switching): the residual
    decreases quadratically once small.  Above the round-off floor,
    r_{k+1} <= C r_k^2 with a moderate C."""
    p, card, m, U, En, mask, g = _tiny(4, depth=0.02, eta_offset=0.1)
    log = []
    U1, it, ok = S.newton_step(p, card, U, En, mask, g, rtol=1e-12, log=log)
    assert ok and it <= 8
    r = log[1:]
    ratios = [r[k + 1] / r[k] ** 2 for k in range(len(r) - 1) if r[k] < 1e-2 and r[k + 1] > 1e-12]
    assert ratios and max(ratios) < 1e2
    assert np.allclose(U1.reshape(-1, NDOF)[mask], (U.reshape(-1, NDOF) + g)[mask])


def _block_system(n=6, bs=9, coupled=True, seed=3):
    """Random operator with well-conditioned dense bs x bs diagonal blocks and
    (optionally) off-diagonal blocks coupling neighbouring nodes."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n * bs, n * bs))
    for a in range(n):
        blk = rng.standard_normal((bs, bs)) + bs * np.eye(bs)
        A[a * bs:(a + 1) * bs, a * bs:(a + 1) * bs] = blk
        if coupled and a + 1 < n:
            off = 0.3 * rng.standard_normal((bs, bs))
            A[a * bs:(a + 1) * bs, (a + 1) * bs:(a + 2) * bs] = off
            A[(a + 1) * bs:(a + 2) * bs, a * bs:(a + 1) * bs] = off.T
    return A, rng.standard_normal(n * bs)


def _one_level_mg(A, bs, omega):
    lev = S.Level(mesh=None, mask=np.zeros((A.shape[0] // bs, bs), dtype=bool), A=sp.csr_matrix(A))
    last = S.Level(mesh=None, mask=np.zeros((1, bs), dtype=bool), A=sp.identity(bs, format="csr"))
    return S.Multigrid.from_levels([lev, last], bs, S.MGOptions(omega=omega)), lev


def test_point_block_inverse_and_first_sweep():
    """Point-block Jacobi (Sec. 3.4): the smoother inverts the whole 9x9 block
    of each node.  block_diagonal_inverse(A)[n] A_nn = I for the dense
    diagonal blocks, and one damped sweep from x = 0 gives
    x = omega A_nn^-1 b_n on every node whatever the off-diagonal blocks are.
    A scalar (pointwise) Jacobi, a wrong block size, a wrong sign or a missing
    damping factor all fail."""
    bs, omega = 9, 0.55
    A, b = _block_system(bs=bs)
    n = A.shape[0] // bs
    Dinv = S.block_diagonal_inverse(sp.csr_matrix(A), bs)
    for a in range(n):
        Ann = A[a * bs:(a + 1) * bs, a * bs:(a + 1) * bs]
        assert np.allclose(Dinv[a] @ Ann, np.eye(bs), atol=1e-13)
    mg, lev = _one_level_mg(A, bs, omega)
    x = mg.smooth(lev, np.zeros_like(b), b, 1)
    for a in range(n):
        Ann = A[a * bs:(a + 1) * bs, a * bs:(a + 1) * bs]
        assert np.allclose(Ann @ x[a * bs:(a + 1) * bs], omega * b[a * bs:(a + 1) * bs], atol=1e-12)


def test_point_block_jacobi_exact_on_block_diagonal():
    """On a block-diagonal operator each node's error is multiplied by
    (1 - omega) per sweep, so k sweeps from zero give
    x_k = (1 - (1 - omega)^k) A^-1 b."""
    bs, omega = 9, 0.55
    A, b = _block_system(coupled=False, seed=5)
    mg, lev = _one_level_mg(A, bs, omega)
    xs = np.linalg.solve(A, b)
    for k in (1, 2, 3):
        x = mg.smooth(lev, np.zeros_like(b), b, k)
        assert np.allclose(x, (1.0 - (1.0 - omega) ** k) * xs, rtol=1e-12, atol=1e-13)


def _uniform_state_problem():
    """8 x 8 x 4 box (3 levels), no top constraint (cap at depth 0: only the
    bottom face, which every level resolves), a homogeneous deformation
    u = G X and uniform eta: the Gauss-point Hessians are the same at every
    point of every level (injection of a linear field is exact)."""
    p = synth.Problem(8, 8, 4, lz=0.5, n_levels=3, kind="cap", radius=0.2, depth_increment=0.0)
    card = Card(p.material)
    m = Mesh.from_problem(p)
    i, j, k = m.node_ijk(np.arange(m.n_nodes))
    X = np.stack([i, j, k], 1) * m.h
    G = np.array([[0.010, 0.004, -0.002], [0.003, -0.006, 0.001], [-0.001, 0.002, 0.008]])
    U = np.zeros((m.n_nodes, NDOF))
    U[:, :3] = X @ G.T
    U[:, 3:] = np.array([0.02, 0.05, 0.01, 0.03, 0.04, 0.02])
    mask, _ = S.dirichlet(m, "cap", radius=0.2, depth=0.0)
    return p, card, m, U.ravel(), U[:, 3:].ravel().copy(), mask


def test_galerkin_equals_reassembly_on_uniform_state():
    """For nested Q1 spaces the coarse discretisation integrates exactly what
    P^T A P integrates when the Hessian is constant: both constructions give
    the same coarse operators (up to rounding) at a homogeneous state, with a
    Dirichlet set every level resolves."""
    p, card, m, U, En, mask = _uniform_state_problem()
    sys0 = S.NewtonSystem(p, card, U, En, mask, np.zeros(mask.shape))
    re = S.Multigrid(p, card, U, En, mask, K_fine=sys0.K, coarse="reassemble")
    ga = S.Multigrid(p, card, U, En, mask, K_fine=sys0.K, coarse="galerkin")
    for l in range(1, p.n_levels):
        Ar, Ag = re.levels[l].A, ga.levels[l].A
        scale = abs(Ar).max()
        assert abs(Ar - Ag).max() <= 1e-12 * scale, (l, abs(Ar - Ag).max() / scale)
        assert np.array_equal(re.levels[l].mask, ga.levels[l].mask)


def test_galerkin_coarse_correction_is_orthogonal():
    """Two-level correction with the Galerkin operator, using the V-cycle's
    transfers (restriction zeroed on constrained coarse dofs, prolongation
    not added on constrained fine dofs): the corrected error is A-orthogonal
    to every admissible coarse function, at a non-uniform state where the
    penalty is active on part of the nodes."""
    p, card, m, U, En, mask, g = _tiny(n=8, levels=2, eta_offset=-0.02)
    sysk = S.NewtonSystem(p, card, U, En, mask, g)
    mg = S.Multigrid(p, card, U, En, mask, K_fine=sysk.K, coarse="galerkin")
    f, c = mg.levels
    e = np.random.default_rng(5).standard_normal(f.A.shape[0])
    e[f.mask.ravel()] = 0.0
    r = f.A @ e
    bc = f.P.T @ r
    bc[c.mask.ravel()] = 0.0
    corr = f.P @ np.linalg.solve(c.A.toarray(), bc)
    corr[f.mask.ravel()] = 0.0
    e2 = e - corr
    free_c = ~c.mask.ravel()
    keep = np.where(f.mask.ravel(), 0.0, 1.0)
    before = (f.P.T @ (keep * (f.A @ e)))[free_c]
    after = (f.P.T @ (keep * (f.A @ e2)))[free_c]
    assert np.linalg.norm(after) <= 1e-11 * np.linalg.norm(before)
    # the penalty is active at some Gauss points (the state is not uniform)
    assert (U.reshape(-1, NDOF)[:, 3:] < 0).any()


def test_nodal_transfers_used_by_the_full_size_galerkin_check():
    """The numpy transfers of the GPU tests' full-size Galerkin check are the
    oracle's prolongation and its transpose (same matrix, compared on random
    vectors), on a non-cubic grid with several unknowns per node."""
    from gpu_util import prolong_nodal, restrict_nodal
    fine, coarse = Mesh(6, 4, 8, 0.1), Mesh(3, 2, 4, 0.2)
    P = S.prolongation(coarse, fine, bs=1)
    rng = np.random.default_rng(11)
    xc = rng.standard_normal((coarse.n_nodes, 3))
    yf = rng.standard_normal((fine.n_nodes, 3))
    assert np.allclose(prolong_nodal(xc, (4, 2, 3)), P @ xc, rtol=0, atol=1e-14)
    assert np.allclose(restrict_nodal(yf, (4, 2, 3)), P.T @ yf, rtol=0, atol=1e-13)


def test_full_size_galerkin_rows_from_local_elements():
    """The full-size GPU tests' sampled Galerkin rows (finest elements around
    the support of each sampled coarse node's column of the composite
    prolongation) reproduce the rows of the oracle's assembled Galerkin
    hierarchy on levels 1 and 2, and their rounding scale bounds |A_l| |x|."""
    from oracle.fem import NDOF
    from gpu_util import OracleCase
    from test_gpu_fullsize import GalerkinRows, sample_nodes
    p = synth.Problem(16, 16, 8, lz=0.5, n_levels=3, kind="cap", radius=0.2, depth_increment=0.02)
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    oc = OracleCase(p, U, U[:, 3:], p.depth_increment, coarse="galerkin", direct=False)
    rng = np.random.default_rng(1)
    for l in (1, 2):
        cm = Mesh.from_problem(p, l)
        x = rng.standard_normal(cm.n_nodes * NDOF)
        gr = GalerkinRows(p, U, U[:, 3:], p.depth_increment, l, sample_nodes(cm, 1, seed=3, n_random=5), x)
        A = oc.mg.levels[l].A
        ref = (A @ x)[gr.dofs]
        assert np.abs(gr.y - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.all(gr.y_abs >= (abs(A) @ np.abs(x))[gr.dofs] * (1 - 1e-12))
