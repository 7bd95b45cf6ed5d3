"""Parity at the workloads' full sizes, in the configuration bench.py times
(mixed precision, matrix-free finest level, autotuned launch shapes), on
sampled outputs the oracle computes one by one: it evaluates only the
elements (and contact faces) around a sample of nodes, which fixes those
nodes' rows of the residual, the right-hand side and the eliminated
tangent exactly.

Samples: the 8 corners, edge and face midpoints, nodes of the loaded top
region, and 40 seeded random nodes.  Tolerances, entry by entry relative to
the entry's node scale (the largest oracle value among its 9 unknowns) plus
its rounding scale (the sum of the absolute values of the terms summed:
(|A||x|) for operator products, sum_e |R_e| over the element contributions
for the residual): FP64 rows <= 1e-12, FP32 operator rows <= 2e-6; the solve's true FP64
relative residual (evaluated by the GPU's FP64 operator, whose rows are the
checked ones) <= 1e-8, the accuracy the solver is run at.

The workloads run with Galerkin coarse operators, as the benchmark times them:
the oracle also forms sampled rows of the level-1 and level-2 operators,
A_l = Q_l^T K Q_l on the free unknowns, where Q_l is the composite of the
trilinear prolongations with the rows of constrained unknowns zeroed at every
level and K the finest tangent, from the finest elements around the support of
each sampled coarse node's column of Q_l; its rounding scale is
Q_l^T |K| Q_l |x|, a bound on the sum of the absolute values of the terms.
The deeper levels are checked by the identity A_l x = P~^T A_{l-1} P~ x on
the free unknowns (GPU operators on both sides, transfers in numpy)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from gpu_util import check_entries, coarse_masks, prolong_nodal, residual_abs, restrict_nodal, say
from oracle import solver as S
from oracle.contact import SphereContact
from oracle.fem import Discretisation, Mesh, NDOF
from oracle.material import Card

pytestmark = pytest.mark.gpu


def sample_nodes(m, top_centre_radius, seed=17, n_random=40):
    ii = [0, m.nx // 2, m.nx]
    jj = [0, m.ny // 2, m.ny]
    kk = [0, m.nz // 2, m.nz]
    nodes = {m.node_id(i, j, k) for i in ii for j in jj for k in kk}
    cx, cy = m.nx // 2, m.ny // 2
    r = top_centre_radius
    for di in (-r, -1, 0, 1, r):
        for dj in (-r, 0, r):
            nodes.add(m.node_id(cx + di, cy + dj, m.nz))
            nodes.add(m.node_id(cx + di, cy + dj, m.nz - 1))
    rng = np.random.default_rng(seed)
    nodes.update(int(v) for v in rng.integers(0, m.n_nodes, n_random))
    return np.array(sorted(nodes))


class LocalRows:
    """Oracle rows of the sampled nodes from the elements around them.  On a
    coarser level (level > 0) the state is the injection of the finest state
    and a dof is constrained iff its coincident finest dof is (the multigrid
    hierarchy's rediscretisation); only the operator rows are formed there."""

    def __init__(self, p, U, En, depth, nodes, level=0):
        m0 = Mesh.from_problem(p)
        mask0, target = S.dirichlet(m0, p.kind, p.patch, p.radius, depth=depth)
        g0 = S.increment(mask0, target, U)
        m = Mesh.from_problem(p, level)
        if level:
            f = 2 ** level
            I, J, K = m.node_ijk(np.arange(m.n_nodes))
            fid = m0.node_id(f * I, f * J, f * K)
            U, En, mask0, g0 = U[fid], En[fid], mask0[fid], np.zeros_like(g0[fid])
        self.m, self.nodes = m, nodes
        disc = Discretisation(m, Card(p.material))
        elems = m.elements_of_nodes(nodes)
        n = m.n_nodes * NDOF
        self.R = disc.residual(U.ravel(), En.ravel(), elems)
        r, c, v = disc.tangent_coo(U.ravel(), En.ravel(), elems)
        if p.kind == "sphere":
            sc = SphereContact(m, p.radius, p.eps_n)
            self.R = self.R + sc.residual(U.ravel(), depth)
            rc, cc, vc = sc.tangent_coo(U.ravel(), depth)
            r, c, v = np.concatenate([r, rc]), np.concatenate([c, cc]), np.concatenate([v, vc])
        self.K = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
        # rounding scale of the residual rows: sum of |element contributions|
        self.R_abs = residual_abs(disc, U, En, elems)
        if p.kind == "sphere":
            self.R_abs = self.R_abs + np.abs(sc.residual(U.ravel(), depth))
        self.mask = mask0
        self.g = g0.ravel()
        self.dofs = (nodes[:, None] * NDOF + np.arange(NDOF)).ravel()

    def rhs(self, absolute=False):
        """Sampled rows of the right-hand side; with absolute, their rounding
        scale sum_e |R_e| + |K| |g| (|g| on constrained dofs)."""
        m = self.mask.ravel()
        gv = np.where(m, self.g, 0.0)
        if absolute:
            b = self.R_abs[self.dofs] + abs(self.K[self.dofs]) @ np.abs(gv)
        else:
            b = -self.R[self.dofs] - self.K[self.dofs] @ gv
        con = m[self.dofs]
        b[con] = (np.abs(gv) if absolute else gv)[self.dofs][con]
        return b

    def apply(self, x, absolute=False):
        """Sampled rows of the eliminated operator times x; with absolute,
        (|A| |x|) on those rows (the rounding scale of the product)."""
        m = self.mask.ravel()
        K = abs(self.K) if absolute else self.K
        xf = np.where(m, 0.0, x)
        y = K[self.dofs] @ (np.abs(xf) if absolute else xf)
        con = m[self.dofs]
        y[con] = (np.abs(x) if absolute else x)[self.dofs][con]
        return y


class GalerkinRows:
    """Oracle rows of the Galerkin operator of a coarse level at sampled nodes
    of that level, A_l x = Q_l^T K Q_l x~ on free unknowns (x~ = x with the
    constrained coarse unknowns zeroed; constrained rows = x), with their
    rounding scale Q_l^T |K| Q_l |x~| (|x| on constrained rows).  Q_l e_I is
    supported on the finest nodes within 2^l - 1 of node 2^l I along every
    axis, so the finest rows of those nodes (LocalRows) fix the sampled rows;
    the transfers act on whole vectors, whose entries away from the samples
    are discarded."""

    def __init__(self, p, U, En, depth, level, nodes, x):
        m0, ml = Mesh.from_problem(p), Mesh.from_problem(p, level)
        self.shapes = [(m.nz, m.ny, m.nx) for m in (Mesh.from_problem(p, l) for l in range(level + 1))]
        mask0, _ = S.dirichlet(m0, p.kind, p.patch, p.radius, depth=depth)
        self.masks = coarse_masks(mask0.reshape(-1, NDOF), self.shapes[0], level + 1)
        f = 2 ** level
        I, J, K = ml.node_ijk(nodes)
        off = np.arange(-(f - 1), f)
        fi = (f * I[:, None, None, None] + off[None, None, None, :])
        fj = (f * J[:, None, None, None] + off[None, None, :, None])
        fk = (f * K[:, None, None, None] + off[None, :, None, None])
        fi, fj, fk = np.broadcast_arrays(fi, fj, fk)
        ok = (fi >= 0) & (fi <= m0.nx) & (fj >= 0) & (fj <= m0.ny) & (fk >= 0) & (fk <= m0.nz)
        support = np.unique(m0.node_id(fi[ok], fj[ok], fk[ok]))
        lr = LocalRows(p, U, En, depth, support)
        self.level, self.nodes = level, nodes
        self.dofs = (nodes[:, None] * NDOF + np.arange(NDOF)).ravel()
        x = np.asarray(x, dtype=float).reshape(-1, NDOF)
        xt = np.where(self.masks[level], 0.0, x)
        self.y = self._rows(lr, xt, x, False)
        self.y_abs = self._rows(lr, np.abs(xt), np.abs(x), True)

    def _rows(self, lr, xt, x, absolute):
        v = xt
        for l in range(self.level, 0, -1):
            v = np.where(self.masks[l - 1], 0.0, prolong_nodal(v, self.shapes[l]))
        Y = np.zeros(v.shape)
        Y.reshape(-1)[lr.dofs] = lr.apply(v.ravel(), absolute=absolute)
        for l in range(1, self.level + 1):
            Y = restrict_nodal(np.where(self.masks[l - 1], 0.0, Y), self.shapes[l])
        Y = np.where(self.masks[self.level], x, Y)
        return Y.ravel()[self.dofs]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check(p, depth, radius_nodes, tag, precision="mixed", coarse="galerkin", coarse_levels=False,
           galerkin_samples=(None, 6)):
    """Sampled rows of the residual, the right-hand side and the finest
    operator (FP64 copy; in mixed mode also the FP32 copy), each entry against
    the oracle's (element-wise, relative to its node's scale); with
    rediscretised coarse levels and coarse_levels, the sampled rows of every
    coarser level's operator; with Galerkin coarse levels, the sampled rows of
    levels 1 and 2 (galerkin_samples: the number of seeded random nodes among
    each level's samples, None = the default sample; level 2 keeps every other
    sampled node) and the identity
    A_l = P~^T A_{l-1} P~ on the deeper ones; then the solve's true FP64
    residual."""
    from paper_2011_08802_amd import mvpf
    m = Mesh.from_problem(p)
    U = np.zeros((m.n_nodes, NDOF))
    U[:, 3:] = p.eta0()
    nodes = sample_nodes(m, radius_nodes)
    say(f"[{tag}] oracle rows of {len(nodes)} sampled nodes")
    lr = LocalRows(p, U, U[:, 3:], depth, nodes)
    coarse_rows = []
    if coarse_levels:
        for l in range(1, p.n_levels):
            cm = Mesh.from_problem(p, l)
            cn = sample_nodes(cm, max(1, radius_nodes >> l), seed=17 + l)
            say(f"[{tag}] oracle rows of {len(cn)} sampled nodes on level {l}")
            coarse_rows.append((l, LocalRows(p, U, U[:, 3:], depth, cn, level=l)))
    galerkin = []
    if coarse == "galerkin":
        rng = np.random.default_rng(23)
        for l, nr in zip((1, 2), galerkin_samples):
            if l >= p.n_levels - 1:
                break
            cm = Mesh.from_problem(p, l)
            cn = sample_nodes(cm, max(1, radius_nodes >> l), seed=31 + l,
                              **({} if nr is None else {"n_random": nr}))[::l]  # level 2: every other one
            say(f"[{tag}] oracle Galerkin rows of {len(cn)} sampled nodes on level {l}")
            xc = rng.standard_normal(cm.n_nodes * NDOF)
            galerkin.append((xc, GalerkinRows(p, U, U[:, 3:], depth, l, cn, xc)))
    say(f"[{tag}] GPU system {p.nx}x{p.ny}x{p.nz} {precision}, {coarse} coarse operators")
    gp = mvpf.Problem(p, precision, rtol=1e-8, coarse=coarse)
    try:
        return _check_gpu(gp, p, depth, tag, precision, lr, coarse, coarse_rows, m, galerkin)
    finally:
        gp.close()


def _galerkin_identity(gp, p, depth, precision, first, tag):
    """Levels first..L-1: A_l x against P~^T A_{l-1} P~ x~ on the free
    unknowns (constrained rows: x), both operators the GPU's; norm-wise
    relative error of the free part.  The mixed mode keeps FP32 copies of the
    levels above the coarsest (entries rounded from the FP64 products, applied
    in FP32): 1e-5 there, about 100 units of FP32 rounding; FP64 copies: 1e-11."""
    from paper_2011_08802_amd import mvpf
    shapes = [(m.nz, m.ny, m.nx) for m in (Mesh.from_problem(p, l) for l in range(p.n_levels))]
    mask0, _ = S.dirichlet(Mesh.from_problem(p), p.kind, p.patch, p.radius, depth=depth)
    mask0 = mask0.reshape(-1, NDOF)
    masks = coarse_masks(mask0, shapes[0], p.n_levels)
    rng = np.random.default_rng(29)

    def prec(l):
        return mvpf.FP64 if precision == "fp64" or l in (0, p.n_levels - 1) else mvpf.MIXED

    for l in range(first, p.n_levels):
        x = rng.standard_normal((masks[l].shape[0], NDOF))
        xt = np.where(masks[l], 0.0, x)
        v = np.where(masks[l - 1], 0.0, prolong_nodal(xt, shapes[l]))
        w = gp.jacobian_apply(l - 1, torch.as_tensor(v.ravel()).cuda(), prec(l - 1)).cpu().numpy()
        ref = restrict_nodal(np.where(masks[l - 1], 0.0, w.reshape(-1, NDOF)), shapes[l])
        y = gp.jacobian_apply(l, torch.as_tensor(x.ravel()).cuda(), prec(l)).cpu().numpy().reshape(-1, NDOF)
        free = ~masks[l]
        err = _rel(y[free], ref[free])
        tol = 1e-11 if prec(l) == prec(l - 1) == mvpf.FP64 else 1e-5
        say(f"    Galerkin identity level {l}: relative error {err:.2e} (free), "
            f"constrained rows {float(np.abs(y[~free] - x[~free]).max(initial=0.0)):.1e}")
        assert err <= tol, (tag, l, err)
        assert np.allclose(y[~free], x[~free], rtol=1e-7, atol=0), (tag, l)


def _check_gpu(gp, p, depth, tag, precision, lr, coarse, coarse_rows, m, galerkin):
    from paper_2011_08802_amd import mvpf
    assert gp.get_tuning("matrix_free") == 1
    gp.init_random(p.seed)
    gp.newton_system(depth)
    gp.autotune()
    R, _ = gp.residual()
    check_entries(R.cpu().numpy()[lr.dofs], lr.R[lr.dofs], 1e-12, "residual", lr.R_abs[lr.dofs])
    check_entries(gp.get_rhs().cpu().numpy()[lr.dofs], lr.rhs(), 1e-12, "rhs", lr.rhs(absolute=True))
    rng = np.random.default_rng(5)
    x = rng.standard_normal(m.n_nodes * NDOF)
    xd = torch.as_tensor(x).cuda()
    yo, ya = lr.apply(x), lr.apply(x, absolute=True)
    check_entries(gp.jacobian_apply(0, xd, mvpf.FP64).cpu().numpy()[lr.dofs], yo, 1e-12, "FP64 K x", ya)
    if precision == "mixed":
        check_entries(gp.jacobian_apply(0, xd, mvpf.MIXED).cpu().numpy()[lr.dofs], yo, 2e-6, "FP32 K x", ya)
    for l, cr in coarse_rows:
        xc = rng.standard_normal(cr.m.n_nodes * NDOF)
        yc = gp.jacobian_apply(l, torch.as_tensor(xc).cuda(), mvpf.FP64).cpu().numpy()[cr.dofs]
        check_entries(yc, cr.apply(xc), 1e-12, f"FP64 K x level {l}", cr.apply(xc, absolute=True))
    for xc, gr in galerkin:
        l = gr.level
        pr = mvpf.FP64 if precision == "fp64" or l == p.n_levels - 1 else mvpf.MIXED
        yc = gp.jacobian_apply(l, torch.as_tensor(xc).cuda(), pr).cpu().numpy()[gr.dofs]
        check_entries(yc, gr.y, 1e-12 if pr == mvpf.FP64 else 2e-6,
                      f"{'FP64' if pr == mvpf.FP64 else 'FP32'} Galerkin K x level {l}", gr.y_abs)
    if coarse == "galerkin":
        _galerkin_identity(gp, p, depth, precision, len(galerkin) + 1, tag)
    say(f"[{tag}] solve")
    dx, st = gp.solve()
    b = gp.get_rhs()
    r = b - gp.jacobian_apply(0, dx, mvpf.FP64)
    assert st.converged and st.rel_residual <= 1e-8
    assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= 1.0001e-8
    return st


def test_fullsize_patch_64():
    """The 64^3 patch workload (2,471,625 dof, 5 levels), Galerkin levels."""
    p = synth.medium()
    _check(p, p.depth_increment, p.patch // 2 + 1, "64^3")


def test_fullsize_patch_64_fp64():
    """The 64^3 patch workload in the plain FP64 method (every multigrid level
    and the smoother in FP64): sampled rows of the residual, the right-hand
    side and the operator on all 5 levels (the coarser ones rediscretised at
    the injected state, the paper's hierarchy), and the solve's true FP64
    residual."""
    p = synth.medium()
    _check(p, p.depth_increment, p.patch // 2 + 1, "64^3 fp64", precision="fp64", coarse="rediscretise",
           coarse_levels=True)


def test_fullsize_patch_128():
    """The 128^3 patch workload (19,320,201 dof, 5 levels), Galerkin levels."""
    p = synth.large()
    _check(p, p.depth_increment, p.patch // 2 + 1, "128^3")


def test_fullsize_cap_scale():
    """The 256x256x128 spherical-cap workload on the 1x1x0.5 box (76,682,889
    dof, 6 levels): the cap of radius 0.2 pushed 0.0025 touches the top nodes
    within sqrt(2*0.2*0.0025) = 0.0316 of the centre, about 8 node spacings;
    the sampled top nodes straddle that rim.  Galerkin levels, as benchmarked."""
    p = synth.scale_limit()
    _check(p, p.depth_increment, 8, "256x256x128")


def test_fullsize_batched():
    """The batched workload at full size (32 problems of n^3 elements, n in
    {16,...,48}, own rotation, seed and depth, 4 levels), solved in lockstep:
    every problem's sampled rows of the right-hand side and of the FP64 and
    FP32 finest operators against the oracle, and every increment's true FP64
    relative residual, b - J dx with dx = the state change of the update and J
    assembled again from the initial state (assembly is deterministic: the
    right-hand side must come out bitwise the same)."""
    from paper_2011_08802_amd import mvpf
    probs = synth.batched(32)
    rows = []
    for i, p in enumerate(probs):
        m = Mesh.from_problem(p)
        U = np.zeros((m.n_nodes, NDOF))
        U[:, 3:] = p.eta0()
        rows.append((U, LocalRows(p, U, U[:, 3:], p.depth_increment, sample_nodes(m, p.patch // 2 + 1, seed=17 + i))))
    say(f"[batch] GPU systems of {len(probs)} problems")
    B = mvpf.Batch(probs, "mixed", rtol=1e-8)
    try:
        _batched_gpu(B, probs, rows)
    finally:
        B.close()


def _batched_gpu(B, probs, rows):
    from paper_2011_08802_amd import mvpf
    for i, p in enumerate(probs):
        B.problem(i).init_random(p.seed)
    depths = [p.depth_increment for p in probs]
    B.newton_system(depths)
    for i in range(len(probs)):
        B.problem(i).autotune()
    B.newton_system(depths)
    rng = np.random.default_rng(5)
    bs = []
    for i, (U, lr) in enumerate(rows):
        gp = B.problem(i)
        R, _ = gp.residual()
        check_entries(R.cpu().numpy()[lr.dofs], lr.R[lr.dofs], 1e-12, f"problem {i} residual", lr.R_abs[lr.dofs])
        b = gp.get_rhs()
        check_entries(b.cpu().numpy()[lr.dofs], lr.rhs(), 1e-12, f"problem {i} rhs", lr.rhs(absolute=True))
        x = rng.standard_normal(U.size)
        xd = torch.as_tensor(x).cuda()
        yo, ya = lr.apply(x), lr.apply(x, absolute=True)
        check_entries(gp.jacobian_apply(0, xd, mvpf.FP64).cpu().numpy()[lr.dofs], yo, 1e-12, f"problem {i} FP64 K x", ya)
        check_entries(gp.jacobian_apply(0, xd, mvpf.MIXED).cpu().numpy()[lr.dofs], yo, 2e-6, f"problem {i} FP32 K x", ya)
        bs.append(b)
    say("[batch] lockstep solve")
    stats = B.solve()
    B.newton_update()
    dxs = []
    for i, (U, lr) in enumerate(rows):
        assert stats[i].converged and stats[i].rel_residual <= 1e-8, (i, stats[i].rel_residual)
        u, e, _, _ = B.problem(i).get_state()
        dxs.append(torch.cat([u, e], 1).reshape(-1) - torch.as_tensor(U.ravel()).cuda())
        B.problem(i).set_state(U[:, :3], U[:, 3:], U[:, 3:], 0.0)
    say("[batch] true residuals (the same systems assembled again)")
    B.newton_system(depths)
    for i, (b, dx) in enumerate(zip(bs, dxs)):
        assert torch.equal(B.problem(i).get_rhs(), b), i
        r = b - B.problem(i).jacobian_apply(0, dx, mvpf.FP64)
        assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= 1.0001e-8, i


def test_fullsize_sphere_indentation():
    """The 64x64x32 sphere-contact workload (1,254,825 dof, 5 levels) at
    depth 0.02: the sampled top nodes include nodes in contact.  Galerkin
    levels (the contact stiffness enters them through the finest tangent)."""
    p = synth.indentation()
    _check(p, 0.02, 6, "indent")
