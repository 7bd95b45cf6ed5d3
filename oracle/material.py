"""Material card: transformation stretches and elastic stiffnesses.

Oracle (test infrastructure only; see the package docstring).

* Transformation stretch tensors of the six orthorhombic CuAlNi variants in the
  cubic basis: Sec. 4.1, matrices U_{1,2}, U_{3,4}, U_{5,6}; U_0 = I for the
  austenite (Sec. 2.1, Eq. LinMix).
* Stiffnesses: Table 1.  Cubic austenite (c11, c12, c44); orthorhombic
  martensite (c11..c66, c12, c13, c23).  The table gives the martensite
  constants in the orthorhombic axes; each variant's axes are the principal
  axes of its stretch tensor, axis 1 <-> alpha, axis 2 <-> beta,
  axis 3 <-> gamma (reading of Sec. 4.1 + Table 1).
* Everything is finally rotated into the sample frame by Q (rows of Q are the
  sample axes in cubic coordinates), Sec. 4.1: [011] parallel to the loading
  axis z.

A second kind of card describes materials with any number N of variants
(the paper's footnote in Sec. 4.4 mentions NiTi with 12 variants, i.e. 15
unknowns per node): the variants are the distinct images Q U_1 Q^T of one
given stretch tensor U_1 under the 24 rotations of the cube (the
transformation's crystallographic equivalence, Sec. 2.1), each with the
stiffness L_1 rotated alike.  No NiTi data is used: the values are synthetic.

Mixing rule of the transformation stretch (Sec. 2.1): linear, F^t = sum
eta_i U_i (Eq. LinMix, the paper's choice), or logarithmic, F^t =
exp(sum eta_i log U_i) (the alternative the paper discusses); log U_i of the
symmetric positive definite U_i is taken through its spectral decomposition.

Fourth-order tensors are kept as full 3x3x3x3 arrays (no Voigt bookkeeping)
so that each operation can be checked by eye.
"""
from __future__ import annotations

import numpy as np

R2 = 1.0 / np.sqrt(2.0)

# Voigt index map used only to read the tabulated 6x6 constants:
# 0:11 1:22 2:33 3:23 4:13 5:12
_VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3,
          (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}


def stretch_tensors(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """U_0..U_6 in the cubic basis (Sec. 4.1), shape (7, 3, 3)."""
    p = 0.5 * (alpha + gamma)
    m = 0.5 * (alpha - gamma)
    U = np.zeros((7, 3, 3))
    U[0] = np.eye(3)
    for k, s in ((1, 1.0), (2, -1.0)):
        U[k] = [[p, 0, s * m], [0, beta, 0], [s * m, 0, p]]
    for k, s in ((3, 1.0), (4, -1.0)):
        U[k] = [[p, s * m, 0], [s * m, p, 0], [0, 0, beta]]
    for k, s in ((5, 1.0), (6, -1.0)):
        U[k] = [[beta, 0, 0], [0, p, s * m], [0, s * m, p]]
    return U


def variant_axes() -> np.ndarray:
    """Columns = (alpha-, beta-, gamma-) principal axes of U_1..U_6 in the
    cubic basis, shape (7, 3, 3); entry 0 is the identity (austenite).

    Derived from the matrices of Sec. 4.1: e.g. U_1 maps (1,0,1)/sqrt2 to
    alpha times itself, (0,1,0) to beta, (1,0,-1)/sqrt2 to gamma.
    """
    R = np.zeros((7, 3, 3))
    R[0] = np.eye(3)
    cols = {
        1: ([R2, 0, R2], [0, 1, 0], [R2, 0, -R2]),
        2: ([R2, 0, -R2], [0, 1, 0], [R2, 0, R2]),
        3: ([R2, R2, 0], [0, 0, 1], [R2, -R2, 0]),
        4: ([R2, -R2, 0], [0, 0, 1], [R2, R2, 0]),
        5: ([0, R2, R2], [1, 0, 0], [0, R2, -R2]),
        6: ([0, R2, -R2], [1, 0, 0], [0, R2, R2]),
    }
    for k, (a, b, g) in cols.items():
        R[k] = np.array([a, b, g], dtype=float).T
    return R


def voigt_to_tensor(C6: np.ndarray) -> np.ndarray:
    """Full stiffness L_ijkl = C6[v(ij), v(kl)] from a 6x6 Voigt matrix."""
    L = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    L[i, j, k, l] = C6[_VOIGT[(i, j)], _VOIGT[(k, l)]]
    return L


def cubic_stiffness(c11: float, c12: float, c44: float) -> np.ndarray:
    C6 = np.zeros((6, 6))
    C6[:3, :3] = c12
    np.fill_diagonal(C6[:3, :3], c11)
    C6[3, 3] = C6[4, 4] = C6[5, 5] = c44
    return voigt_to_tensor(C6)


def orthorhombic_stiffness(c11, c22, c33, c44, c55, c66, c12, c13, c23) -> np.ndarray:
    C6 = np.array([
        [c11, c12, c13, 0, 0, 0],
        [c12, c22, c23, 0, 0, 0],
        [c13, c23, c33, 0, 0, 0],
        [0, 0, 0, c44, 0, 0],
        [0, 0, 0, 0, c55, 0],
        [0, 0, 0, 0, 0, c66],
    ], dtype=float)
    return voigt_to_tensor(C6)


def rotate4(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """L'_ijkl = R_ia R_jb R_kc R_ld L_abcd."""
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, L)


def rotate2(A: np.ndarray, R: np.ndarray) -> np.ndarray:
    return R @ A @ R.T


def cubic_rotations() -> list:
    """The 24 proper rotations of the cube: signed permutation matrices with
    determinant +1, Q[i, perm[i]] = sign[i], in a fixed order (permutations
    of (0, 1, 2) in lexicographic order, then sign patterns with the sign of
    row 0 varying slowest, + before -)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            Q = np.zeros((3, 3))
            for i in range(3):
                Q[i, perm[i]] = signs[i]
            if np.linalg.det(Q) > 0:
                out.append(Q)
    return out


def orbit_variants(U1: np.ndarray, tol: float = 1e-12):
    """Distinct Q U1 Q^T over cubic_rotations(), in that order, with the
    first rotation that produces each: (list of U_k, list of R_k)."""
    Us, Rs = [], []
    for Q in cubic_rotations():
        V = Q @ U1 @ Q.T
        if not any(np.max(np.abs(V - W)) <= tol for W in Us):
            Us.append(V)
            Rs.append(Q)
    return Us, Rs


def spd_log(U: np.ndarray) -> np.ndarray:
    """log U of a symmetric positive definite matrix: V diag(log lambda) V^T."""
    lam, V = np.linalg.eigh(U)
    return V @ np.diag(np.log(lam)) @ V.T


class Card:
    """All material data in the sample frame.

    U   (7,3,3)      transformation stretches, U[0] = I
    L   (7,3,3,3,3)  phase stiffnesses (GPa)
    F0  (7,)         chemical energies
    W   (7,7)        double-obstacle coefficients w_ij = 4 gamma_ij/(pi l_ij),
                     zero diagonal
    ell2 (7,7)       l_ij^2
    rho (7,)         viscous coefficients 1/(m_i tau)
    eps              penalty parameter eps_eta
    """

    def __init__(self, mp):
        if hasattr(mp, "U1"):  # a card generated from one stretch tensor
            self._init_orbit(mp)
            return
        Q = np.asarray(mp.Q, dtype=float).reshape(3, 3)
        Uc = stretch_tensors(mp.alpha, mp.beta, mp.gamma)
        Rv = variant_axes()
        L0c = cubic_stiffness(*mp.cubic)
        Lm = orthorhombic_stiffness(*mp.ortho)
        self.U = np.stack([rotate2(Uc[k], Q) for k in range(7)])
        Lc = [L0c] + [rotate4(Lm, Rv[k]) for k in range(1, 7)]
        self.L = np.stack([rotate4(Lk, Q) for Lk in Lc])
        self.F0 = np.asarray(mp.F0, dtype=float)
        W = np.full((7, 7), mp.w_mm)
        W[0, :] = W[:, 0] = mp.w_am
        np.fill_diagonal(W, 0.0)
        self.W = W
        self.ell2 = np.full((7, 7), mp.ell ** 2)
        self.rho = np.full(7, mp.rho)
        self.eps = float(mp.eps_eta)
        self.pade = int(mp.pade)
        self._mixing(getattr(mp, "mixing", "linear"))

    def _mixing(self, mixing: str):
        if mixing not in ("linear", "log"):
            raise ValueError(f"unknown mixing rule {mixing}")
        self.mixing = mixing
        self.logU = np.stack([spd_log(U) for U in self.U])

    @property
    def n_var(self) -> int:
        return self.U.shape[0] - 1

    def _init_orbit(self, om):
        """Card of N variants from one stretch tensor (see the module
        docstring): om holds U1 (3x3, cubic axes), L1 (6x6 Voigt, engineering
        shear, cubic axes), cubic (austenite c11, c12, c44), Q (sample
        rotation), F0_a, F0_m, w_am, w_mm, ell, rho, eps_eta, pade, mixing."""
        c = self
        Q = np.asarray(om.Q, dtype=float).reshape(3, 3)
        Us, Rs = orbit_variants(np.asarray(om.U1, dtype=float).reshape(3, 3))
        L1 = voigt_to_tensor(np.asarray(om.L1, dtype=float).reshape(6, 6))
        n = len(Us)
        c.U = np.stack([np.eye(3)] + [rotate2(U, Q) for U in Us])
        c.L = np.stack([rotate4(cubic_stiffness(*om.cubic), Q)] + [rotate4(rotate4(L1, R), Q) for R in Rs])
        c.F0 = np.array([om.F0_a] + [om.F0_m] * n)
        W = np.full((n + 1, n + 1), om.w_mm)
        W[0, :] = W[:, 0] = om.w_am
        np.fill_diagonal(W, 0.0)
        c.W = W
        c.ell2 = np.full((n + 1, n + 1), om.ell ** 2)
        c.rho = np.full(n + 1, om.rho)
        c.eps = float(om.eps_eta)
        c.pade = int(om.pade)
        c._mixing(om.mixing)
        if c.n_var != om.n_var:
            raise ValueError(f"the orbit of U1 has {c.n_var} variants, the card states {om.n_var}")
