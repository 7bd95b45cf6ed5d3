"""Seeded synthetic inputs for the indentation workloads.

This module is used by the tests, the benchmark and the CPU oracle (the HIP
path's binding imports nothing from it; callers hand it Problem objects).  It
holds raw input values only -- mesh sizes, loading geometry,
material constants as printed in the paper, seeds and counter-based random
numbers -- and none of the method's arithmetic (no stiffness rotation, no
transformation stretch matrices, no boundary-condition logic).

Random numbers: splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used as a counter hash.  The initial order
parameter of node ``a`` and variant ``i`` (1-based, i = 1..6) is
``0.05 * (splitmix64(seed ^ (9*a + 3 + (i-1))) >> 11) * 2**-53``, i.e. uniform
in [0, 0.05).  The counter ``9*a + 3 + (i-1)`` is the node-interleaved dof index
of that order parameter.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

MASK64 = (1 << 64) - 1
BASE_SEED = 20110880


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function applied to the counters ``x`` (uint64 array).

    z = x + 0x9E3779B97F4A7C15; z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB; return z ^ (z >> 31).
    """
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0,1) from 53 high bits of splitmix64(seed ^ counter)."""
    c = np.asarray(counters, dtype=np.uint64) ^ np.uint64(seed & MASK64)
    return (splitmix64(c) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def initial_eta(seed: int, n_nodes: int, amplitude: float = 0.05, n_var: int = 6) -> np.ndarray:
    """Initial order parameters, shape (n_nodes, n_var), uniform in
    [0, amplitude); the counter of node a and variant i (0-based) is its
    node-interleaved dof index (3 + n_var) a + 3 + i."""
    a = np.arange(n_nodes, dtype=np.uint64)[:, None]
    i = np.arange(n_var, dtype=np.uint64)[None, :]
    return amplitude * uniform01(seed, np.uint64(3 + n_var) * a + np.uint64(3) + i)


# ---------------------------------------------------------------------------
# Material constants as printed in the paper (Table 1, Section 4.1) and the
# nondimensional card used by the synthetic workloads.
# ---------------------------------------------------------------------------

@dataclass
class MaterialParams:
    """Raw material inputs (GPa for stresses/energy densities, domain width = 1).

    cubic: (c11, c12, c44) of the austenite (Table 1).
    ortho: (c11, c22, c33, c44, c55, c66, c12, c13, c23) of the martensite in
           its own orthorhombic axes (Table 1).
    alpha, beta, gamma: transformation stretch parameters.
    Q: rotation, rows = sample axes expressed in cubic-crystal coordinates.
    F0: chemical energy densities of the 7 phases (austenite first).
    w_am, w_mm: double-obstacle barrier coefficients 4*gamma_ij/(pi*l_ij).
    ell: interface thickness parameter l_ij (same for all pairs).
    rho: viscous coefficient 1/(m*tau) (same for all phases).
    eps_eta: penalty parameter of the order-parameter constraints.
    pade: Pade order of the Hencky strain approximation (11, 22 or 33 = (1,1), (2,2), (3,3)).
    """
    cubic: tuple = (142.0, 126.0, 96.0)
    ortho: tuple = (189.0, 141.0, 205.0, 54.9, 19.7, 62.6, 124.0, 45.5, 115.0)
    alpha: float = 1.0424
    beta: float = 0.9178
    gamma: float = 1.0619
    Q: tuple = tuple(np.eye(3).ravel())
    F0: tuple = (0.0, 0.005, 0.005, 0.005, 0.005, 0.005, 0.005)
    w_am: float = 0.25
    w_mm: float = 0.025
    ell: float = 0.01
    rho: float = 1.0
    eps_eta: float = 1000.0
    pade: int = 22
    mixing: str = "linear"
    n_var: int = 6


@dataclass
class OrbitMaterial:
    """Raw inputs of a synthetic card with N variants generated from one
    stretch tensor by the cubic symmetry (the variants are the distinct
    images Q U1 Q^T under the 24 rotations of the cube, each with L1 rotated
    alike).  Stresses in GPa.

    U1: variant 1's stretch tensor (row-major 3x3, symmetric, cubic axes).
    L1: variant 1's stiffness, 6x6 Voigt (order 11,22,33,23,13,12,
        engineering shear strains), cubic axes.
    cubic: austenite (c11, c12, c44).  Q: sample rotation (rows = sample
    axes in cubic coordinates).  F0_a, F0_m: chemical energy of the
    austenite and of every variant.  n_var: the number of distinct variants
    the orbit gives (stated, so that sizes are known without building the
    card)."""
    U1: tuple
    L1: tuple
    n_var: int
    cubic: tuple = (142.0, 126.0, 96.0)
    Q: tuple = tuple(np.eye(3).ravel())
    F0_a: float = 0.0
    F0_m: float = 0.005
    w_am: float = 0.25
    w_mm: float = 0.025
    ell: float = 0.01
    rho: float = 1.0
    eps_eta: float = 1000.0
    pade: int = 22
    mixing: str = "linear"


def _ortho_voigt(c11, c22, c33, c44, c55, c66, c12, c13, c23):
    """The nine orthotropic constants laid out as a 6x6 Voigt matrix (raw
    layout of input values, row-major)."""
    return (c11, c12, c13, 0, 0, 0,
            c12, c22, c23, 0, 0, 0,
            c13, c23, c33, 0, 0, 0,
            0, 0, 0, c44, 0, 0,
            0, 0, 0, 0, c55, 0,
            0, 0, 0, 0, 0, c66)


def twelve_variant_material(**over) -> OrbitMaterial:
    """A synthetic 12-variant card (not NiTi data): a monoclinic-type
    stretch U1 = [[1.05, 0.02, 0.02], [0.02, 0.98, 0.04], [0.02, 0.04, 0.98]]
    (eigenvalues 0.940, 1.003, 1.067; 12 distinct images under the cubic
    rotations) with the orthorhombic constants of Table 1 as its stiffness in
    the cubic axes, the austenite and the remaining coefficients of the
    six-variant workloads, [011] along z."""
    base = dict(U1=(1.05, 0.02, 0.02, 0.02, 0.98, 0.04, 0.02, 0.04, 0.98),
                L1=_ortho_voigt(*MaterialParams().ortho), n_var=12, Q=Q_011_Z)
    base.update(over)
    return OrbitMaterial(**base)


# Sample axes x = [100], y = [01-1]/sqrt2, z = [011]/sqrt2: the [011] crystal
# direction is the loading (z) axis, as in the paper's indentation problem.
S2 = 1.0 / np.sqrt(2.0)
Q_011_Z = (1.0, 0.0, 0.0,
           0.0, S2, -S2,
           0.0, S2, S2)

PAPER_STRETCHES = dict(alpha=1.0619, beta=0.9178, gamma=1.0230)


def config_material(**over) -> MaterialParams:
    """Material card of the synthetic indentation workloads ([011] along z)."""
    return replace(MaterialParams(Q=Q_011_Z), **over)


@dataclass
class Problem:
    """One synthetic indentation problem on a structured Q1 hex mesh.

    The domain is [0,lx]x[0,ly]x[0,lz] cut into nx*ny*nz cubes of side h.
    Loading kind 'patch': the top-face nodes within the centred square of
    ``patch`` x ``patch`` elements get a prescribed vertical displacement
    increment of ``-depth_increment`` per step.  Kind 'cap': spherical cap
    profile of radius ``radius`` (see the library header).  Kind 'sphere':
    no prescribed top displacements; a rigid sphere of radius ``radius``
    centred above the top face acts by penalty contact with parameter
    ``eps_n`` (energy per area per squared length; the paper's 10^2 GPa/nm is
    3.5e4 in units of a 350 nm domain width).  ``n_levels`` is the number of
    multigrid levels (each coarsening halves nx, ny, nz).
    """
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    n_levels: int = 3
    kind: str = "patch"
    patch: int = 2
    radius: float = 0.2
    eps_n: float = 3.5e4
    depth_increment: float = 0.02
    steps: int = 1
    seed: int = BASE_SEED
    material: MaterialParams = field(default_factory=config_material)

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_var(self) -> int:
        return self.material.n_var

    @property
    def n_dof(self) -> int:
        return (3 + self.n_var) * self.n_nodes

    def eta0(self) -> np.ndarray:
        return initial_eta(self.seed, self.n_nodes, n_var=self.n_var)


def tiny() -> Problem:
    """8^3 unit cube, 2x2 patch pushed 0.02 in one step, 3 levels, FP64."""
    return Problem(8, 8, 8, n_levels=3, patch=2, depth_increment=0.02, steps=1)


def medium() -> Problem:
    """64^3 unit cube (2,471,625 dof), 8x8 patch, 5 steps of 0.01, 5 levels."""
    return Problem(64, 64, 64, n_levels=5, patch=8, depth_increment=0.01, steps=5)


def large() -> Problem:
    """128^3 unit cube (19,320,201 dof), 16x16 patch, 10 steps of 0.005, 5 levels."""
    return Problem(128, 128, 128, n_levels=5, patch=16, depth_increment=0.005, steps=10)


def scale_limit() -> Problem:
    """256x256x128 (76,682,889 dof), domain 1x1x0.5, spherical cap R=0.2, 20 steps."""
    return Problem(256, 256, 128, lz=0.5, n_levels=6, kind="cap", radius=0.2,
                   depth_increment=0.0025, steps=20)


def indentation() -> Problem:
    """64x64x32 hex elements (1 254 825 dof), domain 1x1x0.5, rigid sphere
    R = 0.2 in penalty contact (eps_N = 3.5e4), 5 levels (4x4x2 coarsest)."""
    return Problem(64, 64, 32, lz=0.5, n_levels=5, kind="sphere", radius=0.2, depth_increment=0.0025)


# Indentation run of the workload above: load to depth 0.03 and unload at
# v / m = 2.857e-4 GPa (the paper's v = 1 nm/s and m = 0.01 (MPa s)^-1 in
# units of a 350 nm domain width), steps from 0.0005 within [1e-5, 0.005].
INDENT_RUN = dict(depth_max=0.03, dd_init=0.0005, dd_min=1e-5, dd_max=0.005, visc_depth=2.857e-4)


def random_rotation(seed: int) -> np.ndarray:
    """Rotation matrix from a normalised quaternion with four uniform-derived
    Gaussian components (Box-Muller on splitmix64 counters 0..7)."""
    u = uniform01(seed, np.arange(8, dtype=np.uint64))
    u = np.clip(u, 1e-300, 1.0)
    g = np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * np.pi * u[1::2])
    w, x, y, z = g / np.linalg.norm(g)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def batched(n_problems: int = 32, base_seed: int = BASE_SEED) -> List[Problem]:
    """Independent problems with n in {16,24,32,40,48}, depth U[0.005,0.02],
    a random crystal rotation and their own eta seed (problem p: base + p).
    The top patch spans 2*max(1, n//16) elements (even, so it is centred on a
    node).  Levels: n is halved while it is even and the half is at least 2
    (48: 5 levels down to 3^3, 40: 4 down to 5^3, 32: 5 down to 2^3, 24: 4
    down to 3^3, 16: 4 down to 2^3), so no coarsest level exceeds 1944
    unknowns."""
    out = []
    for p in range(n_problems):
        s = base_seed + p
        u = uniform01(s, np.array([1001, 1002], dtype=np.uint64))
        n = (16, 24, 32, 40, 48)[min(int(u[0] * 5), 4)]
        d = 0.005 + 0.015 * u[1]
        Q = random_rotation(s)
        levels, m = 1, n
        while m % 2 == 0 and m // 2 >= 2:
            m //= 2
            levels += 1
        out.append(Problem(n, n, n, n_levels=levels, patch=2 * max(1, n // 16),
                           depth_increment=float(d), steps=1, seed=s,
                           material=config_material(Q=tuple(Q.ravel()))))
    return out
