"""ctypes binding of libmvpf (include/mvpf.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory
(CUDA/HIP tensors) and the stream.  ``Problem`` methods map one-to-one onto the
C calls: ``Problem.X(...)`` calls ``mvpf_X`` on the handle.  If the library is
not built, ``load()`` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmvpf.so")


def lib_path(nvar: int = 6) -> str:
    """The library built for nvar martensite variants (a compile-time
    constant of its kernels): libmvpf.so for 6, libmvpf_n<N>.so otherwise."""
    return LIB_PATH if nvar == 6 else os.path.join(HERE, f"libmvpf_n{nvar}.so")

FP64, MIXED = 0, 1
MIX_LINEAR, MIX_LOG = 0, 1
LOAD_PATCH, LOAD_CAP, LOAD_SPHERE = 0, 1, 2
COARSE_REDISCRETISE, COARSE_GALERKIN = 0, 1
COARSE = {"rediscretise": COARSE_REDISCRETISE, "galerkin": COARSE_GALERKIN}
_LOAD_KINDS = {"patch": LOAD_PATCH, "cap": LOAD_CAP, "sphere": LOAD_SPHERE}
OK, ENOTCONV = 0, 1
MAX_COARSE_DOF = 8192

_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESINGULAR", -5: "ESTATE", 1: "ENOTCONV"}


class MvpfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mvpf error {_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double), ("n_levels", C.c_int)]


class Material(C.Structure):
    _fields_ = [("cubic", C.c_double * 3), ("ortho", C.c_double * 9), ("alpha", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("Q", C.c_double * 9), ("F0", C.c_double * 7),
                ("w_am", C.c_double), ("w_mm", C.c_double), ("ell", C.c_double), ("rho", C.c_double),
                ("eps_eta", C.c_double), ("pade", C.c_int), ("mixing", C.c_int)]


class OrbitMaterial(C.Structure):
    _fields_ = [("U1", C.c_double * 9), ("L1", C.c_double * 36), ("cubic", C.c_double * 3), ("Q", C.c_double * 9),
                ("F0_a", C.c_double), ("F0_m", C.c_double), ("w_am", C.c_double), ("w_mm", C.c_double),
                ("ell", C.c_double), ("rho", C.c_double), ("eps_eta", C.c_double), ("pade", C.c_int),
                ("mixing", C.c_int)]


class Loading(C.Structure):
    _fields_ = [("kind", C.c_int), ("patch", C.c_int), ("radius", C.c_double), ("eps_n", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("restart", C.c_int), ("max_it", C.c_int),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("omega", C.c_double), ("newton_max", C.c_int),
                ("newton_rtol", C.c_double), ("coarse", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("solve_ms", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("newton_iterations", C.c_int), ("linear_iterations", C.c_int), ("halvings", C.c_int),
                ("converged", C.c_int), ("residual0", C.c_double), ("residual", C.c_double),
                ("assemble_ms", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


class IndentOpts(C.Structure):
    _fields_ = [("depth_max", C.c_double), ("unload", C.c_int), ("dd_init", C.c_double), ("dd_min", C.c_double),
                ("dd_max", C.c_double), ("grow", C.c_double), ("shrink", C.c_double), ("newton_desired", C.c_int),
                ("visc_depth", C.c_double), ("max_steps", C.c_int)]


class IndentRecord(C.Structure):
    _fields_ = [("depth", C.c_double), ("load", C.c_double), ("dd", C.c_double), ("newton_iterations", C.c_int),
                ("linear_iterations", C.c_int), ("rejected", C.c_int), ("assemble_ms", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


IndentCallback = C.CFUNCTYPE(None, C.POINTER(IndentRecord), C.c_int, C.c_void_p)


class Info(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("nx", C.c_int * 8), ("ny", C.c_int * 8), ("nz", C.c_int * 8),
                ("n_nodes", C.c_int64 * 8), ("bytes_device", C.c_int64)]


# exported symbols: name -> (restype, argtypes)
_P = C.c_void_p
_D = C.POINTER(C.c_double)
SIGNATURES = {
    "mvpf_default_opts": (None, [C.POINTER(Opts)]),
    "mvpf_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Material), C.POINTER(Loading), C.POINTER(Opts), _P,
                              C.POINTER(_P)]),
    "mvpf_create_orbit": (C.c_int, [C.POINTER(Mesh), C.POINTER(OrbitMaterial), C.POINTER(Loading), C.POINTER(Opts),
                                    _P, C.POINTER(_P)]),
    "mvpf_nvar": (C.c_int, []),
    "mvpf_destroy": (None, [_P]),
    "mvpf_last_error": (C.c_char_p, [_P]),
    "mvpf_get_info": (C.c_int, [_P, C.POINTER(Info)]),
    "mvpf_set_opts": (C.c_int, [_P, C.POINTER(Opts)]),
    "mvpf_set_state": (C.c_int, [_P, _P, _P, _P, C.c_double]),
    "mvpf_get_state": (C.c_int, [_P, _P, _P, _P, _D]),
    "mvpf_init_random": (C.c_int, [_P, C.c_uint64]),
    "mvpf_residual": (C.c_int, [_P, _P, _D]),
    "mvpf_residual_noalloc": (C.c_int, [_P, _P, _D]),
    "mvpf_residual_noalloc_max_layer": (C.c_int, []),
    "mvpf_newton_system": (C.c_int, [_P, C.c_double]),
    "mvpf_get_rhs": (C.c_int, [_P, _P]),
    "mvpf_jacobian_apply": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "mvpf_precondition": (C.c_int, [_P, _P, _P]),
    "mvpf_solve": (C.c_int, [_P, _P, _P, C.POINTER(SolveStats)]),
    "mvpf_newton_update": (C.c_int, [_P]),
    "mvpf_newton_step": (C.c_int, [_P, C.c_double, C.POINTER(SolveStats)]),
    "mvpf_time_step": (C.c_int, [_P, C.c_double, C.POINTER(StepStats)]),
    "mvpf_set_viscosity": (C.c_int, [_P, C.c_double]),
    "mvpf_contact_load": (C.c_int, [_P, _D]),
    "mvpf_default_indent_opts": (None, [C.POINTER(IndentOpts)]),
    "mvpf_indent": (C.c_int, [_P, C.POINTER(IndentOpts), C.c_void_p, _P, C.POINTER(IndentRecord), C.c_int,
                             C.POINTER(C.c_int)]),
    "mvpf_set_tuning": (C.c_int, [_P, C.c_char_p, C.c_int, C.c_int]),
    "mvpf_get_tuning": (C.c_int, [_P, C.c_char_p, C.c_int, C.POINTER(C.c_int)]),
    "mvpf_autotune": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "mvpf_kernel_timing": (C.c_int, [_P, C.c_int]),
    "mvpf_kernel_stats": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int), _D, _D]),
    "mvpf_create_batch": (C.c_int, [C.c_int, C.POINTER(Mesh), C.POINTER(Material), C.POINTER(Loading),
                                    C.POINTER(Opts), _P, C.POINTER(_P)]),
    "mvpf_destroy_batch": (None, [_P]),
    "mvpf_batch_last_error": (C.c_char_p, [_P]),
    "mvpf_batch_problem": (_P, [_P, C.c_int]),
    "mvpf_batch_newton_system": (C.c_int, [_P, _D]),
    "mvpf_batch_solve": (C.c_int, [_P, C.POINTER(SolveStats)]),
    "mvpf_batch_newton_update": (C.c_int, [_P]),
}

_libs = {}


def load(nvar: int = 6) -> C.CDLL:
    """Load the library for nvar variants (raises if it has not been built)."""
    if nvar in _libs:
        return _libs[nvar]
    path = lib_path(nvar)
    if not os.path.exists(path):
        raise MvpfError(-3, f"{path} not found: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.mvpf_nvar() != nvar:
        raise MvpfError(-1, f"{path} is built for {lib.mvpf_nvar()} variants, not {nvar}")
    _libs[nvar] = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


MIXING = {"linear": MIX_LINEAR, "log": MIX_LOG}


def orbit_struct(om) -> OrbitMaterial:
    m = OrbitMaterial()
    m.U1[:] = list(om.U1)
    m.L1[:] = list(om.L1)
    m.cubic[:] = list(om.cubic)
    m.Q[:] = list(om.Q)
    m.F0_a, m.F0_m, m.w_am, m.w_mm = om.F0_a, om.F0_m, om.w_am, om.w_mm
    m.ell, m.rho, m.eps_eta, m.pade, m.mixing = om.ell, om.rho, om.eps_eta, om.pade, MIXING[om.mixing]
    return m


def material_struct(mp) -> Material:
    m = Material()
    m.cubic[:] = list(mp.cubic)
    m.ortho[:] = list(mp.ortho)
    m.alpha, m.beta, m.gamma = mp.alpha, mp.beta, mp.gamma
    m.Q[:] = list(mp.Q)
    m.F0[:] = list(mp.F0)
    m.w_am, m.w_mm, m.ell, m.rho, m.eps_eta, m.pade = mp.w_am, mp.w_mm, mp.ell, mp.rho, mp.eps_eta, mp.pade
    m.mixing = MIXING[getattr(mp, "mixing", "linear")]
    return m


def default_opts() -> Opts:
    o = Opts()
    load().mvpf_default_opts(C.byref(o))
    return o


def mesh_struct(prob) -> Mesh:
    return Mesh(prob.nx, prob.ny, prob.nz, prob.lx / prob.nx, prob.n_levels)


def loading_struct(prob) -> Loading:
    return Loading(_LOAD_KINDS[prob.kind], prob.patch, prob.radius, getattr(prob, "eps_n", 0.0))


def indent_opts(**kw) -> IndentOpts:
    o = IndentOpts()
    load().mvpf_default_indent_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def opts_struct(precision: str, **opts) -> Opts:
    """Default options with precision ('fp64' or 'mixed') and overrides;
    coarse may be given by name ('rediscretise' or 'galerkin')."""
    o = default_opts()
    o.precision = MIXED if precision == "mixed" else FP64
    for k, v in opts.items():
        if k == "coarse" and isinstance(v, str):
            v = COARSE[v]
        setattr(o, k, v)
    return o


class Problem:
    """One indentation problem on the GPU (handle of mvpf_create)."""

    def __init__(self, prob, precision: str = "fp64", device: int = 0, _handle=None, _opts=None, **opts):
        self.nvar = getattr(prob, "n_var", 6)
        lib = load(self.nvar)
        self.lib = lib
        self.prob = prob
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.n_nodes = prob.n_nodes
        self.ndof = 3 + self.nvar
        self.owned = _handle is None
        if _handle is not None:  # a problem owned by a Batch
            self.h = _handle
            self.opts = _opts
            return
        o = opts_struct(precision, **opts)
        self.opts = o
        h = C.c_void_p()
        if hasattr(prob.material, "U1"):  # card generated from one stretch tensor
            self.mat = orbit_struct(prob.material)
            rc = lib.mvpf_create_orbit(C.byref(mesh_struct(prob)), C.byref(self.mat), C.byref(loading_struct(prob)),
                                       C.byref(o), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            self.mat = material_struct(prob.material)
            rc = lib.mvpf_create(C.byref(mesh_struct(prob)), C.byref(self.mat), C.byref(loading_struct(prob)),
                                 C.byref(o), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise MvpfError(rc, lib.mvpf_last_error(None).decode())
        self.h = h

    def _check(self, rc, allow=(OK,)):
        if rc not in allow:
            raise MvpfError(rc, self.lib.mvpf_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            if self.owned:
                self.lib.mvpf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, n_nodes=None, comps=None):
        comps = self.ndof if comps is None else comps
        return torch.zeros((n_nodes or self.n_nodes) * comps, dtype=torch.float64, device=self.device)

    def info(self) -> Info:
        i = Info()
        self._check(self.lib.mvpf_get_info(self.h, C.byref(i)))
        return i

    def set_opts(self, **kw):
        for k, v in kw.items():
            if k == "coarse" and isinstance(v, str):
                v = COARSE[v]
            setattr(self.opts, k, v)
        self._check(self.lib.mvpf_set_opts(self.h, C.byref(self.opts)))

    def set_state(self, u=None, eta=None, eta_prev=None, depth=0.0):
        def dev(a):
            if a is None:
                return None
            return torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        u, eta, eta_prev = dev(u), dev(eta), dev(eta_prev)
        self._check(self.lib.mvpf_set_state(self.h, _ptr(u), _ptr(eta), _ptr(eta_prev), depth))

    def get_state(self):
        n = self.nvar
        u, e, en = self._vec(comps=3), self._vec(comps=n), self._vec(comps=n)
        d = C.c_double()
        self._check(self.lib.mvpf_get_state(self.h, _ptr(u), _ptr(e), _ptr(en), C.byref(d)))
        return u.view(-1, 3), e.view(-1, n), en.view(-1, n), d.value

    def init_random(self, seed: int):
        self._check(self.lib.mvpf_init_random(self.h, C.c_uint64(seed)))

    def residual(self):
        R = self._vec()
        nf = C.c_double()
        self._check(self.lib.mvpf_residual(self.h, _ptr(R), C.byref(nf)))
        return R, nf.value

    def residual_noalloc(self, R: Optional[torch.Tensor] = None):
        """mvpf_residual_noalloc: the residual with the library's fixed device
        scratch (no allocation by the library); R: optional caller-owned
        output (a new tensor if None)."""
        R = self._vec() if R is None else R
        nf = C.c_double()
        self._check(self.lib.mvpf_residual_noalloc(self.h, _ptr(R), C.byref(nf)))
        return R, nf.value

    def newton_system(self, depth: float):
        self._check(self.lib.mvpf_newton_system(self.h, depth))

    def get_rhs(self):
        b = self._vec()
        self._check(self.lib.mvpf_get_rhs(self.h, _ptr(b)))
        return b

    def jacobian_apply(self, level: int, x: torch.Tensor, precision: int = FP64):
        y = torch.zeros_like(x)
        self._check(self.lib.mvpf_jacobian_apply(self.h, level, precision, _ptr(x), _ptr(y)))
        return y

    def precondition(self, v: torch.Tensor):
        z = torch.zeros_like(v)
        self._check(self.lib.mvpf_precondition(self.h, _ptr(v), _ptr(z)))
        return z

    def solve(self, b: Optional[torch.Tensor] = None, want_x: bool = True):
        x = self._vec() if want_x else None
        st = SolveStats()
        self._check(self.lib.mvpf_solve(self.h, _ptr(b), _ptr(x), C.byref(st)), allow=(OK, ENOTCONV))
        return x, st

    def newton_update(self):
        self._check(self.lib.mvpf_newton_update(self.h))

    def newton_step(self, depth: float):
        """mvpf_newton_step: system at `depth`, solve, update; the solve's stats."""
        st = SolveStats()
        self._check(self.lib.mvpf_newton_step(self.h, depth, C.byref(st)), allow=(OK, ENOTCONV))
        return st

    def time_step(self, depth: float):
        st = StepStats()
        self._check(self.lib.mvpf_time_step(self.h, depth, C.byref(st)), allow=(OK, ENOTCONV))
        return st

    def set_viscosity(self, rho: float):
        self._check(self.lib.mvpf_set_viscosity(self.h, rho))

    def contact_load(self) -> float:
        P = C.c_double()
        self._check(self.lib.mvpf_contact_load(self.h, C.byref(P)))
        return P.value

    def indent(self, on_step=None, **kw):
        """mvpf_indent with mvpf_default_indent_opts overridden by ``kw``;
        on_step(record, index) is called after every accepted step.  Returns
        (records of the accepted steps, return code)."""
        o = indent_opts(**kw)
        recs = (IndentRecord * o.max_steps)()
        n = C.c_int()
        cb = IndentCallback(lambda r, i, u: on_step(r.contents, i)) if on_step else None
        rc = self._check(self.lib.mvpf_indent(self.h, C.byref(o), C.cast(cb, C.c_void_p) if cb else None, None, recs,
                                              o.max_steps, C.byref(n)), allow=(OK, ENOTCONV))
        return list(recs[: n.value]), rc

    def set_tuning(self, key: str, level: int, value: int):
        self._check(self.lib.mvpf_set_tuning(self.h, key.encode(), level, value))

    def get_tuning(self, key: str, level: int = 0) -> int:
        v = C.c_int()
        self._check(self.lib.mvpf_get_tuning(self.h, key.encode(), level, C.byref(v)))
        return v.value

    def autotune(self):
        out = (C.c_int * 8)()
        self._check(self.lib.mvpf_autotune(self.h, out))
        return list(out[: self.prob.n_levels])

    def kernel_timing(self, enable: bool):
        self._check(self.lib.mvpf_kernel_timing(self.h, int(enable)))

    def kernel_stats(self, name: str):
        n, ms, by = C.c_int(), C.c_double(), C.c_double()
        self._check(self.lib.mvpf_kernel_stats(self.h, name.encode(), C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value


class Batch:
    """Independent problems solved in lockstep (mvpf_create_batch); problem(i)
    returns a Problem view of problem i (owned by the batch)."""

    def __init__(self, probs, precision: str = "mixed", device: int = 0, **opts):
        lib = load()
        self.lib = lib
        self.probs = list(probs)
        n = len(self.probs)
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.opts = opts_struct(precision, **opts)
        meshes = (Mesh * n)(*[mesh_struct(p) for p in self.probs])
        mats = (Material * n)(*[material_struct(p.material) for p in self.probs])
        loads = (Loading * n)(*[loading_struct(p) for p in self.probs])
        h = C.c_void_p()
        rc = lib.mvpf_create_batch(n, meshes, mats, loads, C.byref(self.opts), C.c_void_p(self.stream.cuda_stream),
                                   C.byref(h))
        if rc != 0:
            raise MvpfError(rc, lib.mvpf_batch_last_error(None).decode())
        self.h = h
        self.views = [Problem(p, device=device, _handle=C.c_void_p(lib.mvpf_batch_problem(h, i)), _opts=self.opts)
                      for i, p in enumerate(self.probs)]

    def __len__(self):
        return len(self.probs)

    def problem(self, i: int) -> Problem:
        return self.views[i]

    def _check(self, rc, allow=(OK,)):
        if rc not in allow:
            raise MvpfError(rc, self.lib.mvpf_batch_last_error(self.h).decode())
        return rc

    def newton_system(self, depths):
        d = (C.c_double * len(self.probs))(*[float(x) for x in depths])
        self._check(self.lib.mvpf_batch_newton_system(self.h, d))

    def solve(self):
        st = (SolveStats * len(self.probs))()
        self._check(self.lib.mvpf_batch_solve(self.h, st), allow=(OK, ENOTCONV))
        return list(st)

    def newton_update(self):
        self._check(self.lib.mvpf_batch_newton_update(self.h))

    def close(self):
        if getattr(self, "h", None):
            for v in self.views:
                v.h = None
            self.lib.mvpf_destroy_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stats_dict(st) -> dict:
    return {f: getattr(st, f) for f, _ in st._fields_}
