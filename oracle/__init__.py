"""FP64 CPU oracle for the implicit viscous solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never does, and this package imports nothing from the
product: the two sides share only the seeded inputs they are handed.

``mas_oracle.c`` holds the arithmetic (geometry, assembly, operator apply,
Jacobi-preconditioned CG, adjoint gradient, RKL2 super time-step, block-Jacobi
ILU(0) preconditioner and its PCG); this module is ctypes
marshalling plus numpy array allocation.  ``dense`` holds small dense-matrix
helpers for tiny grids.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, a manufactured solution, dense LU,
brute-force finite differences, the Legendre closed form of the RKL2
stability polynomial and the matrix exponential; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mas_oracle.c")
_LIB = os.path.join(_HERE, "libmas_oracle.so")
# the same source built -O3 -march=native on the machine that times it (the
# CPU-baseline leg of the benchmark; tests use the portable -O2 build)
_LIB_NATIVE = os.path.join(_HERE, "libmas_oracle_native.so")
NATIVE_FLAGS = ["-O3", "-march=native"]

DIRICHLET = 0
NEUMANN = 1


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc into oracle/libmas_oracle.so (native:
    oracle/libmas_oracle_native.so, -O3 -march=native)."""
    lib = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + f".tmp{os.getpid()}"
        opt = NATIVE_FLAGS if native else ["-O2"]
        cmd = ["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


_lib = None
_lib_path = _LIB


def use_native_build() -> str:
    """Build and load the -O3 -march=native oracle (for timing only); must be
    called before anything else in this process uses the oracle."""
    global _lib_path
    if _lib is not None and _lib_path != _LIB_NATIVE:
        raise RuntimeError("the oracle library is already loaded")
    _lib_path = build(force=True, native=True)
    return _lib_path


def _gomp():
    return ctypes.CDLL("libgomp.so.1")


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops."""
    _load()
    _gomp().omp_set_num_threads(int(n))


def max_threads() -> int:
    _load()
    return int(_gomp().omp_get_max_threads())


def _dp():
    return ctypes.POINTER(ctypes.c_double)


class _Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nt", ctypes.c_int32), ("np", ctypes.c_int32),
                ("r_faces", ctypes.POINTER(ctypes.c_double)),
                ("t_faces", ctypes.POINTER(ctypes.c_double)),
                ("bc_inner", ctypes.c_int32), ("bc_outer", ctypes.c_int32)]


class _Op(ctypes.Structure):
    _fields_ = [("g", _Grid), ("dt", ctypes.c_double)] + [
        (name, ctypes.POINTER(ctypes.c_double))
        for name in ("V", "Ar", "Hr", "At", "Ht", "Ap", "Hp", "cr", "ct", "cp", "diag")]


def rkl2_coefficients(s: int):
    """(mu, nu, mt, gt) arrays of length s+1 for the s-stage RKL2 recursion."""
    lib = _load()
    out = [np.zeros(s + 1) for _ in range(4)]
    lib.ora_rkl2_coefficients(int(s), *[_ptr(a) for a in out])
    return tuple(out)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build(force=False, native=_lib_path == _LIB_NATIVE)
        lib = ctypes.CDLL(_lib_path)
        P = ctypes.POINTER
        lib.ora_geometry.argtypes = [P(_Op)]
        lib.ora_geometry.restype = ctypes.c_int
        lib.ora_assemble.argtypes = [P(_Op), _dp()]
        lib.ora_assemble.restype = ctypes.c_int
        lib.ora_apply.argtypes = [P(_Op), _dp(), _dp()]
        lib.ora_apply.restype = None
        lib.ora_rhs.argtypes = [P(_Op), _dp(), _dp()]
        lib.ora_rhs.restype = None
        lib.ora_dot.argtypes = [P(_Grid), _dp(), _dp()]
        lib.ora_dot.restype = ctypes.c_double
        lib.ora_pcg.argtypes = [P(_Op), _dp(), _dp(), ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, _dp(), _dp()]
        lib.ora_pcg.restype = ctypes.c_int
        lib.ora_gradient.argtypes = [P(_Op), _dp(), _dp(), _dp(), _dp()]
        lib.ora_gradient.restype = None
        lib.ora_rkl2_coefficients.argtypes = [ctypes.c_int, _dp(), _dp(), _dp(), _dp()]
        lib.ora_rkl2_coefficients.restype = None
        lib.ora_rkl2_stages.argtypes = [P(_Op)]
        lib.ora_rkl2_stages.restype = ctypes.c_int
        lib.ora_rkl2_step.argtypes = [P(_Op), _dp(), _dp(), ctypes.c_int]
        lib.ora_rkl2_step.restype = ctypes.c_int
        ci = ctypes.c_int
        lib.ora_pc2_factor.argtypes = [P(_Op), ci, ci, ci, _dp()]
        lib.ora_pc2_factor.restype = None
        lib.ora_pc2_apply.argtypes = [P(_Op), ci, ci, ci, _dp(), _dp(), _dp()]
        lib.ora_pc2_apply.restype = None
        lib.ora_pcg_pc2.argtypes = [P(_Op), ci, ci, ci, _dp(), _dp(), ctypes.c_double, ci, ci,
                                    _dp(), _dp()]
        lib.ora_pcg_pc2.restype = ci
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Operator:
    """Oracle geometry + assembled operator for one grid, nu and dt.

    Arrays (numpy, float64):
      V  (nr, nt, np)          cell volumes
      Ar, Hr, cr (nr+1, nt, np)  r-face area, distance, conductance
      At, Ht, ct (nr, nt+1, np)  theta-face area, distance, conductance
      Ap, Hp, cp (nr, nt, np)    phi-face (k+1/2) area, distance, conductance
      diag (nr, nt, np)        diagonal of A
    """

    def __init__(self, r_faces, t_faces, np_, nu, dt, bc_inner=DIRICHLET, bc_outer=DIRICHLET):
        lib = _load()
        self.r_faces = _f64(r_faces)
        self.t_faces = _f64(t_faces)
        self.nr = self.r_faces.size - 1
        self.nt = self.t_faces.size - 1
        self.np = int(np_)
        self.shape = (self.nr, self.nt, self.np)
        self.dt = float(dt)
        nr, nt, n_p = self.shape
        self.V = np.zeros(self.shape)
        self.Ar = np.zeros((nr + 1, nt, n_p))
        self.Hr = np.zeros((nr + 1, nt, n_p))
        self.At = np.zeros((nr, nt + 1, n_p))
        self.Ht = np.zeros((nr, nt + 1, n_p))
        self.Ap = np.zeros(self.shape)
        self.Hp = np.zeros(self.shape)
        self.cr = np.zeros((nr + 1, nt, n_p))
        self.ct = np.zeros((nr, nt + 1, n_p))
        self.cp = np.zeros(self.shape)
        self.diag = np.zeros(self.shape)
        self._grid = _Grid(nr, nt, n_p, _ptr(self.r_faces), _ptr(self.t_faces),
                           int(bc_inner), int(bc_outer))
        self._op = _Op(self._grid, self.dt, *[_ptr(getattr(self, n)) for n in
                       ("V", "Ar", "Hr", "At", "Ht", "Ap", "Hp", "cr", "ct", "cp", "diag")])
        if lib.ora_geometry(ctypes.byref(self._op)) != 0:
            raise ValueError("bad grid")
        self.set_nu(nu)

    def set_nu(self, nu):
        self.nu = _f64(nu).reshape(self.shape)
        _load().ora_assemble(ctypes.byref(self._op), _ptr(self.nu))

    def apply(self, x) -> np.ndarray:
        x = _f64(x).reshape(self.shape)
        y = np.empty(self.shape)
        _load().ora_apply(ctypes.byref(self._op), _ptr(x), _ptr(y))
        return y

    def rhs_to_b(self, rhs) -> np.ndarray:
        rhs = _f64(rhs).reshape(self.shape)
        b = np.empty(self.shape)
        _load().ora_rhs(ctypes.byref(self._op), _ptr(rhs), _ptr(b))
        return b

    def dot(self, a, b) -> float:
        return float(_load().ora_dot(ctypes.byref(self._grid), _ptr(_f64(a).reshape(self.shape)),
                                     _ptr(_f64(b).reshape(self.shape))))

    def pcg(self, b, tol=1e-10, max_iters=100000, x0=None, history=False):
        """Jacobi-PCG on A x = b.  Returns (x, iterations, rel_res_recursive,
        rel_res_true[, history])."""
        b = _f64(b).reshape(self.shape)
        x = np.zeros(self.shape) if x0 is None else _f64(x0).reshape(self.shape).copy()
        stats = np.zeros(2)
        hist = np.zeros(max_iters + 1) if history else None
        it = _load().ora_pcg(ctypes.byref(self._op), _ptr(b), _ptr(x), float(tol),
                             int(max_iters), int(x0 is not None), _ptr(stats),
                             _ptr(hist) if history else None)
        if it < 0:
            raise FloatingPointError("PCG breakdown: (p, Ap) <= 0")
        if history:
            return x, it, stats[0], stats[1], hist[: it + 1]
        return x, it, stats[0], stats[1]

    def solve_rhs(self, rhs, tol=1e-12, max_iters=100000):
        """x = A^-1 (V .* rhs) by PCG to a tight tolerance."""
        return self.pcg(self.rhs_to_b(rhs), tol=tol, max_iters=max_iters)[0]

    def gradient(self, x, lam):
        """(dL/dnu, dL/drhs) given the solution x and the adjoint lam = A^-1 dL/dx."""
        x = _f64(x).reshape(self.shape)
        lam = _f64(lam).reshape(self.shape)
        gnu = np.empty(self.shape)
        grhs = np.empty(self.shape)
        _load().ora_gradient(ctypes.byref(self._op), _ptr(x), _ptr(lam), _ptr(gnu), _ptr(grhs))
        return gnu, grhs

    def rkl2_stages(self) -> int:
        """Stages the stability bound requires for one step of dt."""
        return int(_load().ora_rkl2_stages(ctypes.byref(self._op)))

    def rkl2_step(self, u0, stages=None) -> np.ndarray:
        """One RKL2 super time-step of du/dt = L u over dt."""
        s = self.rkl2_stages() if stages is None else int(stages)
        u0 = _f64(u0).reshape(self.shape)
        u1 = np.empty(self.shape)
        if _load().ora_rkl2_step(ctypes.byref(self._op), _ptr(u0), _ptr(u1), s) != 0:
            raise ValueError("need at least 2 stages")
        return u1

    def pc2_factor(self, blocks=(8, 8, 64)) -> np.ndarray:
        """Modified diagonal of the block-Jacobi ILU(0) factorization."""
        d = np.empty(self.shape)
        _load().ora_pc2_factor(ctypes.byref(self._op), *map(int, blocks), _ptr(d))
        return d

    def pc2_apply(self, r, blocks=(8, 8, 64), d=None) -> np.ndarray:
        """z = M^-1 r for the block-Jacobi ILU(0) preconditioner M."""
        d = self.pc2_factor(blocks) if d is None else _f64(d).reshape(self.shape)
        r = _f64(r).reshape(self.shape)
        z = np.empty(self.shape)
        _load().ora_pc2_apply(ctypes.byref(self._op), *map(int, blocks), _ptr(d), _ptr(r), _ptr(z))
        return z

    def pcg_pc2(self, b, blocks=(8, 8, 64), tol=1e-10, max_iters=100000, x0=None, history=False):
        """PCG with the block-Jacobi ILU(0) preconditioner.  Returns (x, iterations,
        rel_res_recursive, rel_res_true[, history])."""
        b = _f64(b).reshape(self.shape)
        x = np.zeros(self.shape) if x0 is None else _f64(x0).reshape(self.shape).copy()
        stats = np.zeros(2)
        hist = np.zeros(max_iters + 1) if history else None
        it = _load().ora_pcg_pc2(ctypes.byref(self._op), *map(int, blocks), _ptr(b), _ptr(x),
                                 float(tol), int(max_iters), int(x0 is not None), _ptr(stats),
                                 _ptr(hist) if history else None)
        if it < 0:
            raise FloatingPointError("PCG breakdown: (p, Ap) <= 0")
        if history:
            return x, it, stats[0], stats[1], hist[: it + 1]
        return x, it, stats[0], stats[1]

    def rel_residual(self, b, x) -> float:
        b = _f64(b).reshape(self.shape)
        r = b - self.apply(x)
        return float(np.sqrt(self.dot(r, r)) / np.sqrt(self.dot(b, b)))
