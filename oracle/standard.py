"""Plain FP64 CPU oracle of standard two-block ADMM with a warm-started CG
solve of the block system eq. lin (Sections II-B and III-B), for the
orthant and products of Lorentz cones.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests and the
benchmark's CPU leg use it; the solver library never does.  The arithmetic is
in ``standard_oracle.c`` (plain C); this module builds it with gcc and
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "standard_oracle.c")
_LIB = os.environ.get("UVADMM_STD_ORACLE_LIB", os.path.join(_HERE, "libstdoracle.so"))

_lib = None

RESIDUAL_KEYS = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_x1_x2", "cg_steps")


def build(verbose: bool = False, src: str = _SRC, out: str | None = None) -> str:
    """Compile ``standard_oracle.c`` into ``oracle/libstdoracle.so`` (gcc -O2)."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ors_create.restype = P
    lib.ors_create.argtypes = [i32, i32, i64, P, P, P, P, P, i32, i32, P, f64, i32, f64]
    lib.ors_destroy.argtypes = [P]
    lib.ors_destroy.restype = None
    lib.ors_set_state.argtypes = [P, P, P, P]
    lib.ors_set_state.restype = None
    lib.ors_get_state.argtypes = [P, P, P, P, P, P]
    lib.ors_get_state.restype = None
    lib.ors_iteration.argtypes = [P]
    lib.ors_iteration.restype = i64
    lib.ors_cg_steps.argtypes = [P]
    lib.ors_cg_steps.restype = i64
    lib.ors_iterate.argtypes = [P, i64]
    lib.ors_iterate.restype = None
    lib.ors_residuals.argtypes = [P, P]
    lib.ors_residuals.restype = None
    lib.ors_project.argtypes = [i32, i32, P, P, P]
    lib.ors_project.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def project(w, n_orth: int, soc_sizes=()) -> np.ndarray:
    """proj_K(w) with this oracle's own projection (eq. proj per cone)."""
    lib = _load()
    w = _f64(w)
    sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
    out = np.empty_like(w)
    lib.ors_project(int(n_orth), int(sizes.size), _ptr(sizes) if sizes.size else None, _ptr(w), _ptr(out))
    return out


class StandardADMM:
    """Standard ADMM + CG on one problem (A in CSR, b, c; K = n_orth orthant
    coordinates, then Lorentz cones of soc_sizes; default: all orthant)."""

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, mu=1.0, cg_iters=10, cg_tol=0.0,
                 n_orth=None, soc_sizes=()):
        lib = _load()
        self._lib = lib
        self.m, self.n = int(m), int(n)
        self._row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self._val = _f64(val)
        self._b = _f64(b)
        self._c = _f64(c)
        self._sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
        n_orth = self.n if n_orth is None else int(n_orth)
        h = lib.ors_create(self.m, self.n, int(self._row_ptr[-1]), _ptr(self._row_ptr),
                           _ptr(self._col_idx), _ptr(self._val), _ptr(self._b), _ptr(self._c),
                           n_orth, int(self._sizes.size), _ptr(self._sizes) if self._sizes.size else None,
                           float(mu), int(cg_iters), float(cg_tol))
        if not h:
            raise ValueError("standard-ADMM oracle rejected the problem")
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst["m"], inst["n"], inst["row_ptr"], inst["col_idx"], inst["val"],
                   inst["b"], inst["c"], n_orth=inst["n_orth"], soc_sizes=inst["soc_sizes"], **kw)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ors_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_state(self, x2=None, lam=None, nu=None):
        args = [_f64(v) for v in (x2, lam, nu)]
        self._lib.ors_set_state(self._h, *[_ptr(a) for a in args])

    def state(self):
        x1, x2, lam, d = (np.empty(self.n) for _ in range(4))
        nu = np.empty(self.m)
        self._lib.ors_get_state(self._h, _ptr(x1), _ptr(x2), _ptr(lam), _ptr(nu), _ptr(d))
        return {"x1": x1, "x2": x2, "lam": lam, "nu": nu, "delta": d}

    @property
    def iteration(self) -> int:
        return int(self._lib.ors_iteration(self._h))

    @property
    def cg_steps(self) -> int:
        return int(self._lib.ors_cg_steps(self._h))

    def iterate(self, k: int):
        self._lib.ors_iterate(self._h, int(k))

    def residuals(self) -> dict:
        out = np.empty(8)
        self._lib.ors_residuals(self._h, _ptr(out))
        return dict(zip(RESIDUAL_KEYS, out.tolist()))

    def solve(self, eps=1e-4, check_every=10, max_iter=100_000) -> dict:
        while self.iteration < max_iter:
            self.iterate(min(check_every, max_iter - self.iteration))
            r = self.residuals()
            if r["kkt"] <= eps:
                return r
        return self.residuals()
