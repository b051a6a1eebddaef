"""Plain FP64 CPU oracle of the UV-decomposition ADMM (Section IV, Algorithm 1).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the solver library and its binding never
do.  The arithmetic lives in ``uvadmm_oracle.c`` (plain C, OpenMP); this module
only builds it with gcc and marshals numpy arrays through ctypes.

The oracle keeps Algorithm 1's own o-space variables (y and gamma, one entry
per stored nonzero) and applies U, U', V, V' as explicit sums over the nonzero
index, so it shares neither code nor algebra with the GPU solver's reduced
form.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uvadmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a different build of the same source (the mutation tests point this at a
# copy with a planted mistake)
_LIB = os.environ.get("UVADMM_ORACLE_LIB", _LIB)

_lib = None


def build(verbose: bool = False, src: str = _SRC, out: str | None = None) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, -O2, OpenMP)."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wextra", "-o", out + ".tmp", src, "-lm"]
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
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [i32, i32, i64, P, P, P, P, P, i32, i32, P, f64]
    lib.orc_destroy.argtypes = [P]
    lib.orc_destroy.restype = None
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_diagonals.argtypes = [P, P, P]
    lib.orc_diagonals.restype = None
    lib.orc_project.argtypes = [i32, i32, P, P, P]
    lib.orc_project.restype = None
    lib.orc_set_state.argtypes = [P, P, P, P, P, P, P]
    lib.orc_set_state.restype = None
    lib.orc_set_start.argtypes = [P, P, P, P, P]
    lib.orc_set_start.restype = None
    lib.orc_resume.argtypes = [P, P, P, P, P]
    lib.orc_resume.restype = None
    lib.orc_get_state.argtypes = [P, P, P, P, P, P, P]
    lib.orc_get_state.restype = None
    lib.orc_iteration.argtypes = [P]
    lib.orc_iteration.restype = i64
    lib.orc_iterate.argtypes = [P, i64]
    lib.orc_iterate.restype = None
    lib.orc_residuals.argtypes = [P, P]
    lib.orc_residuals.restype = None
    lib.orc_solve.argtypes = [P, f64, i64, i64, P]
    lib.orc_solve.restype = i64
    lib.orc_uv_dense.argtypes = [i32, i32, i64, P, P, P, P, P]
    lib.orc_uv_dense.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


RESIDUAL_KEYS = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj",
                 "res_ax_b", "res_x_z", "prim_inf", "dual_inf", "scale_p", "scale_d", "pobj_x")


def project(w, n_orth: int, soc_sizes=()) -> np.ndarray:
    """proj_K(w) for K = R_+^{n_orth} x K_{soc_sizes[0]} x ... (eq. proj)."""
    lib = _load()
    w = _f64(w)
    sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
    out = np.empty_like(w)
    lib.orc_project(int(n_orth), int(sizes.size), _ptr(sizes), _ptr(w), _ptr(out))
    return out


def uv_dense(m: int, n: int, rows, cols, vals):
    """Dense (U, V) of eqs. UU/VV for nonzeros listed in the given order."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = _f64(vals)
    o = rows.size
    U = np.empty((m, o))
    V = np.empty((n, o))
    lib.orc_uv_dense(int(m), int(n), int(o), _ptr(rows), _ptr(cols), _ptr(vals),
                     _ptr(U), _ptr(V))
    return U, V


class Oracle:
    """Algorithm 1 on one problem (A in CSR, b, c, K, mu)."""

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, n_orth, soc_sizes=(),
                 mu: float = 1.0):
        lib = _load()
        self._lib = lib
        self.m, self.n = int(m), int(n)
        self._row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self._val = _f64(val)
        self._b = _f64(b)
        self._c = _f64(c)
        self._sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
        self.nnz = int(self._row_ptr[-1])
        self.mu = float(mu)
        h = lib.orc_create(self.m, self.n, self.nnz, _ptr(self._row_ptr),
                           _ptr(self._col_idx), _ptr(self._val), _ptr(self._b),
                           _ptr(self._c), int(n_orth), int(self._sizes.size),
                           _ptr(self._sizes), self.mu)
        if not h:
            raise ValueError("oracle rejected the problem (malformed CSR, cone "
                             "sizes not summing to n, or mu <= 0)")
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_instance(cls, inst, mu: float = 1.0):
        return cls(inst["m"], inst["n"], inst["row_ptr"], inst["col_idx"],
                   inst["val"], inst["b"], inst["c"], inst["n_orth"],
                   inst["soc_sizes"], mu=mu)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def diagonals(self):
        FU = np.empty(self.m)
        FV = np.empty(self.n)
        self._lib.orc_diagonals(self._h, _ptr(FU), _ptr(FV))
        return FU, FV

    def set_state(self, x=None, z=None, delta=None, y=None, gamma=None, lam=None):
        args = [_f64(v) for v in (x, z, delta, y, gamma, lam)]
        self._lib.orc_set_state(self._h, *[_ptr(a) for a in args])

    def set_start(self, x=None, z=None, delta=None, lam=None):
        args = [_f64(v) for v in (x, z, delta, lam)]
        self._lib.orc_set_start(self._h, *[_ptr(a) for a in args])

    def resume(self, x=None, z=None, delta=None, lam=None):
        """State at the end of an iteration from (x, z, delta, lambda)."""
        args = [_f64(v) for v in (x, z, delta, lam)]
        self._lib.orc_resume(self._h, *[_ptr(a) for a in args])

    def state(self):
        x, z, d = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        y, g = np.empty(self.nnz), np.empty(self.nnz)
        lam = np.empty(self.m)
        self._lib.orc_get_state(self._h, _ptr(x), _ptr(z), _ptr(d), _ptr(y),
                                _ptr(g), _ptr(lam))
        return {"x": x, "z": z, "delta": d, "y": y, "gamma": g, "lambda": lam}

    @property
    def iteration(self) -> int:
        return int(self._lib.orc_iteration(self._h))

    def iterate(self, k: int):
        self._lib.orc_iterate(self._h, int(k))

    def residuals(self) -> dict:
        out = np.empty(len(RESIDUAL_KEYS))
        self._lib.orc_residuals(self._h, _ptr(out))
        return dict(zip(RESIDUAL_KEYS, out.tolist()))

    def solve(self, eps: float, check_every: int = 10, max_iter: int = 100000):
        out = np.empty(len(RESIDUAL_KEYS))
        it = self._lib.orc_solve(self._h, float(eps), int(check_every),
                                 int(max_iter), _ptr(out))
        r = dict(zip(RESIDUAL_KEYS, out.tolist()))
        r["iter"] = int(it)
        return r
