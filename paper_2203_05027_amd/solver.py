"""ctypes binding of ``libuvadmm.so`` (the C ABI declared in include/uvadmm.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  The binding refuses to work without the built library; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuvadmm.so")

UV_OK, UV_EINVAL, UV_EBADCSR, UV_ECONE, UV_ENOMEM, UV_EHIP, UV_ENUMERIC, UV_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7
UV_ENOSCRATCH = -8
UV_FP64, UV_MIXED = 0, 1
UV_MAX_CONE = 1024
STATUS = {0: "running", 1: "converged", 2: "max_iter", 3: "numeric"}


class UvCsr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class UvCones(ctypes.Structure):
    _fields_ = [("n_orthant", ctypes.c_int32), ("n_soc", ctypes.c_int32),
                ("soc_sizes", ctypes.c_void_p)]


class UvOpts(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("eps_kkt", ctypes.c_double),
                ("max_iter", ctypes.c_int64), ("hip_stream", ctypes.c_void_p),
                ("lanes_row", ctypes.c_int32), ("lanes_col", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("unroll_row", ctypes.c_int32),
                ("unroll_col", ctypes.c_int32), ("slabs_row", ctypes.c_int32),
                ("slabs_col", ctypes.c_int32), ("criterion", ctypes.c_int32),
                ("eps_abs", ctypes.c_double), ("slab_kernel", ctypes.c_int32),
                ("eps_gap", ctypes.c_double), ("resident", ctypes.c_int32),
                ("history", ctypes.c_int32), ("full_checks", ctypes.c_int32)]


class UvResiduals(ctypes.Structure):
    _fields_ = [("r_prim", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("r_gap", ctypes.c_double), ("kkt", ctypes.c_double),
                ("pobj", ctypes.c_double), ("dobj", ctypes.c_double),
                ("res_ax_b", ctypes.c_double), ("prim_inf", ctypes.c_double),
                ("dual_inf", ctypes.c_double), ("scale_p", ctypes.c_double),
                ("scale_d", ctypes.c_double), ("iter", ctypes.c_int64),
                ("status", ctypes.c_int32), ("pobj_x", ctypes.c_double),
                ("gap_x", ctypes.c_double)]


class UvHistory(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("r_prim", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("r_gap", ctypes.c_double), ("kkt", ctypes.c_double),
                ("pobj", ctypes.c_double), ("dobj", ctypes.c_double),
                ("res_ax_b", ctypes.c_double), ("gap_x", ctypes.c_double)]


def _struct_dtype(cls):
    """numpy view of a ctypes Structure of doubles and integers."""
    fmt = {ctypes.c_double: "<f8", ctypes.c_int64: "<i8", ctypes.c_int32: "<i4"}
    names = [k for k, _ in cls._fields_]
    return np.dtype({"names": names, "formats": [fmt[t] for _, t in cls._fields_],
                     "offsets": [getattr(cls, k).offset for k in names], "itemsize": ctypes.sizeof(cls)})


_RES_DTYPE = _struct_dtype(UvResiduals)


class UvError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib().solver_strerror(code).decode()} (code {code})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # PyTorch ships its own HIP runtime under the same soname; loading torch
    # first makes this library bind to that one, so a process that also uses
    # torch for device memory holds a single HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.uv_default_opts.argtypes = [ctypes.POINTER(UvOpts)]
    L.uv_default_opts.restype = None
    L.solver_create.argtypes = [ctypes.POINTER(UvCsr), P, P, ctypes.POINTER(UvCones),
                                ctypes.POINTER(UvOpts), ctypes.POINTER(P)]
    L.solver_create.restype = ctypes.c_int
    L.solver_set_start.argtypes = [P, P, P, P, P]
    L.solver_set_start.restype = ctypes.c_int
    L.solver_resume.argtypes = [P, P, P, P, P]
    L.solver_resume.restype = ctypes.c_int
    L.solver_iterate.argtypes = [P, i64, ctypes.POINTER(i32)]
    L.solver_iterate.restype = ctypes.c_int
    L.solver_solve.argtypes = [ctypes.POINTER(UvCsr), P, P, ctypes.POINTER(UvCones), ctypes.POINTER(UvOpts),
                               i64, P, P, P, P, ctypes.POINTER(UvResiduals)]
    L.solver_solve.restype = ctypes.c_int
    L.solver_solve_noalloc.argtypes = L.solver_solve.argtypes
    L.solver_solve_noalloc.restype = ctypes.c_int
    L.solver_residuals.argtypes = [P, ctypes.POINTER(UvResiduals)]
    L.solver_residuals.restype = ctypes.c_int
    L.solver_solution.argtypes = [P, P, P, P, P]
    L.solver_solution.restype = ctypes.c_int
    L.solver_destroy.argtypes = [P]
    L.solver_destroy.restype = None
    L.solver_strerror.argtypes = [ctypes.c_int]
    L.solver_strerror.restype = ctypes.c_char_p
    L.solver_time_kernels.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    L.solver_time_kernels.restype = ctypes.c_int
    L.solver_launch_shape.argtypes = [P, ctypes.POINTER(i32)]
    L.solver_launch_shape.restype = ctypes.c_int
    L.solver_set_rhs.argtypes = [P, P]
    L.solver_set_rhs.restype = ctypes.c_int
    L.solver_history.argtypes = [P, i32, ctypes.POINTER(UvHistory), ctypes.POINTER(i32)]
    L.solver_history.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != UV_OK:
        raise UvError(rc, where)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, size=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if size is not None and a.size != size:
        raise ValueError(f"expected {size} entries, got {a.size}")
    return a


def _csr(m, row_ptr, col_idx, val):
    """Contiguous int64 / int32 / float64 copies of a CSR matrix with m rows,
    checked for lengths the library cannot see (it reads m + 1 row offsets
    and row_ptr[m] indices and values); the values themselves (order,
    ranges) are the library's to check.  Returns (rp, ci, va, nnz)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    if rp.ndim != 1 or rp.size != int(m) + 1:
        raise ValueError(f"row_ptr needs m + 1 = {int(m) + 1} entries, got {rp.size}")
    nnz = int(rp[-1])
    if nnz < 0 or ci.size < nnz or va.size < nnz:
        raise ValueError(f"row_ptr[m] = {nnz} entries, but col_idx has {ci.size} and val {va.size}")
    return rp, ci, va, nnz


def default_opts() -> UvOpts:
    o = UvOpts()
    lib().uv_default_opts(ctypes.byref(o))
    return o


def _problem(m, n, row_ptr, col_idx, val, b, c, n_orth, soc_sizes):
    """ctypes views of a problem (the arrays are returned too, to keep them
    alive while the library reads them)."""
    rp, ci, va, nnz = _csr(m, row_ptr, col_idx, val)
    sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
    csr = UvCsr(m, n, nnz, _ptr(rp), _ptr(ci), _ptr(va))
    cones = UvCones(int(n_orth), int(sizes.size), _ptr(sizes) if sizes.size else None)
    bb = _f64(b, m)
    cc = _f64(c, n)
    return (rp, ci, va, sizes), csr, cones, bb, cc


def _opts(*, mu=1.0, precision="fp64", check_every=10, eps=1e-4, max_iter=0, lanes_row=0, lanes_col=0,
          unroll_row=0, unroll_col=0, slabs_row=0, slabs_col=0, criterion="kkt", eps_abs=0.0, eps_gap=0.0,
          slab_kernel="auto", resident="auto", history=0, full_checks=False, use_graph=True, stream=None):
    o = default_opts()
    o.mu = float(mu)
    o.precision = {"fp64": UV_FP64, "mixed": UV_MIXED}[precision]
    o.check_every = int(check_every)
    o.eps_kkt = float(eps)
    o.max_iter = int(max_iter)
    o.hip_stream = stream
    o.lanes_row, o.lanes_col = int(lanes_row), int(lanes_col)
    o.unroll_row, o.unroll_col = int(unroll_row), int(unroll_col)
    o.slabs_row, o.slabs_col = int(slabs_row), int(slabs_col)
    o.criterion = {"kkt": 0, "inf": 1, "pogs": 2}[criterion]
    o.eps_gap = float(eps_gap)
    o.resident = {"auto": 0, "never": 1, "required": 2}[resident]
    o.slab_kernel = {"auto": 0, "chunked": 1, "lanes": 2, "chunked4": 3}[slab_kernel]
    o.eps_abs = float(eps_abs)
    o.history = int(history)
    o.full_checks = 1 if full_checks else 0
    o.use_graph = 1 if use_graph else 0
    return o


def solve(inst, iters, noalloc=False, **kw):
    """solver_solve (or, with noalloc, solver_solve_noalloc) on an instance
    dict: (return code, solution dict, residuals dict).  Options as for
    Solver."""
    m, n = int(inst["m"]), int(inst["n"])
    keep, csr, cones, bb, cc = _problem(m, n, inst["row_ptr"], inst["col_idx"], inst["val"], inst["b"],
                                        inst["c"], inst["n_orth"], inst["soc_sizes"])
    o = _opts(**kw)
    x, z, d, lam = np.empty(n), np.empty(n), np.empty(n), np.empty(m)
    r = UvResiduals()
    fn = lib().solver_solve_noalloc if noalloc else lib().solver_solve
    rc = fn(ctypes.byref(csr), _ptr(bb), _ptr(cc), ctypes.byref(cones), ctypes.byref(o),
            ctypes.c_int64(int(iters)), _ptr(x), _ptr(z), _ptr(lam), _ptr(d), ctypes.byref(r))
    res = {k: getattr(r, k) for k, _ in UvResiduals._fields_}
    res["status"] = STATUS.get(res["status"], res["status"])
    return rc, {"x": x, "z": z, "delta": d, "lambda": lam}, res


class Solver:
    """One problem on the GPU: ``min c'x s.t. A x = b, x in K``.

    ``A`` is given in CSR (``row_ptr`` int64, ``col_idx`` int32, ``val``
    float64); ``K`` is ``n_orth`` orthant coordinates followed by the
    second-order cones of ``soc_sizes``.
    """

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, n_orth, soc_sizes=(), *,
                 mu=1.0, precision="fp64", check_every=10, eps=1e-4, max_iter=0,
                 lanes_row=0, lanes_col=0, unroll_row=0, unroll_col=0, slabs_row=0, slabs_col=0,
                 criterion="kkt", eps_abs=0.0, eps_gap=0.0, slab_kernel="auto", resident="auto", history=0,
                 full_checks=False, use_graph=True, stream=None):
        L = lib()
        self.m, self.n = int(m), int(n)
        keep, csr, cones, bb, cc = _problem(self.m, self.n, row_ptr, col_idx, val, b, c, n_orth, soc_sizes)
        o = _opts(mu=mu, precision=precision, check_every=check_every, eps=eps, max_iter=max_iter,
                  lanes_row=lanes_row, lanes_col=lanes_col, unroll_row=unroll_row, unroll_col=unroll_col,
                  slabs_row=slabs_row, slabs_col=slabs_col, criterion=criterion, eps_abs=eps_abs,
                  eps_gap=eps_gap, slab_kernel=slab_kernel, resident=resident, history=history,
                  full_checks=full_checks, use_graph=use_graph, stream=stream)
        self.precision = precision
        self._history_cap = int(history)
        self.nnz = csr.nnz
        h = ctypes.c_void_p()
        _check(L.solver_create(ctypes.byref(csr), _ptr(bb), _ptr(cc), ctypes.byref(cones),
                               ctypes.byref(o), ctypes.byref(h)), "solver_create")
        self._h = h

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst["m"], inst["n"], inst["row_ptr"], inst["col_idx"], inst["val"],
                   inst["b"], inst["c"], inst["n_orth"], inst["soc_sizes"], **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_start(self, x=None, z=None, delta=None, lam=None):
        n, m = self.n, self.m
        args = (_f64(x, n), _f64(z, n), _f64(delta, n), _f64(lam, m))
        _check(lib().solver_set_start(self._h, *[_ptr(a) for a in args]), "solver_set_start")

    def set_rhs(self, b):
        """New right-hand side (same A, c, cones); call set_start or resume
        before iterating again."""
        _check(lib().solver_set_rhs(self._h, _ptr(_f64(b, self.m))), "solver_set_rhs")

    def resume(self, x=None, z=None, delta=None, lam=None):
        """Continue a run from a state returned by solution() (checkpoint)."""
        n, m = self.n, self.m
        args = (_f64(x, n), _f64(z, n), _f64(delta, n), _f64(lam, m))
        _check(lib().solver_resume(self._h, *[_ptr(a) for a in args]), "solver_resume")

    def iterate(self, k: int) -> bool:
        done = ctypes.c_int32(0)
        rc = lib().solver_iterate(self._h, int(k), ctypes.byref(done))
        if rc not in (UV_OK, UV_ENUMERIC):
            _check(rc, "solver_iterate")
        return bool(done.value)

    def residuals(self) -> dict:
        r = UvResiduals()
        _check(lib().solver_residuals(self._h, ctypes.byref(r)), "solver_residuals")
        d = {k: getattr(r, k) for k, _ in UvResiduals._fields_}
        d["status"] = STATUS.get(d["status"], d["status"])
        return d

    def solution(self) -> dict:
        x, z, d = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        lam = np.empty(self.m)
        _check(lib().solver_solution(self._h, _ptr(x), _ptr(z), _ptr(lam), _ptr(d)),
               "solver_solution")
        return {"x": x, "z": z, "delta": d, "lambda": lam}

    def time_kernels(self, iters: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().solver_time_kernels(self._h, int(iters), ctypes.byref(a), ctypes.byref(b)),
               "solver_time_kernels")
        return a.value, b.value

    def history(self, max_records: int | None = None) -> list:
        """The residual history (kept when created with history=N > 0): the
        latest checks of the iteration, oldest first, as dicts with iter,
        seconds (GPU time since the start) and the residuals."""
        cap = self._history_cap if max_records is None else int(max_records)
        if cap <= 0:
            return []
        buf = (UvHistory * cap)()
        cnt = ctypes.c_int32()
        _check(lib().solver_history(self._h, cap, buf, ctypes.byref(cnt)), "solver_history")
        return [{k: getattr(buf[i], k) for k, _ in UvHistory._fields_} for i in range(cnt.value)]

    def launch_shape(self) -> dict:
        """Lanes and gathers in flight per lane of the row and column passes."""
        a = (ctypes.c_int32 * 7)()
        _check(lib().solver_launch_shape(self._h, a), "solver_launch_shape")
        return {"lanes_row": a[0], "unroll_row": a[1], "lanes_col": a[2], "unroll_col": a[3],
                "slabs_row": a[4], "slabs_col": a[5], "resident": bool(a[6])}


def _bind_batch(L):
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.batch_create.argtypes = [i32, P, P, P, ctypes.POINTER(UvOpts), ctypes.POINTER(P)]
    L.batch_create.restype = ctypes.c_int
    L.batch_iterate.argtypes = [P, i64, ctypes.POINTER(i32)]
    L.batch_iterate.restype = ctypes.c_int
    L.batch_residuals.argtypes = [P, i32, ctypes.POINTER(UvResiduals)]
    L.batch_residuals.restype = ctypes.c_int
    L.batch_solution.argtypes = [P, i32, P, P, P, P]
    L.batch_solution.restype = ctypes.c_int
    L.batch_set_start.argtypes = [P, i32, P, P, P, P]
    L.batch_set_start.restype = ctypes.c_int
    L.batch_set_tiles.argtypes = [P, i32, P]
    L.batch_set_tiles.restype = ctypes.c_int
    L.batch_get_tiles.argtypes = [P, ctypes.POINTER(i32), P]
    L.batch_get_tiles.restype = ctypes.c_int
    L.batch_time.argtypes = [P, i32, i32, ctypes.POINTER(ctypes.c_double)]
    L.batch_time.restype = ctypes.c_int
    L.batch_info.argtypes = [P, P]
    L.batch_info.restype = ctypes.c_int
    L.batch_destroy.argtypes = [P]
    L.batch_destroy.restype = None


class Batch:
    """Many independent LPs (orthant cone) solved together on the GPU by one
    persistent launch.  ``instances`` is a list of dicts with m, n, row_ptr,
    col_idx, val, b, c."""

    BUCKETS = (0, 128, 512, 2048)  # lower bounds of the size buckets on m

    def __init__(self, instances, *, mu=1.0, precision="mixed", check_every=10, eps=1e-4,
                 max_iter=0, full_checks=False, use_graph=True, stream=None):
        L = lib()
        if not hasattr(L, "_batch_bound"):
            _bind_batch(L)
            L._batch_bound = True
        self.count = len(instances)
        self.ms = [int(i["m"]) for i in instances]
        self.ns = [int(i["n"]) for i in instances]
        keep = []
        csrs = (UvCsr * self.count)()
        bp = (ctypes.c_void_p * self.count)()
        cpp = (ctypes.c_void_p * self.count)()
        for k, inst in enumerate(instances):
            rp, ci, va, nnz = _csr(self.ms[k], inst["row_ptr"], inst["col_idx"], inst["val"])
            bb = _f64(inst["b"], self.ms[k])
            cc = _f64(inst["c"], self.ns[k])
            keep += [rp, ci, va, bb, cc]
            csrs[k] = UvCsr(self.ms[k], self.ns[k], nnz, _ptr(rp), _ptr(ci), _ptr(va))
            bp[k] = bb.ctypes.data
            cpp[k] = cc.ctypes.data
        o = default_opts()
        o.mu = float(mu)
        o.precision = {"fp64": UV_FP64, "mixed": UV_MIXED}[precision]
        o.check_every = int(check_every)
        o.eps_kkt = float(eps)
        o.max_iter = int(max_iter)
        o.full_checks = 1 if full_checks else 0
        o.hip_stream = stream
        o.use_graph = 1 if use_graph else 0
        self.precision = precision
        h = ctypes.c_void_p()
        _check(L.batch_create(self.count, csrs, bp, cpp, ctypes.byref(o), ctypes.byref(h)),
               "batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def iterate(self, k: int) -> int:
        """Runs up to k iterations of every running instance; returns how
        many are still running."""
        a = ctypes.c_int32(0)
        _check(lib().batch_iterate(self._h, int(k), ctypes.byref(a)), "batch_iterate")
        return a.value

    def residuals(self, i: int) -> dict:
        r = UvResiduals()
        rc = lib().batch_residuals(self._h, int(i), ctypes.byref(r))
        if rc != UV_ENUMERIC:  # a numeric failure is reported in the status
            _check(rc, "batch_residuals")
        d = {k: getattr(r, k) for k, _ in UvResiduals._fields_}
        d["status"] = STATUS.get(d["status"], d["status"])
        return d

    def solution(self, i: int) -> dict:
        n, m = self.ns[i], self.ms[i]
        x, z, d, lam = np.empty(n), np.empty(n), np.empty(n), np.empty(m)
        _check(lib().batch_solution(self._h, int(i), _ptr(x), _ptr(z), _ptr(lam), _ptr(d)),
               "batch_solution")
        return {"x": x, "z": z, "delta": d, "lambda": lam}

    def set_start(self, i: int, x=None, z=None, delta=None, lam=None):
        n, m = self.ns[i], self.ms[i]
        args = (_f64(x, n), _f64(z, n), _f64(delta, n), _f64(lam, m))
        _check(lib().batch_set_start(self._h, int(i), *[_ptr(a) for a in args]), "batch_set_start")

    def set_tiles(self, threads: int, lanes):
        arr = (ctypes.c_int32 * 8)(*[int(v) for v in lanes])
        _check(lib().batch_set_tiles(self._h, int(threads), arr), "batch_set_tiles")

    def get_tiles(self):
        t = ctypes.c_int32()
        arr = (ctypes.c_int32 * 8)()
        _check(lib().batch_get_tiles(self._h, ctypes.byref(t), arr), "batch_get_tiles")
        return t.value, list(arr)

    def time(self, bucket: int, iters: int) -> float:
        ms = ctypes.c_double()
        _check(lib().batch_time(self._h, int(bucket), int(iters), ctypes.byref(ms)), "batch_time")
        return ms.value

    def info(self) -> dict:
        arr = (ctypes.c_int64 * 6)()
        _check(lib().batch_info(self._h, arr), "batch_info")
        return dict(zip(("count", "rows", "cols", "nnz", "workgroups", "lds_bytes"), list(arr)))

    def bucket_counts(self):
        out = [0, 0, 0, 0]
        for m in self.ms:
            out[sum(m >= lo for lo in self.BUCKETS) - 1] += 1
        return out


def _bind_family(L):
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.family_create.argtypes = [ctypes.POINTER(UvCsr), P, i32, ctypes.POINTER(UvOpts), ctypes.POINTER(P)]
    L.family_create.restype = ctypes.c_int
    L.family_set_rhs.argtypes = [P, i32, P]
    L.family_set_rhs.restype = ctypes.c_int
    L.family_set_start.argtypes = [P, P, P, P, P]
    L.family_set_start.restype = ctypes.c_int
    L.family_set_start_predicted.argtypes = [P, P, i64, i32]
    L.family_set_start_predicted.restype = ctypes.c_int
    L.family_refill.argtypes = [P, i32, P, P, P, i64, i32]
    L.family_refill.restype = ctypes.c_int
    L.family_iterate.argtypes = [P, i64, ctypes.POINTER(i32)]
    L.family_iterate.restype = ctypes.c_int
    L.family_residuals.argtypes = [P, P]
    L.family_residuals.restype = ctypes.c_int
    L.family_solution.argtypes = [P, P, P, P, P]
    L.family_solution.restype = ctypes.c_int
    L.family_member_state.argtypes = [P, i32, P, P, P, P]
    L.family_member_state.restype = ctypes.c_int
    L.family_solution_device.argtypes = [P, P, i64]
    L.family_solution_device.restype = ctypes.c_int
    L.family_destroy.argtypes = [P]
    L.family_destroy.restype = None


class Family:
    """One A and c (orthant cone) with up to B right-hand sides iterated
    together (B a multiple of 64)."""

    def __init__(self, m, n, row_ptr, col_idx, val, c, B=64, *, mu=1.0, precision="mixed",
                 check_every=10, eps=1e-4, max_iter=0, use_graph=True, stream=None):
        L = lib()
        if not hasattr(L, "_family_bound"):
            _bind_family(L)
            L._family_bound = True
        self.m, self.n, self.B = int(m), int(n), int(B)
        rp, ci, va, nnz = _csr(self.m, row_ptr, col_idx, val)
        cc = _f64(c, self.n)
        csr = UvCsr(self.m, self.n, nnz, _ptr(rp), _ptr(ci), _ptr(va))
        o = default_opts()
        o.mu = float(mu)
        o.precision = {"fp64": UV_FP64, "mixed": UV_MIXED}[precision]
        o.check_every = int(check_every)
        o.eps_kkt = float(eps)
        o.max_iter = int(max_iter)
        o.hip_stream = stream
        o.use_graph = 1 if use_graph else 0
        self.precision = precision
        self.nb = 0
        h = ctypes.c_void_p()
        _check(L.family_create(ctypes.byref(csr), _ptr(cc), self.B, ctypes.byref(o), ctypes.byref(h)),
               "family_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().family_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _mat(self, a, cols):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (self.nb, cols):
            raise ValueError(f"expected shape {(self.nb, cols)}, got {a.shape}")
        return a

    def set_rhs(self, b):
        b = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
        if b.shape[1] != self.m or not 1 <= b.shape[0] <= self.B:
            raise ValueError(f"right-hand sides must be (nb <= {self.B}, {self.m})")
        self.nb = b.shape[0]
        _check(lib().family_set_rhs(self._h, self.nb, _ptr(b)), "family_set_rhs")

    def set_start(self, x=None, z=None, delta=None, lam=None):
        args = (self._mat(x, self.n), self._mat(z, self.n), self._mat(delta, self.n),
                self._mat(lam, self.m))
        _check(lib().family_set_start(self._h, *[_ptr(a) for a in args]), "family_set_start")

    def set_start_predicted(self, dev_ptr: int, ld: int, parts: str = "both"):
        """Start from a device FP32 matrix whose row l is [x ; lambda];
        parts: "primal", "dual" or "both" of the prediction are used."""
        code = {"primal": 1, "dual": 2, "both": 3}[parts]
        _check(lib().family_set_start_predicted(self._h, ctypes.c_void_p(dev_ptr), int(ld), code),
               "family_set_start_predicted")

    def refill(self, slots, b, dev_ptr=None, ld=0, parts="both"):
        """New members into stopped slots: right-hand sides b (len(slots) x m)
        and the zero start, or the predicted start of the device FP32 rows
        [x ; lambda] at dev_ptr (row stride ld) for the members in order."""
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        b = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
        if b.shape != (sl.size, self.m):
            raise ValueError(f"right-hand sides must be ({sl.size}, {self.m})")
        code = {"primal": 1, "dual": 2, "both": 3}[parts]
        ptr = ctypes.c_void_p(dev_ptr) if dev_ptr else None
        _check(lib().family_refill(self._h, int(sl.size), _ptr(sl), _ptr(b), ptr, int(ld), code),
               "family_refill")

    def iterate(self, k: int) -> int:
        a = ctypes.c_int32(0)
        _check(lib().family_iterate(self._h, int(k), ctypes.byref(a)), "family_iterate")
        return a.value

    def residuals(self):
        arr = (UvResiduals * max(self.nb, 1))()
        rc = lib().family_residuals(self._h, arr)
        if rc != UV_ENUMERIC:  # a numeric failure is reported in the statuses
            _check(rc, "family_residuals")
        out = []
        for r in arr[: self.nb]:
            d = {k: getattr(r, k) for k, _ in UvResiduals._fields_}
            d["status"] = STATUS.get(d["status"], d["status"])
            out.append(d)
        return out

    def status_iters(self):
        """(status codes, iteration counts) of the nb members as numpy
        arrays (0 running, 1 converged, 2 max_iter, 3 numeric): residuals()
        without building a dict per member, for drivers that poll often."""
        arr = (UvResiduals * max(self.nb, 1))()
        rc = lib().family_residuals(self._h, arr)
        if rc != UV_ENUMERIC:
            _check(rc, "family_residuals")
        a = np.frombuffer(arr, dtype=_RES_DTYPE, count=self.nb)
        return a["status"].copy(), a["iter"].copy()

    def solution(self) -> dict:
        nb, n, m = self.nb, self.n, self.m
        x, z, d, lam = np.empty((nb, n)), np.empty((nb, n)), np.empty((nb, n)), np.empty((nb, m))
        _check(lib().family_solution(self._h, _ptr(x), _ptr(z), _ptr(lam), _ptr(d)), "family_solution")
        return {"x": x, "z": z, "delta": d, "lambda": lam}

    def member_state(self, slot: int) -> dict:
        """The iterate of the member in one slot (the state Solver.resume
        takes to continue its run)."""
        n, m = self.n, self.m
        x, z, d, lam = np.empty(n), np.empty(n), np.empty(n), np.empty(m)
        _check(lib().family_member_state(self._h, int(slot), _ptr(x), _ptr(z), _ptr(lam), _ptr(d)),
               "family_member_state")
        return {"x": x, "z": z, "delta": d, "lambda": lam}

    def solution_device(self, dev_ptr: int, ld: int):
        """Writes FP32 rows [z ; lambda] of the current instances to device memory."""
        _check(lib().family_solution_device(self._h, ctypes.c_void_p(dev_ptr), int(ld)),
               "family_solution_device")


class Literal:
    """Algorithm 1 as printed on the GPU (FP64, orthant cone, y and gamma stored)."""

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, *, mu=1.0, stream=None):
        L = lib()
        if not hasattr(L, "_literal_bound"):
            P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            L.literal_create.argtypes = [ctypes.POINTER(UvCsr), P, P, ctypes.POINTER(UvOpts), ctypes.POINTER(P)]
            L.literal_create.restype = ctypes.c_int
            L.literal_iterate.argtypes = [P, i64]
            L.literal_iterate.restype = ctypes.c_int
            L.literal_solution.argtypes = [P, P, P, P, P, P, P]
            L.literal_solution.restype = ctypes.c_int
            L.literal_time.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
            L.literal_time.restype = ctypes.c_int
            L.literal_destroy.argtypes = [P]
            L.literal_destroy.restype = None
            L._literal_bound = True
        self.m, self.n = int(m), int(n)
        rp, ci, va, self.nnz = _csr(self.m, row_ptr, col_idx, val)
        csr = UvCsr(self.m, self.n, self.nnz, _ptr(rp), _ptr(ci), _ptr(va))
        o = default_opts()
        o.mu = float(mu)
        o.hip_stream = stream
        h = ctypes.c_void_p()
        _check(L.literal_create(ctypes.byref(csr), _ptr(_f64(b, self.m)), _ptr(_f64(c, self.n)),
                                ctypes.byref(o), ctypes.byref(h)), "literal_create")
        self._h = h

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst["m"], inst["n"], inst["row_ptr"], inst["col_idx"], inst["val"], inst["b"],
                   inst["c"], **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().literal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def iterate(self, k: int):
        _check(lib().literal_iterate(self._h, int(k)), "literal_iterate")

    def solution(self) -> dict:
        x, z, d = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        lam, y, g = np.empty(self.m), np.empty(self.nnz), np.empty(self.nnz)
        _check(lib().literal_solution(self._h, _ptr(x), _ptr(z), _ptr(lam), _ptr(d), _ptr(y), _ptr(g)),
               "literal_solution")
        return {"x": x, "z": z, "delta": d, "lambda": lam, "y": y, "gamma": g}

    def time(self, iters: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().literal_time(self._h, int(iters), ctypes.byref(a), ctypes.byref(b)), "literal_time")
        return a.value, b.value


def _bind_standard():
    """Argument types of the standard-ADMM entry points (once)."""
    L = lib()
    if not hasattr(L, "_standard_bound"):
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.standard_create.argtypes = [ctypes.POINTER(UvCsr), P, P, ctypes.POINTER(UvCones), ctypes.POINTER(UvOpts),
                                      i32, f64, ctypes.POINTER(P)]
        L.standard_create.restype = ctypes.c_int
        L.standard_set_state.argtypes = [P, P, P, P]
        L.standard_set_state.restype = ctypes.c_int
        L.standard_iterate.argtypes = [P, i64, ctypes.POINTER(i32)]
        L.standard_iterate.restype = ctypes.c_int
        L.standard_residuals.argtypes = [P, ctypes.POINTER(UvResiduals), ctypes.POINTER(i64)]
        L.standard_residuals.restype = ctypes.c_int
        L.standard_solution.argtypes = [P, P, P, P, P, P]
        L.standard_solution.restype = ctypes.c_int
        L.standard_launch_shape.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.standard_launch_shape.restype = ctypes.c_int
        L.standard_destroy.argtypes = [P]
        L.standard_destroy.restype = None
        L._standard_bound = True
    return L


class Standard:
    """Baseline: standard two-block ADMM with a warm-started CG solve of the
    block system every iteration (FP64; orthant and Lorentz cones), on the
    same sparse product kernels as the UV solver."""

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, *, n_orth=None, soc_sizes=(), mu=1.0, cg_iters=10,
                 cg_tol=0.0, check_every=10, eps=1e-4, max_iter=0, slabs_row=0, slabs_col=0, full_checks=False,
                 use_graph=True, stream=None):
        L = _bind_standard()
        self.m, self.n = int(m), int(n)
        rp, ci, va, self.nnz = _csr(self.m, row_ptr, col_idx, val)
        csr = UvCsr(self.m, self.n, self.nnz, _ptr(rp), _ptr(ci), _ptr(va))
        o = default_opts()
        o.mu = float(mu)
        o.check_every = int(check_every)
        o.eps_kkt = float(eps)
        o.max_iter = int(max_iter)
        o.slabs_row = int(slabs_row)
        o.slabs_col = int(slabs_col)
        o.full_checks = 1 if full_checks else 0
        o.use_graph = 1 if use_graph else 0
        o.hip_stream = stream
        sizes = np.ascontiguousarray(soc_sizes, dtype=np.int32)
        cones = UvCones(self.n if n_orth is None else int(n_orth), int(sizes.size),
                        _ptr(sizes) if sizes.size else None)
        h = ctypes.c_void_p()
        _check(L.standard_create(ctypes.byref(csr), _ptr(_f64(b, self.m)), _ptr(_f64(c, self.n)),
                                 ctypes.byref(cones), ctypes.byref(o), int(cg_iters), float(cg_tol),
                                 ctypes.byref(h)), "standard_create")
        self._h = h

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst["m"], inst["n"], inst["row_ptr"], inst["col_idx"], inst["val"], inst["b"],
                   inst["c"], n_orth=inst["n_orth"], soc_sizes=inst["soc_sizes"], **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().standard_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_state(self, x2=None, lam=None, nu=None):
        args = (_f64(x2, self.n), _f64(lam, self.n), _f64(nu, self.m))
        _check(lib().standard_set_state(self._h, *[_ptr(a) for a in args]), "standard_set_state")

    def iterate(self, k: int) -> bool:
        done = ctypes.c_int32(0)
        rc = lib().standard_iterate(self._h, int(k), ctypes.byref(done))
        if rc not in (UV_OK, UV_ENUMERIC):
            _check(rc, "standard_iterate")
        return bool(done.value)

    def residuals(self) -> dict:
        r = UvResiduals()
        steps = ctypes.c_int64()
        _check(lib().standard_residuals(self._h, ctypes.byref(r), ctypes.byref(steps)), "standard_residuals")
        d = {k: getattr(r, k) for k in ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "iter", "status")}
        d["status"] = STATUS.get(d["status"], d["status"])
        d["cg_steps"] = steps.value
        return d

    def solution(self) -> dict:
        x1, x2, lam, d = (np.empty(self.n) for _ in range(4))
        nu = np.empty(self.m)
        _check(lib().standard_solution(self._h, _ptr(x1), _ptr(x2), _ptr(lam), _ptr(nu), _ptr(d)),
               "standard_solution")
        return {"x1": x1, "x2": x2, "lam": lam, "nu": nu, "delta": d}

    def launch_shape(self) -> dict:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().standard_launch_shape(self._h, ctypes.byref(a), ctypes.byref(b)), "standard_launch_shape")
        return {"slabs_row": a.value, "slabs_col": b.value}


def probe_gather(nnz: int, table_len: int, slabs: int = 1, fp64: bool = True, reps: int = 20,
                 seed: int = 1) -> float:
    """Average duration (ms) of the random-gather probe kernel: nnz streamed
    (index, value) pairs, each gathering a table entry at a random position,
    workgroups confined to one of `slabs` table parts."""
    L = lib()
    if not hasattr(L, "_probe_bound"):
        L.probe_gather.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.probe_gather.restype = ctypes.c_int
        L._probe_bound = True
    ms = ctypes.c_double()
    _check(L.probe_gather(int(nnz), int(table_len), int(slabs), 1 if fp64 else 0, int(reps), int(seed),
                          ctypes.byref(ms)), "probe_gather")
    return ms.value
