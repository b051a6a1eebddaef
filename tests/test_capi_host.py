"""Host-only checks of the C ABI: the library loads, exports every function
include/uvadmm.h declares, and rejects malformed input before any device
call (validation runs on the host first, so these need no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_2203_05027_amd import solver as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, re.M):
            if not m.group(0).lstrip().startswith(("#", "typedef", "return")):
                names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert "solver_create" in names and "solver_iterate" in names
    L = S.lib()
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_strerror_names_every_code():
    L = S.lib()
    for code in range(0, -9, -1):
        assert L.solver_strerror(code).decode() != "unknown error code"
    assert L.solver_strerror(-99).decode() == "unknown error code"


def test_default_opts():
    o = S.default_opts()
    assert o.mu == 1.0 and o.precision == S.UV_FP64 and o.check_every == 10
    assert o.eps_kkt == 1e-4 and o.max_iter == 0 and o.use_graph == 1


def _try_create(m, n, rp, ci, va, b, c, n_orth, sizes=(), **kw):
    with pytest.raises(S.UvError) as ei:
        S.Solver(m, n, rp, ci, va, b, c, n_orth, sizes, **kw)
    return ei.value.code


GOOD = dict(m=2, n=3, rp=[0, 2, 3], ci=[0, 2, 1], va=[1.0, 2.0, 3.0],
            b=[1.0, 1.0], c=[1.0, 1.0, 1.0])


def _args(**over):
    d = dict(GOOD)
    d.update(over)
    return d


@pytest.mark.parametrize("over,code", [
    (dict(rp=[1, 2, 3]), S.UV_EBADCSR),            # row_ptr[0] != 0
    (dict(rp=[0, 3, 2]), S.UV_EBADCSR),            # not monotone / exceeds nnz
    (dict(ci=[0, 3, 1]), S.UV_EBADCSR),            # column out of range
    (dict(ci=[0, -1, 1]), S.UV_EBADCSR),           # negative column
    (dict(ci=[2, 0, 1]), S.UV_EBADCSR),            # not increasing in a row
    (dict(ci=[1, 1, 1]), S.UV_EBADCSR),            # duplicate in a row
])
def test_rejects_malformed_csr(over, code):
    a = _args(**over)
    assert _try_create(a["m"], a["n"], a["rp"], a["ci"], a["va"], a["b"], a["c"], 3) == code


@pytest.mark.parametrize("n_orth,sizes", [(2, ()), (0, (2,)), (1, (1, 0)), (0, (4,)), (-1, (4,))])
def test_rejects_bad_cones(n_orth, sizes):
    a = GOOD
    assert _try_create(a["m"], a["n"], a["rp"], a["ci"], a["va"], a["b"], a["c"],
                       n_orth, sizes) == S.UV_ECONE


def test_rejects_oversized_cone():
    n = S.UV_MAX_CONE + 1
    code = _try_create(1, n, [0, 1], [0], [1.0], [1.0], np.ones(n), 0, (n,))
    assert code == S.UV_ECONE


@pytest.mark.parametrize("kw", [dict(mu=0.0), dict(mu=-1.0), dict(mu=float("nan")),
                                dict(check_every=0), dict(eps=-1.0), dict(max_iter=-5),
                                dict(lanes_row=3), dict(lanes_col=128), dict(unroll_row=3),
                                dict(unroll_col=16)])
def test_rejects_bad_options(kw):
    a = GOOD
    assert _try_create(a["m"], a["n"], a["rp"], a["ci"], a["va"], a["b"], a["c"], 3,
                       **kw) == S.UV_EINVAL


def test_rejects_empty_dimensions():
    assert _try_create(0, 3, [0], [], [], [], [1.0, 1.0, 1.0], 3) == S.UV_EINVAL


def test_rejects_nnz_mismatch():
    """row_ptr[m] must equal the declared nnz."""
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([0, 2, 1], np.int32)
    va = np.array([1.0, 2.0, 3.0])
    b, c = np.ones(2), np.ones(3)
    for nnz in (2, 4):
        csr = S.UvCsr(2, 3, nnz, S._ptr(rp), S._ptr(ci), S._ptr(va))
        cones = S.UvCones(3, 0, None)
        h = ctypes.c_void_p()
        rc = S.lib().solver_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), ctypes.byref(cones),
                                   None, ctypes.byref(h))
        assert rc == S.UV_EBADCSR and not h.value


def test_null_arguments():
    L = S.lib()
    h = ctypes.c_void_p()
    assert L.solver_create(None, None, None, None, None, ctypes.byref(h)) == S.UV_EINVAL
    assert L.solver_iterate(None, 1, None) == S.UV_EINVAL
    assert L.solver_residuals(None, None) == S.UV_EINVAL
    assert L.solver_solution(None, None, None, None, None) == S.UV_EINVAL
    L.solver_destroy(None)


def _batch_err(insts, **kw):
    with pytest.raises(S.UvError) as ei:
        S.Batch(insts, **kw)
    return ei.value.code


def test_batch_rejects_bad_input():
    good = dict(m=2, n=3, row_ptr=[0, 2, 3], col_idx=[0, 2, 1], val=[1.0, 2.0, 3.0],
                b=[1.0, 1.0], c=[1.0, 1.0, 1.0])
    bad = dict(good, col_idx=[2, 0, 1])
    assert _batch_err([good, bad]) == S.UV_EBADCSR
    assert _batch_err([good], mu=0.0) == S.UV_EINVAL
    assert _batch_err([good], check_every=0) == S.UV_EINVAL
    # x and u of an instance must fit in one workgroup's LDS (160 KiB less
    # the kernel's 1 KiB of static LDS: 20,401 FP64 values are 163,208 bytes)
    assert _batch_err([dict(good, m=1, n=20_400, row_ptr=[0, 1], col_idx=[0], val=[1.0], b=[1.0],
                            c=np.ones(20_400))], precision="fp64") == S.UV_ETOOBIG
    n = 41_000
    wide = dict(m=1, n=n, row_ptr=[0, 1], col_idx=[0], val=[1.0], b=[1.0], c=np.ones(n))
    assert _batch_err([good, wide], precision="mixed") == S.UV_ETOOBIG
    assert _batch_err([dict(wide, n=20_500, c=np.ones(20_500))], precision="fp64") == S.UV_ETOOBIG


def _std_err(**kw):
    a = dict(GOOD)
    args = {k: kw.pop(k) for k in list(kw) if k in a}
    a.update(args)
    with pytest.raises(S.UvError) as ei:
        S.Standard(a["m"], a["n"], a["rp"], a["ci"], a["va"], a["b"], a["c"], **kw)
    return ei.value.code


@pytest.mark.parametrize("kw,code", [
    (dict(rp=[1, 2, 3]), S.UV_EBADCSR),
    (dict(ci=[2, 0, 1]), S.UV_EBADCSR),
    (dict(ci=[0, 3, 1]), S.UV_EBADCSR),
    (dict(mu=0.0), S.UV_EINVAL),
    (dict(cg_iters=-1), S.UV_EINVAL),
    (dict(cg_tol=-1e-3), S.UV_EINVAL),
    (dict(cg_tol=float("inf")), S.UV_EINVAL),
    (dict(check_every=0), S.UV_EINVAL),
    (dict(slabs_row=3), S.UV_EINVAL),
    (dict(slabs_col=8), S.UV_EINVAL),
])
def test_standard_rejects_bad_input(kw, code):
    """The standard-ADMM baseline validates on the host before any device call."""
    assert _std_err(**kw) == code


def test_standard_rejects_mixed_precision():
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([0, 2, 1], np.int32)
    va = np.array([1.0, 2.0, 3.0])
    b, c = np.ones(2), np.ones(3)
    csr = S.UvCsr(2, 3, 3, S._ptr(rp), S._ptr(ci), S._ptr(va))
    o = S.default_opts()
    o.precision = S.UV_MIXED
    h = ctypes.c_void_p()
    L = S._bind_standard()
    assert L.standard_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), None, ctypes.byref(o), 2, 0.0,
                             ctypes.byref(h)) == S.UV_EINVAL and not h.value
    assert L.standard_create(None, None, None, None, None, 2, 0.0, ctypes.byref(h)) == S.UV_EINVAL
    assert L.standard_iterate(None, 1, None) == S.UV_EINVAL
    assert L.standard_residuals(None, None, None) == S.UV_EINVAL
    assert L.standard_solution(None, None, None, None, None, None) == S.UV_EINVAL
    L.standard_destroy(None)


@pytest.mark.parametrize("args", [(0, 100, 1, 1, 5), (1 << 31, 100, 1, 1, 5), (100, 100, 0, 1, 5),
                                  (100, 100, 9, 1, 5), (100, 4, 8, 1, 5), (100, 100, 1, 1, 0)])
def test_probe_rejects_bad_arguments(args):
    with pytest.raises(S.UvError) as ei:
        S.probe_gather(*args)
    assert ei.value.code == S.UV_EINVAL


def test_mul_row_vector_rejects_bad_arguments():
    from paper_2203_05027_amd import learn
    L = learn._bind()
    assert L.mul_row_vector(2, 3, None, 3, None, None) == S.UV_EINVAL
    assert L.mul_row_vector(-1, 3, ctypes.c_void_p(8), 3, ctypes.c_void_p(8), None) == S.UV_EINVAL
    assert L.mul_row_vector(2, 3, ctypes.c_void_p(8), 2, ctypes.c_void_p(8), None) == S.UV_EINVAL


def test_rejects_nnz_beyond_32bit_indices():
    """Device indices are 32-bit: a declared nnz of 2^31 is refused before
    any array is read past its first entries."""
    rp = np.array([0, 1], np.int64)
    ci = np.array([0], np.int32)
    va = np.array([1.0])
    b, c = np.ones(1), np.ones(1)
    csr = S.UvCsr(1, 1, 1 << 31, S._ptr(rp), S._ptr(ci), S._ptr(va))
    cones = S.UvCones(1, 0, None)
    h = ctypes.c_void_p()
    L = S.lib()
    assert L.solver_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), ctypes.byref(cones), None,
                           ctypes.byref(h)) == S.UV_ETOOBIG and not h.value
    L = S._bind_standard()
    assert L.standard_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), None, None, 2, 0.0,
                             ctypes.byref(h)) == S.UV_ETOOBIG and not h.value


@pytest.mark.parametrize("n_orth,sizes", [(2, ()), (0, (2,)), (1, (1, 0)), (-1, (4,))])
def test_standard_rejects_bad_cones(n_orth, sizes):
    a = GOOD
    with pytest.raises(S.UvError) as ei:
        S.Standard(a["m"], a["n"], a["rp"], a["ci"], a["va"], a["b"], a["c"], n_orth=n_orth, soc_sizes=sizes)
    assert ei.value.code == S.UV_ECONE


def _csr_is_valid(m, n, rp, ci):
    if rp[0] != 0:
        return False
    for i in range(m):
        if rp[i + 1] < rp[i] or rp[i + 1] > rp[m]:
            return False
        row = ci[rp[i]:rp[i + 1]]
        if any(j < 0 or j >= n for j in row) or any(b <= a for a, b in zip(row, row[1:])):
            return False
    return True


@settings(max_examples=400, deadline=None)
@given(st.data())
def test_csr_validation_agrees_with_a_plain_check(data):
    """Random small CSR inputs, malformed about half the time (offsets out of
    order, indices out of range, repeated or unsorted within a row): the
    library answers UV_EBADCSR exactly when a plain reading of the format
    says the input is malformed (a well-formed one then fails only for the
    missing GPU, or succeeds on one)."""
    m = data.draw(st.integers(1, 5), "m")
    n = data.draw(st.integers(1, 6), "n")
    nnz = data.draw(st.integers(0, 12), "nnz")
    inner = sorted(data.draw(st.lists(st.integers(0, nnz), min_size=m - 1, max_size=m - 1), "rp"))
    rp = [0] + inner + [nnz]
    if m > 1 and data.draw(st.booleans(), "swap offsets"):
        i = data.draw(st.integers(1, m - 1), "at")
        rp[i] = data.draw(st.integers(-1, nnz + 1), "offset")
    if data.draw(st.booleans(), "sorted rows"):
        ci = []
        for i in range(m):
            k = max(0, min(nnz, rp[i + 1]) - max(0, rp[i]))
            ci += sorted(data.draw(st.lists(st.integers(0, n - 1), min_size=k, max_size=k, unique=True), "row")) \
                if k <= n else list(range(k))
        ci = (ci + [0] * nnz)[:nnz]
    else:
        ci = data.draw(st.lists(st.integers(-1, n), min_size=nnz, max_size=nnz), "ci")
    va = [1.0] * nnz
    valid = _csr_is_valid(m, n, rp, ci)
    try:
        S.Solver(m, n, rp, ci, va, np.ones(m), np.ones(n), n).close()
        code = S.UV_OK
    except S.UvError as e:
        code = e.code
    if valid:
        assert code not in (S.UV_EBADCSR, S.UV_EINVAL), (rp, ci, code)
    else:
        assert code == S.UV_EBADCSR, (rp, ci, code)


@settings(max_examples=300, deadline=None)
@given(st.data())
def test_cone_validation_agrees_with_a_plain_check(data):
    """Random cone specifications on a well-formed A: UV_ECONE exactly when
    the orthant count is negative, a Lorentz cone has fewer than 1 or more
    than UV_MAX_CONE coordinates, or the sizes do not add up to n."""
    n = data.draw(st.integers(1, 12), "n")
    n_orth = data.draw(st.integers(-1, n + 1), "n_orth")
    sizes = data.draw(st.lists(st.integers(-1, 8), max_size=4), "sizes")
    if data.draw(st.booleans(), "huge cone"):
        sizes.append(1025)
    m = 2
    rp = [0, 1, 2]
    ci = [0, min(1, n - 1)] if n > 1 else [0, 0]
    valid = n_orth >= 0 and all(1 <= q <= 1024 for q in sizes) and n_orth + sum(sizes) == n
    try:
        S.Solver(m, n, rp, ci, [1.0, 2.0], np.ones(m), np.ones(n), n_orth, sizes).close()
        code = S.UV_OK
    except S.UvError as e:
        code = e.code
    if valid:
        assert code not in (S.UV_ECONE, S.UV_EBADCSR, S.UV_EINVAL), (n_orth, sizes, code)
    else:
        assert code == S.UV_ECONE, (n_orth, sizes, code)


# ctypes mirrors of the header's structs: every field at the C compiler's
# offset and the same total size (a field added on one side only would shift
# every later one and corrupt options silently).
_MIRRORS = {"uv_csr": S.UvCsr, "uv_cones": S.UvCones, "uv_opts": S.UvOpts,
            "uv_residuals": S.UvResiduals, "uv_history": S.UvHistory}


def test_ctypes_structs_match_the_header(tmp_path):
    import shutil
    import subprocess
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "uvadmm.h"', "int main(void) {"]
    for cname, py in _MIRRORS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in _MIRRORS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("field,value", [("full_checks", 2), ("full_checks", -1), ("history", -1),
                                         ("history", (1 << 24) + 1), ("resident", 3), ("criterion", 3)])
def test_rejects_out_of_range_options(field, value):
    """Options the Python keywords cannot express, set on the C struct: the
    library validates them before any device work."""
    a = GOOD
    rp = np.ascontiguousarray(a["rp"], dtype=np.int64)
    ci = np.ascontiguousarray(a["ci"], dtype=np.int32)
    va = np.ascontiguousarray(a["va"], dtype=np.float64)
    b = np.ascontiguousarray(a["b"], dtype=np.float64)
    c = np.ascontiguousarray(a["c"], dtype=np.float64)
    csr = S.UvCsr(a["m"], a["n"], 3, S._ptr(rp), S._ptr(ci), S._ptr(va))
    cones = S.UvCones(3, 0, None)
    o = S.default_opts()
    setattr(o, field, value)
    h = ctypes.c_void_p()
    rc = S.lib().solver_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), ctypes.byref(cones), ctypes.byref(o),
                               ctypes.byref(h))
    assert rc == S.UV_EINVAL and not h.value


def test_batch_and_baseline_reject_out_of_range_full_checks():
    a = GOOD
    rp = np.ascontiguousarray(a["rp"], dtype=np.int64)
    ci = np.ascontiguousarray(a["ci"], dtype=np.int32)
    va = np.ascontiguousarray(a["va"], dtype=np.float64)
    b = np.ascontiguousarray(a["b"], dtype=np.float64)
    c = np.ascontiguousarray(a["c"], dtype=np.float64)
    csr = S.UvCsr(a["m"], a["n"], 3, S._ptr(rp), S._ptr(ci), S._ptr(va))
    o = S.default_opts()
    o.full_checks = 2
    L = S.lib()
    S._bind_batch(L)
    h = ctypes.c_void_p()
    csrs = (S.UvCsr * 1)(csr)
    bp = (ctypes.c_void_p * 1)(b.ctypes.data)
    cp = (ctypes.c_void_p * 1)(c.ctypes.data)
    assert L.batch_create(1, csrs, bp, cp, ctypes.byref(o), ctypes.byref(h)) == S.UV_EINVAL and not h.value
    Ls = S._bind_standard()
    cones = S.UvCones(3, 0, None)
    rc = Ls.standard_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), ctypes.byref(cones), ctypes.byref(o), 2, 0.0,
                            ctypes.byref(h))
    assert rc == S.UV_EINVAL and not h.value
    # the same arguments with full_checks = 1 pass validation (and then need a device)
    o.full_checks = 1
    rc = Ls.standard_create(ctypes.byref(csr), S._ptr(b), S._ptr(c), ctypes.byref(cones), ctypes.byref(o), 2, 0.0,
                            ctypes.byref(h))
    assert rc != S.UV_EINVAL
    if rc == S.UV_OK:
        Ls.standard_destroy(h)
