"""Seeded synthetic problem generators.

These build the inputs that both the solver and its checkers consume.  They
hold none of the solver's arithmetic: they only draw random data and form the
right-hand sides that make each problem feasible and bounded by construction.

Every problem is ``min c'x  s.t.  A x = b,  x in K`` (Section II) with
``K = R_+^{n_orth} x K_{s_1} x ... x K_{s_q}`` (orthant coordinates first, then
the second-order cones in order; each cone's first coordinate is its ``t``).

Workloads (the paper's experiments use random sparse A with N(0,1) values and
K the orthant or a product of small Lorentz cones, Section V; the families
below keep that shape but build b and c from a known primal-dual pair so the
problem is bounded with a known optimum):

* LP family: A holds exactly ``k`` nonzeros per column at distinct uniformly
  random rows, values N(0,1) (rows optionally rescaled to unit 2-norm);
  ``x0 = max(N(0,I), 0)``, ``b = A x0``, ``y0 ~ N(0,I)``,
  ``s0 = U(0,1)`` where ``x0 = 0`` and 0 elsewhere, ``c = A'y0 + s0``.
  Then x0 and (y0, s0) are complementary and primal/dual feasible, so x0 is
  optimal with value ``c'x0 = b'y0``.
* SOCP family: cones of uniform integer size, ``x0`` strictly inside each
  cone (``u ~ N(0,I)``, ``t = ||u|| + U(0.1, 1)``), ``b = A x0``, ``s0`` an
  independent draw of the same recipe, ``c = A'y0 + s0``: strictly feasible
  on both sides, so bounded, with ``b'y0 <= p* <= c'x0``.
* Batched family: many LP-family instances with log-uniform sizes.
* Parametric family: one fixed A and c, ``b(theta) = A max(W theta + w, 0)``.

Random numbers come from numpy's PCG64 generator (``default_rng(seed)``);
sampling ``k`` distinct rows per column redraws collisions until none remain.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "lp_instance", "socp_instance", "conic_instance", "batch_lp_sizes", "batch_lp_instance",
    "ParametricFamily", "config_instance", "CONFIGS",
]


def _distinct_rows(rng, m: int, n: int, k: int) -> np.ndarray:
    """(n, k) array: row indices of column j, k distinct values in [0, m)."""
    if k > m:
        raise ValueError(f"cannot place {k} distinct nonzeros in {m} rows")
    rows = rng.integers(0, m, size=(n, k), dtype=np.int64)
    rows.sort(axis=1)
    while True:
        dup = np.zeros(rows.shape, dtype=bool)
        dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
        cnt = int(dup.sum())
        if cnt == 0:
            return rows
        rows[dup] = rng.integers(0, m, size=cnt, dtype=np.int64)
        rows.sort(axis=1)


def _csr_from_columns(m: int, n: int, rows: np.ndarray, vals: np.ndarray):
    """CSR (row_ptr int64, col_idx int32, val f64) from per-column samples."""
    k = rows.shape[1]
    r = rows.reshape(-1)
    c = np.repeat(np.arange(n, dtype=np.int64), k)
    v = vals.reshape(-1)
    order = np.argsort(r * n + c, kind="stable")
    r, c, v = r[order], c[order], v[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    return row_ptr, c.astype(np.int32), np.ascontiguousarray(v, dtype=np.float64), r


def _rows_of(row_ptr: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(row_ptr.size - 1, dtype=np.int64), np.diff(row_ptr))


def _matvec(m, rows, col_idx, val, x):
    return np.bincount(rows, weights=val * x[col_idx], minlength=m)


def _rmatvec(n, rows, col_idx, val, y):
    return np.bincount(col_idx, weights=val * y[rows], minlength=n)


def _interior_cone_points(rng, sizes: np.ndarray) -> np.ndarray:
    """Per cone of size s: (||u|| + U(0.1, 1), u) with u ~ N(0, I_{s-1})."""
    n = int(sizes.sum())
    off = np.concatenate(([0], np.cumsum(sizes)[:-1]))
    v = rng.standard_normal(n)
    sq = v * v
    sq[off] = 0.0
    norms = np.sqrt(np.add.reduceat(sq, off))
    v[off] = norms + rng.uniform(0.1, 1.0, size=sizes.size)
    return v


def lp_instance(m: int, n: int, k: int, seed: int, unit_rows: bool = False) -> dict:
    """LP family (orthant cone) with known optimum ``c'x0 = b'y0``."""
    rng = np.random.default_rng(seed)
    rows = _distinct_rows(rng, m, n, k)
    vals = rng.standard_normal((n, k))
    row_ptr, col_idx, val, r = _csr_from_columns(m, n, rows, vals)
    if unit_rows:
        nrm = np.sqrt(np.bincount(r, weights=val * val, minlength=m))
        scale = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)
        val = val * scale[r]
    x0 = np.maximum(rng.standard_normal(n), 0.0)
    y0 = rng.standard_normal(m)
    s0 = np.where(x0 == 0.0, rng.uniform(0.0, 1.0, size=n), 0.0)
    b = _matvec(m, r, col_idx, val, x0)
    c = _rmatvec(n, r, col_idx, val, y0) + s0
    return {
        "m": m, "n": n, "nnz": int(row_ptr[-1]), "row_ptr": row_ptr,
        "col_idx": col_idx, "val": val, "b": b, "c": c, "n_orth": n,
        "soc_sizes": np.zeros(0, dtype=np.int32), "x0": x0, "y0": y0, "s0": s0,
        "p_star": float(c @ x0), "d_star": float(b @ y0), "seed": seed, "unit_rows": bool(unit_rows),
    }


def conic_instance(m: int, n_orth: int, soc_sizes, k: int, seed: int) -> dict:
    """General family: K = R_+^{n_orth} x K_{soc_sizes[0]} x ...; x0 and s0
    are drawn strictly inside K (orthant part: |N(0,1)| + U(0.1, 1))."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(soc_sizes, dtype=np.int32)
    n = int(n_orth + sizes.sum())
    rows = _distinct_rows(rng, m, n, k)
    vals = rng.standard_normal((n, k))
    row_ptr, col_idx, val, r = _csr_from_columns(m, n, rows, vals)
    x0 = np.concatenate([np.abs(rng.standard_normal(n_orth)) + rng.uniform(0.1, 1.0, n_orth),
                         _interior_cone_points(rng, sizes) if sizes.size else np.zeros(0)])
    s0 = np.concatenate([np.abs(rng.standard_normal(n_orth)) + rng.uniform(0.1, 1.0, n_orth),
                         _interior_cone_points(rng, sizes) if sizes.size else np.zeros(0)])
    y0 = rng.standard_normal(m)
    b = _matvec(m, r, col_idx, val, x0)
    c = _rmatvec(n, r, col_idx, val, y0) + s0
    return {
        "m": m, "n": n, "nnz": int(row_ptr[-1]), "row_ptr": row_ptr,
        "col_idx": col_idx, "val": val, "b": b, "c": c, "n_orth": n_orth,
        "soc_sizes": sizes, "x0": x0, "y0": y0, "s0": s0,
        "p_upper": float(c @ x0), "d_lower": float(b @ y0), "seed": seed,
    }


def socp_instance(n_cones: int, k: int, seed: int, size_lo: int = 3,
                  size_hi: int = 50, m: int | None = None) -> dict:
    """SOCP family: ``n_cones`` Lorentz cones of size U{size_lo..size_hi}."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_cones).astype(np.int32)
    n = int(sizes.sum())
    if m is None:
        m = n // 2
    rows = _distinct_rows(rng, m, n, k)
    vals = rng.standard_normal((n, k))
    row_ptr, col_idx, val, r = _csr_from_columns(m, n, rows, vals)
    x0 = _interior_cone_points(rng, sizes)
    s0 = _interior_cone_points(rng, sizes)
    y0 = rng.standard_normal(m)
    b = _matvec(m, r, col_idx, val, x0)
    c = _rmatvec(n, r, col_idx, val, y0) + s0
    return {
        "m": m, "n": n, "nnz": int(row_ptr[-1]), "row_ptr": row_ptr,
        "col_idx": col_idx, "val": val, "b": b, "c": c, "n_orth": 0,
        "soc_sizes": sizes, "x0": x0, "y0": y0, "s0": s0,
        "p_upper": float(c @ x0), "d_lower": float(b @ y0), "seed": seed,
    }


def paper_instance(m: int, n: int, density: float, cone: str, seed: int) -> dict:
    """The experiments' own generator (Section V, "Problem instances"): A with
    a fraction `density` of nonzeros at uniformly random positions, values
    N(0,1); b = A proj_K(xdot) with xdot ~ N(0, I); c ~ N(0, I); K the
    orthant ("lp") or a product of size-4 Lorentz cones ("socp", n a multiple
    of 4).  Feasible by construction; unlike the families above it is not
    guaranteed to be bounded (c is unrelated to A)."""
    rng = np.random.default_rng(seed)
    target = max(int(round(density * m * n)), 1)
    pos = np.unique(rng.integers(0, m * n, size=target, dtype=np.int64))
    while pos.size < target:
        more = rng.integers(0, m * n, size=target - pos.size, dtype=np.int64)
        pos = np.unique(np.concatenate([pos, more]))
    r, cidx = pos // n, pos % n
    val = rng.standard_normal(pos.size)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    xdot = rng.standard_normal(n)
    if cone == "lp":
        n_orth, sizes = n, np.zeros(0, dtype=np.int32)
        xk = np.maximum(xdot, 0.0)
    elif cone == "socp":
        if n % 4:
            raise ValueError("n must be a multiple of 4 for (K_4)^(n/4)")
        n_orth, sizes = 0, np.full(n // 4, 4, dtype=np.int32)
        w = xdot.reshape(-1, 4)
        t, u = w[:, 0], w[:, 1:]
        a = np.linalg.norm(u, axis=1)
        xk = np.where((a <= -t)[:, None], 0.0,
                      np.where((a <= t)[:, None], w,
                               np.concatenate([((t + a) / 2)[:, None],
                                               u * ((1 + t / np.where(a > 0, a, 1)) / 2)[:, None]], axis=1)))
        xk = xk.reshape(-1)
    else:
        raise ValueError("cone must be 'lp' or 'socp'")
    b = np.bincount(r, weights=val * xk[cidx], minlength=m)
    c = rng.standard_normal(n)
    return {"m": m, "n": n, "nnz": int(pos.size), "row_ptr": row_ptr, "col_idx": cidx.astype(np.int32),
            "val": val, "b": b, "c": c, "n_orth": n_orth, "soc_sizes": sizes, "x_feasible": xk,
            "seed": seed}


def batch_lp_sizes(count: int, m_lo: int = 50, m_hi: int = 5000,
                   seed_base: int = 3_000_000) -> np.ndarray:
    """m of instance i, log-uniform in [m_lo, m_hi], drawn from seed_base + i."""
    out = np.empty(count, dtype=np.int64)
    for i in range(count):
        rng = np.random.default_rng(seed_base + i)
        out[i] = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
    return out


def batch_lp_instance(i: int, k: int = 6, m_lo: int = 50, m_hi: int = 5000,
                      seed_base: int = 3_000_000) -> dict:
    """Instance i of the batched family: n = 2m, k nonzeros per column."""
    m = int(batch_lp_sizes(1, m_lo, m_hi, seed_base + i)[0])
    return lp_instance(m, 2 * m, k, seed=(seed_base + i) * 7 + 1)


class ParametricFamily:
    """Fixed A and c; ``b(theta) = A max(W theta + w, 0)``, theta in R^p.

    ``c = A'y_c + s_c`` with ``s_c ~ U(0,1)`` on a fixed random half of the
    coordinates and 0 elsewhere, so every member is bounded (the pair
    (y_c, s_c) is dual feasible) and feasible (``max(W theta + w, 0)``).
    """

    def __init__(self, m: int = 50_000, n: int = 100_000, k: int = 8,
                 p: int = 64, seed: int = 4):
        rng = np.random.default_rng(seed)
        rows = _distinct_rows(rng, m, n, k)
        vals = rng.standard_normal((n, k))
        self.row_ptr, self.col_idx, self.val, self._r = _csr_from_columns(m, n, rows, vals)
        self.m, self.n, self.p = m, n, p
        y_c = rng.standard_normal(m)
        half = rng.permutation(n)[: n // 2]
        s_c = np.zeros(n)
        s_c[half] = rng.uniform(0.0, 1.0, size=half.size)
        self.c = _rmatvec(n, self._r, self.col_idx, self.val, y_c) + s_c
        self.W = rng.standard_normal((n, p)) / math.sqrt(p)
        self.w = rng.standard_normal(n)

    @staticmethod
    def theta(seed: int, p: int = 64) -> np.ndarray:
        return np.random.default_rng(seed).standard_normal(p)

    def x_feasible(self, theta: np.ndarray) -> np.ndarray:
        return np.maximum(self.W @ theta + self.w, 0.0)

    def b(self, theta: np.ndarray) -> np.ndarray:
        return _matvec(self.m, self._r, self.col_idx, self.val, self.x_feasible(theta))

    def b_many(self, thetas: np.ndarray) -> np.ndarray:
        """Right-hand sides of many members at once: rows of thetas -> rows
        of b (the same values as b() member by member)."""
        import scipy.sparse as sp
        thetas = np.atleast_2d(np.asarray(thetas, dtype=np.float64))
        X = np.maximum(self.W @ thetas.T + self.w[:, None], 0.0)
        A = sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))
        return np.ascontiguousarray((A @ X).T)

    def instance(self, theta: np.ndarray) -> dict:
        return {
            "m": self.m, "n": self.n, "nnz": int(self.row_ptr[-1]),
            "row_ptr": self.row_ptr, "col_idx": self.col_idx, "val": self.val,
            "b": self.b(theta), "c": self.c, "n_orth": self.n,
            "soc_sizes": np.zeros(0, dtype=np.int32),
        }


# The named workloads: small LP, large LP (unit rows), large SOCP, batched
# LPs, parametric family, and the experiments' own generator at 1e7 stored
# entries (0.5 % density; with m < n and c unrelated to A these are not
# bounded, so only the sweep rate is measured on them).  ``scale`` shrinks m,
# n (and the cone count) for tests; the sparsity per column is kept.
CONFIGS = {
    "lp_small": dict(kind="lp", m=500, n=1000, k=5, seed=0, unit_rows=False),
    "lp_large": dict(kind="lp", m=1_000_000, n=2_000_000, k=10, seed=1, unit_rows=True),
    "socp_large": dict(kind="socp", n_cones=100_000, k=8, seed=2),
    "lp_batched": dict(kind="batch", count=4096, k=6),
    "lp_parametric": dict(kind="param", m=50_000, n=100_000, k=8, p=64, seed=4),
    "paper_lp": dict(kind="paper", m=20_000, n=100_000, density=0.005, cone="lp", seed=5),
    "paper_socp": dict(kind="paper", m=20_000, n=100_000, density=0.005, cone="socp", seed=6),
    # the section's other two densities, at its largest entry count (1e7)
    # for 1.0 % and 2e6 entries for 0.1 %
    "paper_lp_0p1": dict(kind="paper", m=20_000, n=100_000, density=0.001, cone="lp", seed=7),
    "paper_socp_0p1": dict(kind="paper", m=20_000, n=100_000, density=0.001, cone="socp", seed=8),
    "paper_lp_1p0": dict(kind="paper", m=10_000, n=100_000, density=0.01, cone="lp", seed=9),
    "paper_socp_1p0": dict(kind="paper", m=10_000, n=100_000, density=0.01, cone="socp", seed=10),
}


def config_instance(name: str, scale: float = 1.0) -> dict:
    cfg = CONFIGS[name]
    if cfg["kind"] == "lp":
        m = max(int(cfg["m"] * scale), cfg["k"])
        n = max(int(cfg["n"] * scale), 1)
        inst = lp_instance(m, n, cfg["k"], cfg["seed"], cfg["unit_rows"])
    elif cfg["kind"] == "socp":
        inst = socp_instance(max(int(cfg["n_cones"] * scale), 1), cfg["k"], cfg["seed"])
    elif cfg["kind"] == "paper":
        m = max(int(cfg["m"] * scale), 1)
        n = max(int(cfg["n"] * scale) // 4 * 4, 4)
        inst = paper_instance(m, n, cfg["density"], cfg["cone"], cfg["seed"])
        inst["bounded"] = False
    else:
        raise ValueError(f"{name} is not a single-instance workload")
    inst["name"] = name
    return inst
