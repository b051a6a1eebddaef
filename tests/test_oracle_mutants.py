"""The pins must catch plausible mistakes in the oracle: each case plants one
(a dropped term, a wrong sign, a wrong index or factor) in a copy of the
oracle's C source, builds it, and runs the pin suite against it in a
subprocess; the suite has to fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "uvadmm_oracle.c")

MUTANTS = {
    "x-step drops delta/mu": ("+ h->z[j] + h->delta[j] / mu - h->c[j] / mu", "+ h->z[j] - h->c[j] / mu"),
    "x-step sign of c": ("+ h->z[j] + h->delta[j] / mu - h->c[j] / mu", "+ h->z[j] + h->delta[j] / mu + h->c[j] / mu"),
    "y-step lambda scaled by mu": ("(h->b[i] - h->lambda[i] / mu)", "(h->b[i] - h->lambda[i] * mu)"),
    "y-step gamma sign": ("+ h->x[h->ck[k]] - h->gamma[k] / mu;", "+ h->x[h->ck[k]] + h->gamma[k] / mu;"),
    "F_U from absolute values": ("d += h->ak[k] * h->ak[k];", "d += fabs(h->ak[k]);"),
    "F_V off by one": ("for (int64_t p = h->col_ptr[j]; p < h->col_ptr[j + 1]; ++p) d += 1.0;",
                       "for (int64_t p = h->col_ptr[j]; p <= h->col_ptr[j + 1]; ++p) d += 1.0;"),
    "projection head sign": ("out[0] = w1 / 2.0 + alpha / 2.0;", "out[0] = w1 / 2.0 - alpha / 2.0;"),
    "projection case order": ("} else if (alpha <= w1) {", "} else if (alpha <= -w1 + 1e-3) {"),
    "lambda update sign": ("h->lambda[i] += mu * (uy - h->b[i]);", "h->lambda[i] -= mu * (uy - h->b[i]);"),
    "gamma update uses +x": ("h->gamma[k] += mu * (h->y[k] - h->x[h->ck[k]]);",
                             "h->gamma[k] += mu * (h->y[k] + h->x[h->ck[k]]);"),
    "delta update sign": ("h->delta[j] += mu * (h->z[j] - h->x[j]);", "h->delta[j] += mu * (h->x[j] - h->z[j]);"),
    "dual residual drops delta": ("double r = atl + h->c[j] - h->delta[j];", "double r = atl + h->c[j];"),
    "U transposed in y-step sum": ("ut += h->ak[k] * h->t[k];", "ut += h->t[k];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    import oracle
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique: {old}"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle.build(src=str(src), out=str(tmp_path / "libmutant.so"))
    env = dict(os.environ, UVADMM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"


STD_SRC = os.path.join(ROOT, "oracle", "standard_oracle.c")

STD_MUTANTS = {
    "x1 step sign of lam": ("h->a[j] = h->x2[j] - h->lam[j] / mu;", "h->a[j] = h->x2[j] + h->lam[j] / mu;"),
    "v drops c/mu": ("h->v[j] = h->x1[j] + h->lam[j] / mu - h->c[j] / mu;", "h->v[j] = h->x1[j] + h->lam[j] / mu;"),
    "delta from the new x2": ("h->delta[j] = h->lam[j] + mu * (h->x1[j] - h->x2[j]);", "h->delta[j] = h->lam[j];"),
    "CG beta inverted": ("const double beta = rr_new / rr;", "const double beta = rr / rr_new;"),
    "CG residual update sign": ("h->r[i] -= alpha * h->q[i];", "h->r[i] += alpha * h->q[i];"),
    "CG ignores the warm start": ("h->r[i] = h->g[i] - h->q[i];", "h->r[i] = h->g[i];"),
    "x2 sign of A'nu": ("h->x2[j] = h->v[j] - h->tn[j];", "h->x2[j] = h->v[j] + h->tn[j];"),
    "lam update sign": ("h->lam[j] += mu * (h->x1[j] - h->x2[j]);", "h->lam[j] -= mu * (h->x1[j] - h->x2[j]);"),
    "residual multiplier not scaled by mu": ("la[i] = h->mu * h->nu[i];", "la[i] = h->nu[i];"),
    "rhs drops b": ("for (int32_t i = 0; i < m; ++i) h->g[i] -= h->b[i];", ""),
    "Lorentz head sign": ("out[0] = 0.5 * (w1 + a);", "out[0] = 0.5 * (w1 - a);"),
    "Lorentz tail scale": ("const double s = 0.5 * (1.0 + w1 / a);", "const double s = 0.5 * (1.0 - w1 / a);"),
    "Lorentz case order": ("} else if (a <= w1) {", "} else if (a <= w1 + 1e-3) {"),
}


@pytest.mark.parametrize("name", sorted(STD_MUTANTS))
def test_standard_pins_catch_mutant(name, tmp_path):
    from oracle import standard
    old, new = STD_MUTANTS[name]
    text = open(STD_SRC).read()
    assert text.count(old) == 1, f"mutation site not unique: {old}"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = standard.build(src=str(src), out=str(tmp_path / "libmutant.so"))
    env = dict(os.environ, UVADMM_STD_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_standard_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
