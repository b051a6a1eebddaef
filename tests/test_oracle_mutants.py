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
    # the stopping test of Section V-B
    "r_prim normalised by ||b||": ("out[0] = sqrt(rp2) / (1.0 + sqrt(bb));", "out[0] = sqrt(rp2) / sqrt(bb);"),
    "r_prim drops the sqrt": ("out[0] = sqrt(rp2) / (1.0 + sqrt(bb));", "out[0] = rp2 / (1.0 + sqrt(bb));"),
    "r_dual normalised by 1+||c||^2": ("out[1] = sqrt(rd2) / (1.0 + sqrt(cc));", "out[1] = sqrt(rd2) / (1.0 + cc);"),
    "gap denominator of the sum": ("out[2] = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));",
                                   "out[2] = fabs(cz + bl) / (1.0 + fabs(cz + bl));"),
    "gap sign of b'lambda": ("out[2] = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));",
                             "out[2] = fabs(cz - bl) / (1.0 + fabs(cz) + fabs(bl));"),
    "kkt ignores the gap": ("out[3] = fmax(out[0], fmax(out[1], out[2]));", "out[3] = fmax(out[0], out[1]);"),
    "dual residual sign of A'lambda": ("double r = atl + h->c[j] - h->delta[j];",
                                       "double r = -atl + h->c[j] - h->delta[j];"),
    "printed residual at z": ("ax += h->ak[k] * h->x[h->ck[k]];", "ax += h->ak[k] * h->z[h->ck[k]];"),
    "dual objective sign": ("out[5] = -bl;", "out[5] = bl;"),
    # the objective at x of the POGS-form test (Section V-A2)
    "objective at x takes z": ("cx += h->c[j] * h->x[j];", "cx += h->c[j] * h->z[j];"),
}
PIN_FILES = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_pins.py", "test_oracle_residual_pins.py")]


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
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
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
