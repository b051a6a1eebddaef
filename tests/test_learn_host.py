"""CPU pins of the warm-start oracle (finite differences, BF16 rounding) and
of the library's host eigen-solver (against numpy's)."""
import numpy as np
import pytest

from oracle import mlp as M


def test_bf16_rounding_values():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-7, -2.5, 3.0e38, 1e-30, 0.0], dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -2.5, np.nan, np.nan, 0.0])
    got = M.bf16_round(x)
    np.testing.assert_array_equal(got[[0, 1, 2, 3, 4, 7]], want[[0, 1, 2, 3, 4, 7]])
    # every output is a BF16 value (low 16 bits zero) within half a BF16 ulp
    y = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    r = M.bf16_round(y).astype(np.float32)
    assert not (r.view(np.uint32) & 0xFFFF).any()
    assert (np.abs(r - y) <= np.abs(y) * 2.0**-8 * 1.0001).all()


def test_mlp_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    dims = [5, 7, 6, 3]
    ws = [rng.standard_normal((a, b)) * 0.5 for a, b in zip(dims[:-1], dims[1:])]
    bs = [rng.standard_normal(b) * 0.1 for b in dims[1:]]
    x = rng.standard_normal((4, 5))
    t = rng.standard_normal((4, 3))
    loss, gws, gbs = M.loss_and_grads(ws, bs, x, t)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (dims[l] - 1, dims[l + 1] - 1), (1, 2)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h
            wm[l][idx] -= h
            fd = (M.loss_and_grads(wp, bs, x, t)[0] - M.loss_and_grads(wm, bs, x, t)[0]) / (2 * h)
            assert fd == pytest.approx(gws[l][idx], rel=1e-5, abs=1e-9)
        for j in (0, dims[l + 1] - 1):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][j] += h
            bm[l][j] -= h
            fd = (M.loss_and_grads(ws, bp, x, t)[0] - M.loss_and_grads(ws, bm, x, t)[0]) / (2 * h)
            assert fd == pytest.approx(gbs[l][j], rel=1e-5, abs=1e-9)


def check_adam_first_step(mod):
    """With zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mod.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def check_adam_constant_gradient(mod):
    """A constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2
    (geometric sums), so the bias-corrected step is lr g / (|g| + eps) at
    EVERY step t, and after T steps p = p0 - T lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    p, m, v = np.ones(4), np.zeros(4), np.zeros(4)
    lr = 0.01
    for t in range(1, 41):
        p, m, v = mod.adam_step(p, g, m, v, t, lr=lr)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(p, 1 - t * lr * g / (np.abs(g) + 1e-8), rtol=1e-11)


def check_adam_alternating_gradient(mod):
    """g_t = (-1)^(t+1) g: m_t = (1 - b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1)
    (an alternating geometric sum) and v_t = (1 - b2^t) g^2, so the step at t
    is lr m_t / (1 - b1^t) / (|g| sqrt(1) + eps) with that m_t."""
    g = np.array([0.5, -1.5])
    b1, b2, lr, eps = 0.9, 0.999, 0.003, 1e-8
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    want = np.zeros(2)
    for t in range(1, 31):
        gt = g if t % 2 == 1 else -g
        p, m, v = mod.adam_step(p, gt, m, v, t, lr=lr)
        mt = (1 - b1) * g * (-1) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        np.testing.assert_allclose(m, mt, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12)
        want = want - lr * (mt / (1 - b1 ** t)) / (np.abs(g) + eps)
        np.testing.assert_allclose(p, want, rtol=1e-11)


ADAM_CHECKS = (check_adam_first_step, check_adam_constant_gradient, check_adam_alternating_gradient)


@pytest.mark.parametrize("check", ADAM_CHECKS, ids=lambda f: f.__name__)
def test_adam_pins(check):
    check(M)


ADAM_MUTANTS = {
    "no first-moment bias correction after step 1": ("mh = m / (1 - b1 ** step)", "mh = m / (1 - b1)"),
    "no second-moment bias correction after step 1": ("vh = v / (1 - b2 ** step)", "vh = v / (1 - b2)"),
    "first moment decays with b2": ("m = b1 * m + (1 - b1) * g", "m = b2 * m + (1 - b2) * g"),
    "second moment of |g|": ("v = b2 * v + (1 - b2) * g * g", "v = b2 * v + (1 - b2) * np.abs(g)"),
    "eps inside the sqrt": ("(np.sqrt(vh) + eps)", "np.sqrt(vh + eps)"),
    "ascent": ("return p - lr * mh", "return p + lr * mh"),
}


@pytest.mark.parametrize("name", sorted(ADAM_MUTANTS))
def test_adam_pins_catch_mutant(name):
    """A copy of the oracle module with one planted mistake in adam_step must
    fail at least one of the pins above."""
    import types
    old, new = ADAM_MUTANTS[name]
    src = open(M.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("mlp_mutant")
    exec(compile(src.replace(old, new), "mlp_mutant", "exec"), mod.__dict__)
    caught = 0
    for check in ADAM_CHECKS:
        try:
            check(mod)
        except AssertionError:
            caught += 1
    assert caught > 0, f"pins did not catch: {name}"


def test_host_jacobi_eigensolver_matches_numpy():
    from paper_2203_05027_amd import learn
    rng = np.random.default_rng(2)
    for l in (1, 5, 40):
        A = rng.standard_normal((l, l))
        S = A @ A.T + np.diag(rng.uniform(0, 1, l))
        w, V = learn.sym_eig(S)
        wn = np.linalg.eigvalsh(S)[::-1]
        np.testing.assert_allclose(w, wn, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(V.T @ V, np.eye(l), atol=1e-10)
        np.testing.assert_allclose(S @ V, V * w, atol=1e-9 * (1 + np.abs(w).max()))
