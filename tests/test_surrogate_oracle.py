"""Pins of the FP64 surrogate twin (CPU): finite differences of its smooth
form, deep-sets invariances, closed forms of softplus/Adam, the BF16 rounding
helper on hand-checked values, and planted mistakes that the pins catch."""
import numpy as np
import pytest

from oracle import surrogate_oracle as SO

H = 6


def _batch(seed, pairs=3):
    r = np.random.default_rng(seed)
    sizes = r.integers(3, 8, size=2 * pairs)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    X = r.random((off[-1], 3))
    a = np.concatenate([r.dirichlet(np.ones(k)) for k in sizes])
    y = r.uniform(0.1, 0.6, size=pairs)
    return X, a, off, y


def _theta(seed, hidden=H):
    r = np.random.default_rng(seed)
    return r.normal(0.0, 0.6, SO.num_params(hidden))


def _fd_check(theta, X, a, off, y, hidden=H, h=1e-6):
    loss, g = SO.loss_and_grad(theta, X, a, off, y, hidden, rounding=False)
    fd = np.zeros_like(g)
    for k in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp, _ = SO.loss_and_grad(tp, X, a, off, y, hidden, rounding=False)
        lm, _ = SO.loss_and_grad(tm, X, a, off, y, hidden, rounding=False)
        fd[k] = (lp - lm) / (2 * h)
    return g, fd


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_finite_differences(seed):
    X, a, off, y = _batch(seed)
    th = _theta(10 + seed)
    g, fd = _fd_check(th, X, a, off, y)
    assert np.abs(g).max() > 1e-3
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_planted_sign_mistake_is_caught(monkeypatch):
    """Flip the sign of d|u|/du: the finite-difference pin must fail."""
    X, a, off, y = _batch(3)
    th = _theta(13)
    real_sign = np.sign
    monkeypatch.setattr(SO.np, "sign", lambda v: -real_sign(v))
    g, fd = _fd_check(th, X, a, off, y)
    monkeypatch.setattr(SO.np, "sign", real_sign)
    assert not np.allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_planted_sigmoid_mistake_is_caught(monkeypatch):
    X, a, off, y = _batch(4)
    th = _theta(14)
    real = SO.sigmoid
    monkeypatch.setattr(SO, "sigmoid", lambda t: 1.0 - real(t))
    g, fd = _fd_check(th, X, a, off, y)
    monkeypatch.setattr(SO, "sigmoid", real)
    assert not np.allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_pooling_is_a_set_function():
    """Permuting points leaves E unchanged; splitting a point into two copies
    carrying half its mass each also does; a zero-mass point adds nothing."""
    X, a, off, _ = _batch(5, pairs=1)
    th = _theta(15)
    E = SO.embed(th, X, a, off, H, rounding=False)
    lo, hi = off[0], off[1]
    perm = np.arange(len(a))
    perm[lo:hi] = lo + np.random.default_rng(0).permutation(hi - lo)
    np.testing.assert_allclose(SO.embed(th, X[perm], a[perm], off, H, rounding=False), E, rtol=1e-13)
    X2 = np.insert(X, lo, X[lo], axis=0)
    a2 = np.insert(a, lo, a[lo] / 2)
    a2[lo + 1] = a[lo] / 2
    off2 = off.copy()
    off2[1:] += 1
    np.testing.assert_allclose(SO.embed(th, X2, a2, off2, H, rounding=False), E, rtol=1e-13)
    X3 = np.insert(X, lo, [9.0, -3.0, 4.0], axis=0)
    a3 = np.insert(a, lo, 0.0)
    np.testing.assert_allclose(SO.embed(th, X3, a3, off2, H, rounding=False), E, rtol=1e-13)


def test_single_point_sets_reduce_to_the_mlp():
    """One point of mass 1 per set: E = phi(x), computed here by hand."""
    th = _theta(16)
    P = SO.unpack(th, H)
    x = np.array([[0.2, 0.7, 0.4], [0.9, 0.1, 0.5]])
    phi = np.maximum(P["W2"] @ np.maximum(P["W1"] @ x[0] + P["b1"], 0) + P["b2"], 0)
    E = SO.embed(th, x, np.ones(2), np.array([0, 1, 2]), H, rounding=False)
    np.testing.assert_allclose(E[0], phi, rtol=1e-14)
    phi1 = np.maximum(P["W2"] @ np.maximum(P["W1"] @ x[1] + P["b1"], 0) + P["b2"], 0)
    z = np.concatenate([phi, phi1, np.abs(phi - phi1)])
    t = P["w4"] @ np.maximum(P["W3"] @ z + P["b3"], 0) + P["b4"][0]
    pred = SO.head(th, E[0], E[1], H, rounding=False)[0]
    assert pred == pytest.approx(np.log(1 + np.exp(t)), rel=1e-14)
    assert pred > 0


def test_softplus_and_sigmoid_closed_forms():
    t = np.array([-30.0, -1.0, 0.0, 1.0, 19.0, 25.0])
    np.testing.assert_allclose(SO.softplus(t), [np.log1p(np.exp(-30.0)), np.log1p(np.exp(-1.0)), np.log(2.0),
                                                np.log1p(np.e), np.log1p(np.exp(19.0)), 25.0], rtol=1e-12)
    assert SO.sigmoid(0.0) == 0.5


def test_loss_is_zero_at_the_labels():
    X, a, off, _ = _batch(6)
    th = _theta(17)
    y = SO.predict(th, X, a, off, H, rounding=False)
    loss, g = SO.loss_and_grad(th, X, a, off, y, H, rounding=False)
    assert loss == pytest.approx(0.0, abs=1e-28)
    assert np.abs(g).max() < 1e-12


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    lr * g / (|g| + eps)."""
    r = np.random.default_rng(7)
    th, g = r.normal(size=50), r.normal(size=50)
    t1, m, v = SO.adam(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    np.testing.assert_allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_bf16_rounding_hand_values():
    one = 1.0
    ulp = 2.0 ** -7  # BF16 spacing in [1, 2)
    cases = [(one, one), (one + ulp / 2, one), (one + 3 * ulp / 2, one + 2 * ulp),
             (one + ulp / 2 + 2 ** -20, one + ulp), (-(one + 3 * ulp / 2), -(one + 2 * ulp)),
             (3.0, 3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130)]
    for x, want in cases:
        assert SO.bf16(np.array([x]))[0] == want, x


def test_topk_smallest_brute_force():
    r = np.random.default_rng(9)
    for _ in range(20):
        v = r.integers(0, 6, size=40).astype(np.float32)
        k = int(r.integers(1, 40))
        got = SO.topk_smallest(v, k)
        want = sorted(range(40), key=lambda i: (v[i], i))[:k]
        assert list(got) == want
