"""Pins of the warm-start MLP oracle (backprop, MSE, Adam) — CPU only."""
import numpy as np

from oracle import mlp as M
from paper_2509_22462_amd import datagen


def test_backprop_matches_central_differences():
    Ws, bs = datagen.tiny_net((5, 7, 6, 4), seed=20)
    acts = ["tanh", "tanh", "identity"]
    rng = np.random.default_rng(21)
    X = rng.random((8, 5))
    Y = rng.standard_normal((8, 4))
    _, gW, gb = M.grads(Ws, bs, acts, X, Y)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (1, 2), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (M.loss(Wp, bs, acts, X, Y) - M.loss(Wm, bs, acts, X, Y)) / (2 * h)
            assert abs(fd - gW[l][idx]) < 1e-8 * max(1.0, abs(fd))
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += h
        bm[l][1] -= h
        fd = (M.loss(Ws, bp, acts, X, Y) - M.loss(Ws, bm, acts, X, Y)) / (2 * h)
        assert abs(fd - gb[l][1]) < 1e-8 * max(1.0, abs(fd))


def test_least_squares_optimum_has_zero_gradient():
    # one identity layer: the MSE minimiser is the least-squares solution
    rng = np.random.default_rng(22)
    X = rng.standard_normal((40, 6))
    Y = rng.standard_normal((40, 3))
    Xa = np.hstack([X, np.ones((40, 1))])
    sol = np.linalg.lstsq(Xa, Y, rcond=None)[0]
    W = sol[:6].T.copy()
    b = sol[6].copy()
    _, gW, gb = M.grads([W], [b], ["identity"], X, Y)
    assert np.max(np.abs(gW[0])) < 1e-13 and np.max(np.abs(gb[0])) < 1e-13


def test_adam_first_step_is_signed_lr():
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    M.adam_step(p, g, m, v, t=1, lr=0.01, eps=1e-8)
    expect = np.array([1.0, -2.0, 0.5]) - 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    np.testing.assert_allclose(p[0], expect, rtol=1e-15)


def test_adam_training_reduces_loss():
    Ws, bs = datagen.tiny_net((4, 16, 2), seed=23)
    acts = ["tanh", "identity"]
    rng = np.random.default_rng(24)
    X = rng.random((64, 4))
    Y = np.stack([np.sin(X.sum(1)), X[:, 0] * X[:, 1]], axis=1)
    params = Ws + bs
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    l0 = M.loss(Ws, bs, acts, X, Y)
    for t in range(1, 201):
        _, gW, gb = M.grads(Ws, bs, acts, X, Y)
        M.adam_step(params, gW + gb, m, v, t, lr=1e-2)
    assert M.loss(Ws, bs, acts, X, Y) < 0.2 * l0


# ---------------------------------------------------------------- Adam beyond the first step
def _adam_constant_gradient_ok(step_fn, steps=12):
    """With the same gradient g at every step, both moments equal g and g^2
    once bias-corrected (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so every
    step moves each parameter by exactly lr * g / (|g| + eps)."""
    g = np.array([0.3, -4.0, 2.5e-2, 7.0])
    p0 = np.array([1.0, -2.0, 0.5, 0.0])
    lr, eps = 0.01, 1e-8
    p, m, v = [p0.copy()], [np.zeros(4)], [np.zeros(4)]
    for t in range(1, steps + 1):
        step_fn(p, [g], m, v, t, lr=lr, eps=eps)
        expect = p0 - t * lr * g / (np.abs(g) + eps)
        if not np.allclose(p[0], expect, rtol=1e-13, atol=1e-15):
            return False
    return True


# Hand-derived three-step sequence for one scalar parameter starting at 0:
# gradients 1, -2, 0.5; lr 0.1, b1 0.9, b2 0.999, eps 0.  Exact decimal
# arithmetic of the update rule gives
#   t=1: m=0.1,    v=0.001,     m^=1,           v^=1                -> p=-0.1
#   t=2: m=-0.11,  v=0.004999,  m^=-0.11/0.19,  v^=0.004999/0.001999 -> p=-0.0633896472964154434717734569
#   t=3: m=-0.049, v=0.005244001, m^=-0.049/0.271, v^=0.005244001/0.002997001 -> p=-0.0497205809913329818449617629
ADAM_SEQUENCE = [(1.0, -0.1), (-2.0, -0.0633896472964154434717734569), (0.5, -0.0497205809913329818449617629)]


def _adam_sequence_ok(step_fn):
    p, m, v = [np.zeros(1)], [np.zeros(1)], [np.zeros(1)]
    for t, (g, expect) in enumerate(ADAM_SEQUENCE, start=1):
        step_fn(p, [np.array([g])], m, v, t, lr=0.1, b1=0.9, b2=0.999, eps=0.0)
        if abs(p[0][0] - expect) > 1e-15:
            return False
    return True


def test_adam_constant_gradient_moves_lr_per_step():
    assert _adam_constant_gradient_ok(M.adam_step)


def test_adam_hand_computed_sequence():
    assert _adam_sequence_ok(M.adam_step)


def test_adam_without_momentum_is_normalised_sgd():
    """b1 = b2 = 0: m = g, v = g^2 at every step (no bias correction left),
    so each step is lr * g / (|g| + eps) whatever the gradient history."""
    rng = np.random.default_rng(25)
    p = [rng.standard_normal(6)]
    m, v = [np.zeros(6)], [np.zeros(6)]
    for t in range(1, 6):
        g = rng.standard_normal(6)
        before = p[0].copy()
        M.adam_step(p, [g], m, v, t, lr=0.05, b1=0.0, b2=0.0, eps=1e-8)
        np.testing.assert_allclose(p[0], before - 0.05 * g / (np.abs(g) + 1e-8), rtol=1e-14)


def _adam_variant(mistake):
    """adam_step with one plausible mistake planted (for the pins above)."""
    def step(params, grads_, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        for p, g, mi, vi in zip(params, grads_, m, v):
            if mistake != "no_m_decay":
                mi *= b1
            mi += (1.0 - b1) * g
            vi *= b2
            vi += (1.0 - b2) * g * g
            tc = 1 if mistake == "bias_t1" else t
            mhat = mi / (1.0 - b1 ** tc)
            vhat = vi / (1.0 - b2 ** (tc + 1 if mistake == "b2_power" else tc))
            p -= lr * mhat / (np.sqrt(vhat) + eps)
    return step


def test_adam_pins_catch_planted_mistakes():
    for mistake in ("bias_t1", "no_m_decay", "b2_power"):
        bad = _adam_variant(mistake)
        assert not (_adam_constant_gradient_ok(bad) and _adam_sequence_ok(bad)), mistake
    assert _adam_constant_gradient_ok(_adam_variant("none")) and _adam_sequence_ok(_adam_variant("none"))
