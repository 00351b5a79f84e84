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
