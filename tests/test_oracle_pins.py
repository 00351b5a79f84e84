"""Pins of the FP64 oracle against things other than itself (CPU only).

Each Hessian/Jacobian route of the oracle is checked against closed forms
written out by hand, central finite differences, hyper-dual brute force on
tiny networks, structural identities (symmetry, linearity in lambda, the
identity-activation special case) and the paper's printed structure counts.
The planted-mistake tests at the bottom show that these pins catch the
plausible errors (a dropped second-order term, a flipped sign, a dropped
sigma').
"""
import json
import os

import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen

pytestmark = []

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_structure.json")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- activations
@pytest.mark.parametrize("kind", ["tanh", "sigmoid", "softplus", "identity"])
def test_activation_derivatives_match_finite_differences(kind):
    z = np.linspace(-6, 6, 97)
    h = 1e-5
    v, d1, d2 = O.act(kind, z)
    vp, d1p, _ = O.act(kind, z + h)
    vm, d1m, _ = O.act(kind, z - h)
    assert np.max(np.abs((vp - vm) / (2 * h) - d1)) < 1e-9
    assert np.max(np.abs((d1p - d1m) / (2 * h) - d2)) < 1e-9


def test_activation_special_values():
    v, d1, d2 = O.act("tanh", 0.0)
    assert (v, d1, d2) == (0.0, 1.0, 0.0)
    v, d1, d2 = O.act("sigmoid", 0.0)
    assert (v, d1, d2) == (0.5, 0.25, 0.0)
    v, d1, d2 = O.act("softplus", 0.0)
    assert abs(v - np.log(2.0)) < 1e-16 and d1 == 0.5 and d2 == 0.25
    # saturation: finite, no NaN, limits reached
    for kind in ("tanh", "sigmoid", "softplus"):
        v, d1, d2 = O.act(kind, np.array([-800.0, 800.0]))
        assert np.all(np.isfinite(v)) and np.all(np.isfinite(d1)) and np.all(np.isfinite(d2))
        assert np.all(np.abs(d2) < 1e-300)
    assert O.act("softplus", 800.0)[0] == 800.0


@pytest.mark.parametrize("kind", ["tanh", "sigmoid", "softplus"])
def test_activation_matches_hyperdual_composition(kind):
    z = np.linspace(-4, 4, 33)
    hd = O._hd_act(kind, O._HD(z, np.ones_like(z), np.ones_like(z), np.zeros_like(z)))
    v, d1, d2 = O.act(kind, z)
    np.testing.assert_allclose(hd.a, v, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(hd.b, d1, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(hd.d, d2, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- forward / residual
def test_identity_network_is_affine_map():
    Ws, bs = datagen.tiny_net((5, 4, 3, 2), seed=1)
    acts = ["identity"] * 3
    x = np.arange(5.0) / 7.0
    expect = np.linalg.multi_dot([Ws[2], Ws[1], Ws[0], x]) + Ws[2] @ (Ws[1] @ bs[0] + bs[1]) + bs[2]
    np.testing.assert_allclose(O.nn(Ws, bs, acts, x), expect, rtol=1e-14)
    # and its Jacobian is the weight product, its Hessian exactly 0
    np.testing.assert_allclose(O.jacobian(Ws, bs, acts, x), np.linalg.multi_dot(Ws[::-1]), rtol=1e-14)
    assert np.all(O.hess_for(Ws, bs, acts, x, np.array([1.0, -2.0])) == 0.0)
    assert np.all(O.hess_layersum(Ws, bs, acts, x, np.array([1.0, -2.0])) == 0.0)


def test_residual_sign_and_batching():
    Ws, bs = datagen.tiny_net((6, 5, 3), seed=2)
    acts = ["tanh", "identity"]
    X = np.random.default_rng(0).random((4, 6))
    out = O.residual(Ws, bs, acts, X)
    assert out.shape == (4, 3)
    np.testing.assert_allclose(O.residual(Ws, bs, acts, X, np.zeros((4, 3))), -out)
    assert np.all(O.residual(Ws, bs, acts, X, out) == 0.0)


# ---------------------------------------------------------------- closed forms
def one_hidden_tanh(seed=3, n=7, h=5, m=3):
    Ws, bs = datagen.tiny_net((n, h, m), seed=seed)
    rng = np.random.default_rng(seed + 100)
    x = rng.random(n)
    lam = rng.standard_normal(m)
    return Ws, bs, x, lam


def test_jacobian_closed_form_one_hidden_tanh():
    (W1, W2), (b1, b2), x, _ = one_hidden_tanh()
    t = np.tanh(W1 @ x + b1)
    J_hand = W2 @ np.diag(1.0 - t * t) @ W1
    acts = ["tanh", "identity"]
    assert rel(O.jacobian([W1, W2], [b1, b2], acts, x), J_hand) < 1e-14
    assert rel(O.jacobian_reverse([W1, W2], [b1, b2], acts, x), J_hand) < 1e-14


def test_hessian_closed_form_one_hidden_tanh():
    (W1, W2), (b1, b2), x, lam = one_hidden_tanh()
    t = np.tanh(W1 @ x + b1)
    H_hand = W1.T @ np.diag((W2.T @ lam) * (-2.0 * t * (1.0 - t * t))) @ W1
    acts = ["tanh", "identity"]
    assert rel(O.hess_for([W1, W2], [b1, b2], acts, x, lam), H_hand) < 1e-13
    assert rel(O.hess_layersum([W1, W2], [b1, b2], acts, x, lam), H_hand) < 1e-13


@pytest.mark.parametrize("kind,d2", [
    ("tanh", lambda u: -2.0 * np.tanh(u) * (1.0 - np.tanh(u) ** 2)),
    ("sigmoid", lambda u: (lambda s: s * (1 - s) * (1 - 2 * s))(1.0 / (1.0 + np.exp(-u)))),
    ("softplus", lambda u: (lambda s: s * (1 - s))(1.0 / (1.0 + np.exp(-u)))),
])
def test_scalar_neuron_hessian(kind, d2):
    w1, b1, w2, b2, x, lam = 1.3, -0.4, -0.7, 0.2, 0.9, 1.7
    Ws = [np.array([[w1]]), np.array([[w2]])]
    bs = [np.array([b1]), np.array([b2])]
    H = O.hess_for(Ws, bs, [kind, "identity"], np.array([x]), np.array([lam]))
    assert abs(H[0, 0] - lam * w2 * w1 * w1 * d2(w1 * x + b1)) < 1e-15


# ---------------------------------------------------------------- finite differences
ACT_SETS = [
    ["tanh", "tanh", "identity"],
    ["sigmoid", "sigmoid", "identity"],
    ["softplus", "softplus", "identity"],
    ["tanh", "sigmoid", "tanh"],  # Eq. 3 literally: sigma on the output layer too
    ["tanh", "tanh", "softmax"],  # Table 1's classifiers: SoftMax output
    ["sigmoid", "softplus", "softmax"],
]


@pytest.mark.parametrize("acts", ACT_SETS)
def test_jacobian_and_gradient_vs_central_differences(acts):
    Ws, bs = datagen.tiny_net((9, 8, 6, 4), seed=4)
    rng = np.random.default_rng(5)
    x = rng.random(9)
    lam = rng.standard_normal(4)
    h = 1e-6
    J = O.jacobian(Ws, bs, acts, x)
    Jfd = np.stack([(O.nn(Ws, bs, acts, x + h * e) - O.nn(Ws, bs, acts, x - h * e)) / (2 * h)
                    for e in np.eye(9)], axis=1)
    assert rel(J, Jfd) < 1e-8
    grad = O.adjoint(Ws, bs, acts, x, lam)[1][0]
    assert rel(grad, J.T @ lam) < 1e-14


@pytest.mark.parametrize("acts", ACT_SETS)
def test_hessian_vs_central_differences_of_gradient(acts):
    Ws, bs = datagen.tiny_net((9, 8, 6, 4), seed=6)
    rng = np.random.default_rng(7)
    x = rng.random(9)
    lam = rng.standard_normal(4)
    h = 1e-5

    def grad(xx):
        return O.jacobian(Ws, bs, acts, xx).T @ lam

    Hfd = np.stack([(grad(x + h * e) - grad(x - h * e)) / (2 * h) for e in np.eye(9)], axis=1)
    assert rel(O.hess_for(Ws, bs, acts, x, lam), Hfd) < 1e-8


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("acts", ACT_SETS)
def test_hessian_matches_hyperdual_bruteforce(acts):
    Ws, bs = datagen.tiny_net((6, 5, 6, 3), seed=8)
    rng = np.random.default_rng(9)
    x = rng.random(6)
    lam = rng.standard_normal(3)
    Hb = O.hess_hyperdual(Ws, bs, acts, x, lam)
    assert rel(O.hess_for(Ws, bs, acts, x, lam), Hb) < 1e-12
    assert rel(O.hess_layersum(Ws, bs, acts, x, lam), Hb) < 1e-12
    assert rel(O.jacobian(Ws, bs, acts, x), O.jacobian_hyperdual(Ws, bs, acts, x)) < 1e-13


def test_hessian_of_unit_multiplier_is_output_hessian():
    acts = ["tanh", "softplus", "identity"]
    Ws, bs = datagen.tiny_net((5, 4, 4, 3), seed=10)
    x = np.random.default_rng(11).random(5)
    T = O.hess_tensor_hyperdual(Ws, bs, acts, x)
    for i in range(3):
        assert rel(O.hess_for(Ws, bs, acts, x, np.eye(3)[i]), T[i]) < 1e-12


# ---------------------------------------------------------------- structure
def test_symmetry_linearity_and_method_agreement_c1_size():
    Ws, bs = datagen.mlp_weights(datagen.C1_DIMS, seed=0)
    acts = ["tanh", "tanh", "identity"]
    X, Lam = datagen.points(784, 10, 2, seed=1001)
    x = X[0]
    H1 = O.hess_for(Ws, bs, acts, x, Lam[0])
    H2 = O.hess_for(Ws, bs, acts, x, Lam[1])
    Hs = O.hess_layersum(Ws, bs, acts, x, Lam[0])
    assert rel(Hs, Hs.T) < 1e-15  # layer-sum form is symmetric up to BLAS rounding order
    assert rel(H1, H1.T) < 1e-14
    assert rel(H1, Hs) < 1e-13
    H12 = O.hess_for(Ws, bs, acts, x, 2.0 * Lam[0] - 3.0 * Lam[1])
    assert rel(H12, 2.0 * H1 - 3.0 * H2) < 1e-13
    # objective term lands on the diagonal only
    q = np.arange(784.0)
    Hq = O.hess_lag(Ws, bs, acts, X[:1], Lam[:1], obj_factor=0.5, q=q)[0]
    np.testing.assert_allclose(Hq - H1, np.diag(0.5 * q), rtol=0, atol=1e-13)
    off = ~np.eye(784, dtype=bool)
    assert np.all(Hq[off] == H1[off])


def test_paper_structure_counts():
    g = json.load(open(GOLDEN))
    # Table 2: reduced-space Hess NNZ = lower triangle of the n x n Hessian
    for name, row in g["table2_reduced_space"].items():
        if name.startswith("_"):
            continue
        n = row["n_inputs"]
        nnz = n * (n + 1) // 2
        printed = float(row["hess_nnz_printed"].rstrip("k")) * 1000
        if name == "MNIST":
            assert (nnz // 1000) * 1000 == printed  # 307,720 printed truncated as "307k"
        else:  # SCOPF adds power-flow Hessian terms on top of the NN block
            assert nnz <= printed + 500
    # Table 1: parameter counts of the implied architectures
    scale = {"k": 1e3, "M": 1e6}
    for name, row in g["table1_params"].items():
        if name.startswith("_"):
            continue
        d = row["dims"]
        params = sum(d[i] * d[i + 1] + d[i + 1] for i in range(len(d) - 1))
        p = row["printed"]
        printed = float(p[:-1]) * scale[p[-1]]
        # the table truncates to whole units of its suffix (274.9M -> "274M")
        assert int(params // scale[p[-1]]) == int(p[:-1]), (name, params, printed)


def test_hvp_matches_full_hessian_columns():
    Ws, bs = datagen.mlp_weights(datagen.C1_DIMS, seed=0)
    acts = ["tanh", "tanh", "identity"]
    X, Lam = datagen.points(784, 10, 1, seed=1001)
    H = O.hess_layersum(Ws, bs, acts, X[0], Lam[0])
    cols = [3, 100, 783]
    V = np.eye(784)[:, cols]
    assert rel(O.hvp(Ws, bs, acts, X[0], Lam[0], V), H[:, cols]) < 1e-13


# ---------------------------------------------------------------- planted mistakes
def _mutated_act(mutation):
    orig = O.act

    def act(kind, z):
        v, d1, d2 = orig(kind, z)
        if mutation == "drop_d2":
            d2 = np.zeros_like(d2)
        elif mutation == "flip_d2":
            d2 = -d2
        elif mutation == "drop_d1":
            d1 = np.ones_like(d1)
        return v, d1, d2

    return act


@pytest.mark.parametrize("mutation", ["drop_d2", "flip_d2", "drop_d1"])
def test_pins_catch_planted_mistakes(monkeypatch, mutation):
    (W1, W2), (b1, b2), x, lam = one_hidden_tanh()
    t = np.tanh(W1 @ x + b1)
    H_hand = W1.T @ np.diag((W2.T @ lam) * (-2.0 * t * (1.0 - t * t))) @ W1
    J_hand = W2 @ np.diag(1.0 - t * t) @ W1
    monkeypatch.setattr(O, "act", _mutated_act(mutation))
    acts = ["tanh", "identity"]
    H = O.hess_for([W1, W2], [b1, b2], acts, x, lam)
    J = O.jacobian([W1, W2], [b1, b2], acts, x)
    assert rel(H, H_hand) > 1e-3 or rel(J, J_hand) > 1e-3


def test_pins_catch_transposed_operand(monkeypatch):
    Ws, bs = datagen.tiny_net((6, 6, 6, 3), seed=12)  # square hidden weights
    acts = ["tanh", "tanh", "identity"]
    x = np.random.default_rng(13).random(6)
    lam = np.array([0.3, -1.0, 0.5])
    Hb = O.hess_hyperdual(Ws, bs, acts, x, lam)
    bad = [Ws[0], Ws[1].T.copy(), Ws[2]]
    # a transposed hidden weight in the derivative sweeps shows up against brute force
    orig_forward = O.forward
    monkeypatch.setattr(O, "forward", lambda W_, b_, a_, xx: orig_forward(Ws, b_, a_, xx))
    assert rel(O.hess_for(bad, bs, acts, x, lam), Hb) > 1e-3


# ---------------------------------------------------------------- SoftMax output
def test_softmax_invariants():
    """Outputs sum to one, so 1^T J = 0 and lambda = 1 gives H = 0; adding a
    constant to lambda leaves H unchanged; NN is the normalised exponential."""
    acts = ["tanh", "sigmoid", "softmax"]
    Ws, bs = datagen.tiny_net((7, 6, 5, 4), seed=30)
    rng = np.random.default_rng(31)
    x = rng.random(7)
    lam = rng.standard_normal(4)
    z = Ws[2] @ O.forward(Ws, bs, acts, x)[1][1] + bs[2]
    assert rel(O.nn(Ws, bs, acts, x), np.exp(z) / np.sum(np.exp(z))) < 1e-15
    J = O.jacobian(Ws, bs, acts, x)
    assert np.max(np.abs(np.ones(4) @ J)) < 1e-15
    for method in (O.hess_for, O.hess_layersum):
        assert np.max(np.abs(method(Ws, bs, acts, x, np.ones(4)))) < 1e-15
        assert rel(method(Ws, bs, acts, x, lam + 2.5), method(Ws, bs, acts, x, lam)) < 1e-13


def test_two_class_softmax_is_sigmoid_of_the_difference():
    """softmax(z)_0 = sigmoid(z_0 - z_1): a two-output SoftMax net equals a
    one-output sigmoid net whose last layer is the difference of the two rows
    (value, Jacobian row, and the Hessian for lambda = (mu, 0))."""
    Ws, bs = datagen.tiny_net((6, 5, 2), seed=32)
    W2 = (Ws[1][0] - Ws[1][1])[None, :]
    b2 = np.array([bs[1][0] - bs[1][1]])
    x = np.random.default_rng(33).random(6)
    sm = ["tanh", "softmax"]
    sg = ["tanh", "sigmoid"]
    assert abs(O.nn(Ws, bs, sm, x)[0] - O.nn([Ws[0], W2], [bs[0], b2], sg, x)[0]) < 1e-15
    assert rel(O.jacobian(Ws, bs, sm, x)[0], O.jacobian([Ws[0], W2], [bs[0], b2], sg, x)[0]) < 1e-13
    H = O.hess_for(Ws, bs, sm, x, np.array([1.7, 0.0]))
    Hs = O.hess_for([Ws[0], W2], [bs[0], b2], sg, x, np.array([1.7]))
    assert rel(H, Hs) < 1e-12


def test_softmax_pins_catch_a_dropped_coupling(monkeypatch):
    """A SoftMax second derivative without its rank-two coupling terms (only
    diag(g)) fails the brute-force pin."""
    acts = ["tanh", "tanh", "softmax"]
    Ws, bs = datagen.tiny_net((6, 5, 6, 3), seed=34)
    rng = np.random.default_rng(35)
    x = rng.random(6)
    lam = rng.standard_normal(3)
    Hb = O.hess_hyperdual(Ws, bs, acts, x, lam)
    orig = O._second

    def diag_only(layer, abar):
        g, S = orig(layer, abar)
        return g, (np.diag(np.diag(S)) if S.ndim == 2 else S)

    monkeypatch.setattr(O, "_second", diag_only)
    assert rel(O.hess_for(Ws, bs, acts, x, lam), Hb) > 1e-3
    assert rel(O.hess_layersum(Ws, bs, acts, x, lam), Hb) > 1e-3
