"""FP64 oracle for the network constraint y = NN(x) and its derivatives.

TEST INFRASTRUCTURE ONLY (see the package docstring). numpy float64 throughout.

Notation (Section 3, Eq. 3): layers l = 1..L, z_l = W_l a_{l-1} + b_l,
a_l = sigma_l(z_l), a_0 = x, NN(x) = a_L.  W_l has shape (d_l, d_{l-1}).
``acts`` lists sigma_1..sigma_L by name: "identity", "tanh", "sigmoid",
"softplus", and for the output layer only "softmax" (the classifiers of
Table 1 end in SoftMax).  The paper applies sigma_L at the output too (Eq. 3);
passing "identity" as the last activation gives the logits reading used by the
synthetic workloads — all are supported.

SoftMax is not elementwise: p = softmax(z) has the layer Jacobian
dp/dz = diag(p) - p p^T, and for a fixed vector u the scalar u^T p(z) has
gradient g = p * (u - p^T u) and Hessian diag(g) - p g^T - g p^T in z.  Where
the elementwise layers carry vectors sigma', sigma'' the SoftMax layer carries
these matrices.

Readings of the paper used here:
* g(x, y) = y - NN(x) (Section 3.2.1); with no y the residual is NN(x) itself.
* The Hessian returned is obj_factor * diag(q) + sum_i lambda_i Hess NN_i(x):
  the "+NN" quantity of Section 3.2.1 (Eq. 6 with an objective factor, the
  IPOPT form); a driver whose constraint is y - NN(x) passes -lambda.
* The three Hessian methods:
    1. ``hess_for``     — forward-over-reverse: reverse sweep of the scalar
                          lambda^T NN(x) (the "linear layer" trick of Section
                          3.2.1), differentiated forward along n seeds;
    2. ``hess_layersum``— closed form sum_l T_l^T diag(s_l) T_l, which follows
                          because each z_l is affine in a_{l-1};
    3. ``hess_hyperdual``— brute force for tiny nets: the full m x n x n tensor
                          Hess NN by hyper-dual arithmetic built from exp, log
                          and reciprocal only, contracted with lambda (the naive
                          O(m n^2) route the paper describes and avoids).
"""
from __future__ import annotations

import numpy as np

ACTS = ("identity", "tanh", "sigmoid", "softplus", "softmax")


# ----------------------------------------------------------------------------
# Activations sigma, sigma', sigma'' (Section 2 requires C^2 activations;
# Section 4 uses tanh and sigmoid; softplus is the third smooth choice).
# Derivatives are written in hyperbolic-cosine form.
# ----------------------------------------------------------------------------
def act(kind: str, z):
    """Return (sigma(z), sigma'(z), sigma''(z)) elementwise in float64."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(over="ignore"):
        if kind == "identity":
            return z.copy(), np.ones_like(z), np.zeros_like(z)
        if kind == "tanh":
            c = np.cosh(z)
            sech2 = 1.0 / (c * c)
            t = np.tanh(z)
            return t, sech2, -2.0 * t * sech2
        if kind == "sigmoid":
            h = np.cosh(0.5 * z)
            q = 0.25 / (h * h)  # sigmoid'(z) = 1 / (4 cosh^2(z/2))
            v = 0.5 * (1.0 + np.tanh(0.5 * z))
            return v, q, -np.tanh(0.5 * z) * q
        if kind == "softplus":
            h = np.cosh(0.5 * z)
            v = np.logaddexp(0.0, z)  # log(1 + e^z), exact, no threshold
            d1 = 0.5 * (1.0 + np.tanh(0.5 * z))
            return v, d1, 0.25 / (h * h)
    raise ValueError(f"unknown activation {kind!r}")


def softmax(z):
    """p_i = exp(z_i) / sum_j exp(z_j) (shifted by max z, which cancels)."""
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(z - np.max(z))
    return e / np.sum(e)


def _check(Ws, bs, acts):
    L = len(Ws)
    if len(bs) != L or len(acts) != L:
        raise ValueError("Ws, bs and acts must have one entry per layer")
    if "softmax" in acts[:-1]:
        raise ValueError("softmax is supported on the output layer only")
    for l in range(1, L):
        if Ws[l].shape[1] != Ws[l - 1].shape[0]:
            raise ValueError(f"layer {l + 1} input width mismatch")


# ----------------------------------------------------------------------------
# Forward pass (Eq. 3) and residual (Eq. 5, g = y - NN(x)).
# ----------------------------------------------------------------------------
def forward(Ws, bs, acts, x):
    """Per-layer (z_l, sigma(z_l), sigma'(z_l), sigma''(z_l)) for one point x.

    For a SoftMax output layer the third entry is the matrix dp/dz =
    diag(p) - p p^T and the fourth is None (its second derivative depends on
    the multiplier; see ``_second``)."""
    _check(Ws, bs, acts)
    a = np.asarray(x, dtype=np.float64)
    out = []
    for W, b, kind in zip(Ws, bs, acts):
        z = W @ a + b
        if kind == "softmax":
            p = softmax(z)
            out.append((z, p, np.diag(p) - np.outer(p, p), None))
            a = p
            continue
        v, d1, d2 = act(kind, z)
        out.append((z, v, d1, d2))
        a = v
    return out


def _apply_d1(d1, M):
    """D_l M: a row scaling for elementwise layers, dp/dz @ M for SoftMax."""
    return d1 @ M if d1.ndim == 2 else d1[:, None] * M


def _second(layer, abar):
    """(zbar, S): zbar = d(abar^T a_l)/dz_l and S its derivative in z_l --
    diag(abar * sigma'') (a vector, the diagonal) for elementwise layers, the
    full matrix diag(g) - p g^T - g p^T with g = p * (abar - p^T abar) for
    SoftMax."""
    z, v, d1, d2 = layer
    if d1.ndim == 2:
        g = v * (abar - v @ abar)
        return g, np.diag(g) - np.outer(v, g) - np.outer(g, v)
    return abar * d1, abar * d2


def nn(Ws, bs, acts, x):
    """NN(x) for one point (Eq. 3 / Eq. 5)."""
    return forward(Ws, bs, acts, x)[-1][1]


def residual(Ws, bs, acts, X, Y=None):
    """g = Y - NN(X) row by row, or NN(X) when Y is None.  X: (B, n)."""
    X = np.atleast_2d(X)
    out = np.stack([nn(Ws, bs, acts, x) for x in X])
    return out if Y is None else np.atleast_2d(Y) - out


# ----------------------------------------------------------------------------
# Jacobian dNN/dx: the chain-rule product D_L W_L ... D_1 W_1 (two orders).
# ----------------------------------------------------------------------------
def jacobian(Ws, bs, acts, x):
    """J = D_L W_L D_{L-1} W_{L-1} ... D_1 W_1, built right to left (n seeds)."""
    layers = forward(Ws, bs, acts, x)
    M = np.eye(Ws[0].shape[1])
    for W, (_, _, d1, _) in zip(Ws, layers):
        M = _apply_d1(d1, W @ M)
    return M


def jacobian_reverse(Ws, bs, acts, x):
    """The same product built left to right (m reverse passes)."""
    layers = forward(Ws, bs, acts, x)
    R = np.eye(Ws[-1].shape[0])
    for W, (_, _, d1, _) in zip(reversed(Ws), reversed(layers)):
        R = ((R @ d1) if d1.ndim == 2 else (R * d1[None, :])) @ W
    return R


def jacobians(Ws, bs, acts, X):
    """Stacked J for each row of X: shape (B, m, n)."""
    return np.stack([jacobian(Ws, bs, acts, x) for x in np.atleast_2d(X)])


# ----------------------------------------------------------------------------
# Hessian of lambda^T NN(x)  (Section 3.2.1, Eq. 6).
# ----------------------------------------------------------------------------
def adjoint(Ws, bs, acts, x, lam):
    """Reverse sweep of phi(x) = lambda^T NN(x).

    Returns (layers, abar, s) with abar[l] = d phi / d a_l for l = 0..L and
    s[l] = abar[l] * sigma_l''(z_l) for l = 1..L (s[0] unused; a matrix for a
    SoftMax output layer, see ``_second``).  abar[0] is the gradient of phi.
    """
    layers = forward(Ws, bs, acts, x)
    L = len(Ws)
    abar = [None] * (L + 1)
    s = [None] * (L + 1)
    abar[L] = np.asarray(lam, dtype=np.float64)
    for l in range(L, 0, -1):
        zbar, s[l] = _second(layers[l - 1], abar[l])
        abar[l - 1] = Ws[l - 1].T @ zbar
    return layers, abar, s


def _apply_s(sl, T):
    """diag(s_l) T (vector s_l) or S_l T (SoftMax matrix)."""
    return sl @ T if sl.ndim == 2 else sl[:, None] * T


def hvp(Ws, bs, acts, x, lam, V):
    """Forward-over-reverse product Hess(lambda^T NN)(x) @ V for V of shape (n, k).

    Forward tangents T_l = dz_l/dx . V; reverse tangents G_l (of zbar_l) and
    E_l (of abar_l): E_L = 0 because abar_L = lambda is constant,
    G_l = D_l E_l + diag(s_l) T_l, E_{l-1} = W_l^T G_l, result E_0.
    """
    layers, abar, s = adjoint(Ws, bs, acts, x, lam)
    L = len(Ws)
    V = np.asarray(V, dtype=np.float64)
    T = [None] * (L + 1)
    P = V
    for l in range(1, L + 1):
        T[l] = Ws[l - 1] @ P
        P = _apply_d1(layers[l - 1][2], T[l])
    E = np.zeros((Ws[-1].shape[0], V.shape[1]))
    for l in range(L, 0, -1):
        G = _apply_d1(layers[l - 1][2], E) + _apply_s(s[l], T[l])
        E = Ws[l - 1].T @ G
    return E


def hess_for(Ws, bs, acts, x, lam):
    """Method 1: forward-over-reverse with the n unit seeds (V = I_n)."""
    n = Ws[0].shape[1]
    return hvp(Ws, bs, acts, x, lam, np.eye(n))


def hess_layersum(Ws, bs, acts, x, lam):
    """Method 2: H = sum_l T_l^T diag(s_l) T_l with T_l = dz_l/dx."""
    layers, abar, s = adjoint(Ws, bs, acts, x, lam)
    n = Ws[0].shape[1]
    H = np.zeros((n, n))
    T = Ws[0].copy()
    for l in range(1, len(Ws) + 1):
        if l > 1:
            T = Ws[l - 1] @ _apply_d1(layers[l - 2][2], T)
        H += T.T @ _apply_s(s[l], T)
    return H


def hess_lag(Ws, bs, acts, X, Lam, obj_factor=0.0, q=None, method="for"):
    """obj_factor * diag(q) + sum_i lambda_i Hess NN_i(x) for each row of X.

    Returns shape (B, n, n).  ``method`` is "for" or "layersum".
    """
    fn = hess_for if method == "for" else hess_layersum
    X = np.atleast_2d(X)
    Lam = np.atleast_2d(Lam)
    out = []
    for x, lam in zip(X, Lam):
        H = fn(Ws, bs, acts, x, lam)
        if q is not None and obj_factor != 0.0:
            H = H + obj_factor * np.diag(np.asarray(q, dtype=np.float64))
        out.append(H)
    return np.stack(out)


# ----------------------------------------------------------------------------
# Method 3: hyper-dual brute force (tiny networks only).
# A hyper-dual number a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0 carries
# the second mixed partial in d.  Only +, *, exp, log and 1/x are given rules;
# the activations are composed from them, so sigma' and sigma'' are never
# written out here.
# ----------------------------------------------------------------------------
class _HD:
    __slots__ = ("a", "b", "c", "d")

    def __init__(self, a, b, c, d):
        self.a, self.b, self.c, self.d = a, b, c, d

    def __add__(self, o):
        if isinstance(o, _HD):
            return _HD(self.a + o.a, self.b + o.b, self.c + o.c, self.d + o.d)
        return _HD(self.a + o, self.b, self.c, self.d)

    __radd__ = __add__

    def __mul__(self, o):
        if isinstance(o, _HD):
            return _HD(self.a * o.a, self.a * o.b + self.b * o.a,
                       self.a * o.c + self.c * o.a,
                       self.a * o.d + self.b * o.c + self.c * o.b + self.d * o.a)
        return _HD(self.a * o, self.b * o, self.c * o, self.d * o)

    __rmul__ = __mul__

    def neg(self):
        return self * -1.0

    def exp(self):
        e = np.exp(self.a)
        return _HD(e, e * self.b, e * self.c, e * (self.d + self.b * self.c))

    def log(self):
        r = 1.0 / self.a
        return _HD(np.log(self.a), r * self.b, r * self.c,
                   r * self.d - r * r * self.b * self.c)

    def recip(self):
        r = 1.0 / self.a
        return _HD(r, -r * r * self.b, -r * r * self.c,
                   -r * r * self.d + 2.0 * r * r * r * self.b * self.c)

    def matvec(self, W):
        return _HD(W @ self.a, W @ self.b, W @ self.c, W @ self.d)

    def total(self):
        return _HD(np.sum(self.a), np.sum(self.b), np.sum(self.c), np.sum(self.d))


def _hd_act(kind, z: _HD) -> _HD:
    if kind == "identity":
        return z
    if kind == "tanh":  # 1 - 2 / (exp(2z) + 1)
        return (((z * 2.0).exp() + 1.0).recip() * -2.0) + 1.0
    if kind == "sigmoid":  # 1 / (1 + exp(-z))
        return (z.neg().exp() + 1.0).recip()
    if kind == "softplus":  # log(1 + exp(z))
        return (z.exp() + 1.0).log()
    if kind == "softmax":  # exp(z_i) * (1 / sum_j exp(z_j))
        e = z.exp()
        return e * e.total().recip()
    raise ValueError(kind)


def hess_tensor_hyperdual(Ws, bs, acts, x):
    """Full tensor d^2 NN_i / dx_j dx_k, shape (m, n, n), by hyper-dual passes."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    m = Ws[-1].shape[0]
    Htens = np.zeros((m, n, n))
    for j in range(n):
        for k in range(j, n):
            e_j = np.zeros(n)
            e_j[j] = 1.0
            e_k = np.zeros(n)
            e_k[k] = 1.0
            a = _HD(x.copy(), e_j, e_k, np.zeros(n))
            for W, b, kind in zip(Ws, bs, acts):
                a = _hd_act(kind, a.matvec(W) + b)
            Htens[:, j, k] = a.d
            Htens[:, k, j] = a.d
    return Htens


def hess_hyperdual(Ws, bs, acts, x, lam):
    """Method 3: contract the brute-force tensor with lambda over the output index."""
    return np.tensordot(np.asarray(lam, dtype=np.float64),
                        hess_tensor_hyperdual(Ws, bs, acts, x), axes=1)


def jacobian_hyperdual(Ws, bs, acts, x):
    """J from the e1 part of hyper-dual passes (one per input)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        a = _HD(x.copy(), e, np.zeros(n), np.zeros(n))
        for W, b, kind in zip(Ws, bs, acts):
            a = _hd_act(kind, a.matvec(W) + b)
        cols.append(a.b)
    return np.stack(cols, axis=1)
