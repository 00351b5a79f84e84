"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle's tests.

This module holds no arithmetic of the method (no activations, no derivatives):
it only draws weights, evaluation points, multipliers and blob images with
numpy's PCG64 generator, so that both sides can be fed identical arrays.

Workload recipe (stand-ins for the paper's trained networks and datasets,
which are not available here):

* weights: W_l ~ N(0, 1/fan_in) (variance 1/fan_in), biases 0, drawn layer by
  layer in row-major order from ``default_rng(seed)`` (seed 0 by default);
* points: x ~ U[0,1)^n, multipliers lambda ~ N(0,1)^m, from
  ``default_rng(1000 + config_id)``, x drawn before lambda;
* surrogate inputs (SCOPF-like, Section 4.2 of the paper): the first half of
  the inputs are generator set-points U[0,1], the second half loads
  N(1, 0.1^2);
* blob images (MNIST-shaped, Section 4.1): 28x28 images with 1-3 Gaussian
  bumps, clipped to [0,1] and flattened row-major;
* deep, narrow surrogate (the shape Table 1's largest SCOPF network implies:
  117 inputs, 38 hidden layers of 4000, 37 outputs): inputs within +-20 % of
  a nominal operating point of 1 per unit, U[0.8, 1.2]^117.
"""
from __future__ import annotations

import numpy as np

# Layer widths of the synthetic workloads (input ... output).
C1_DIMS = (784, 64, 64, 10)
C2_DIMS = (784, 4096, 8192, 8192, 4096, 10)
C3_DIMS = {
    "A": (120,) + (512,) * 4 + (4,),
    "B": (120,) + (1024,) * 6 + (4,),
    "C": (120,) + (2048,) * 8 + (4,),
}
C3_POINTS = {"A": 64, "B": 512, "C": 1024}
SCOPF_DIMS = (117,) + (4000,) * 38 + (37,)
WARM_DIMS = (794, 512, 512, 804)


def mlp_weights(dims, seed: int = 0, bias_scale: float = 0.0, dtype=np.float64):
    """Weights W_l of shape (d_l, d_{l-1}) with N(0, 1/d_{l-1}) entries, biases.

    Biases are zero unless ``bias_scale`` > 0, in which case they are drawn
    N(0, bias_scale^2) after all weights (used by tests that need b != 0).
    """
    rng = np.random.default_rng(seed)
    Ws = []
    for l in range(1, len(dims)):
        fan_in = dims[l - 1]
        W = rng.standard_normal((dims[l], fan_in))
        W *= 1.0 / np.sqrt(fan_in)
        Ws.append(np.ascontiguousarray(W, dtype=dtype))
    bs = []
    for l in range(1, len(dims)):
        if bias_scale > 0:
            bs.append(rng.standard_normal(dims[l]).astype(dtype) * bias_scale)
        else:
            bs.append(np.zeros(dims[l], dtype=dtype))
    return Ws, bs


def points(n: int, m: int, B: int, seed: int):
    """B points x ~ U[0,1)^n and multipliers lambda ~ N(0,1)^m (x drawn first)."""
    rng = np.random.default_rng(seed)
    x = rng.random((B, n))
    lam = rng.standard_normal((B, m))
    return x, lam


def surrogate_points(n: int, m: int, B: int, seed: int):
    """SCOPF-like inputs: first n//2 set-points U[0,1], rest loads N(1, 0.1^2)."""
    rng = np.random.default_rng(seed)
    h = n // 2
    x = np.empty((B, n))
    x[:, :h] = rng.random((B, h))
    x[:, h:] = 1.0 + 0.1 * rng.standard_normal((B, n - h))
    lam = rng.standard_normal((B, m))
    return x, lam


def scopf_points(B: int, seed: int, n: int = 117, m: int = 37):
    """Operating points x ~ U[0.8, 1.2]^n (+-20 % around 1 per unit) and
    multipliers lambda ~ N(0,1)^m (x drawn first)."""
    rng = np.random.default_rng(seed)
    x = 0.8 + 0.4 * rng.random((B, n))
    lam = rng.standard_normal((B, m))
    return x, lam


def blob_images(count: int, seed: int, side: int = 28):
    """``count`` synthetic 28x28 images of 1-3 Gaussian bumps, values in [0,1].

    Centers U[6,22]^2, widths U[1.5,3.5] px, amplitudes U[0.5,1] (positions
    and widths scale with side/28 for other sizes); the sum is clipped to
    [0,1] and flattened row-major to length side*side.
    """
    rng = np.random.default_rng(seed)
    sc = side / 28.0
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    out = np.zeros((count, side * side))
    for i in range(count):
        k = int(rng.integers(1, 4))
        img = np.zeros((side, side))
        for _ in range(k):
            cy, cx = rng.uniform(6.0 * sc, 22.0 * sc, size=2)
            w = rng.uniform(1.5, 3.5) * sc
            a = rng.uniform(0.5, 1.0)
            img += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * w * w))
        out[i] = np.clip(img, 0.0, 1.0).ravel()
    return out


def tiny_net(dims, seed: int, bias_scale: float = 0.3):
    """Small random network with nonzero biases, for brute-force pins."""
    return mlp_weights(dims, seed=seed, bias_scale=bias_scale)
