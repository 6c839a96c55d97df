"""CPU ORACLE for the learned index's model -- TEST INFRASTRUCTURE ONLY.

Float64 numpy.  Only tests import this module.

The learned index's final answer is pinned by ``oracle.search_lt`` (its
result must equal the plain definition exactly).  This module covers the
model arithmetic in between, written from the model's definition:

* input  z = (log2 x - log2 a[0]) / (log2 a[n-1] - log2 a[0])
* layer 1  h1_j = max(0, w1_j z + b1_j),                 j < 32
* layer 2  h2_k = max(0, b2_k + sum_j W2[k][j] h1_j),    k < 32
* output   p = b3 + sum_k w3_k h2_k
* loss     L = (1/n) sum_i (p(a_i) - i/(n-1))^2  (the table's CDF)

Parameter vector layout (1153 entries): w1[32], b1[32], W2[32][32] (row k =
weights into unit k), b2[32], w3[32], b3.

``loss_and_grad`` is back-propagation written out by hand; it is pinned in
``tests/test_oracle_learned.py`` by central finite differences of ``loss``
and by a network whose output is known in closed form.  The training
trajectory itself (Adam on the device, FP32, its own summation order) has
no oracle: parity unpinned; only its gradient is compared.
"""
from __future__ import annotations

import numpy as np

H = 32
OFF_W1, OFF_B1, OFF_W2 = 0, 32, 64
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (NPARAM,)
    return (p[OFF_W1:OFF_B1], p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(H, H),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def model_input(x, table):
    x = np.asarray(x, dtype=np.float64)
    u0, u1 = np.log2(table[0]), np.log2(table[-1])
    with np.errstate(divide="ignore", invalid="ignore"):
        return (np.log2(x) - u0) / (u1 - u0)


def forward(params, z):
    """p(z) for an array of inputs."""
    w1, b1, W2, b2, w3, b3 = unpack(params)
    z = np.asarray(z, dtype=np.float64)
    h1 = np.maximum(0.0, np.outer(z, w1) + b1)           # [m, 32]
    h2 = np.maximum(0.0, h1 @ W2.T + b2)                 # [m, 32]
    return h2 @ w3 + b3


def loss(params, table):
    n = table.shape[0]
    z = model_input(table, table)
    y = np.arange(n, dtype=np.float64) / (n - 1)
    r = forward(params, z) - y
    return float(np.mean(r * r))


def loss_and_grad(params, table):
    """(L, dL/dparams) by back-propagation (float64)."""
    w1, b1, W2, b2, w3, b3 = unpack(params)
    n = table.shape[0]
    z = model_input(table, table)
    y = np.arange(n, dtype=np.float64) / (n - 1)
    a1 = np.outer(z, w1) + b1
    h1 = np.maximum(0.0, a1)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(0.0, a2)
    p = h2 @ w3 + b3
    r = p - y
    L = float(np.mean(r * r))
    g = 2.0 * r / n                                      # dL/dp
    d2 = np.outer(g, w3) * (a2 > 0)                      # dL/da2
    d1 = (d2 @ W2) * (a1 > 0)                            # dL/da1
    grad = np.empty(NPARAM)
    grad[OFF_W1:OFF_B1] = d1.T @ z
    grad[OFF_B1:OFF_W2] = d1.sum(axis=0)
    grad[OFF_W2:OFF_B2] = (d2.T @ h1).reshape(-1)
    grad[OFF_B2:OFF_W3] = d2.sum(axis=0)
    grad[OFF_W3:OFF_B3] = h2.T @ g
    grad[OFF_B3] = g.sum()
    return L, grad


def grad_scale(params, table):
    """Per-parameter magnitude of the gradient's terms without cancellation:
    back-propagation with every factor replaced by its absolute value, i.e.
    sum_i |dL/dp_i| |dp_i/dparam| (an upper bound of each term's size).  A
    float32 evaluation of the gradient is accurate to a small multiple of
    float32 epsilon times this scale, however much the terms cancel."""
    w1, b1, W2, b2, w3, b3 = unpack(params)
    n = table.shape[0]
    z = model_input(table, table)
    y = np.arange(n, dtype=np.float64) / (n - 1)
    a1 = np.outer(z, w1) + b1
    h1 = np.maximum(0.0, a1)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(0.0, a2)
    p = h2 @ w3 + b3
    g = np.abs(2.0 * (p - y) / n)
    d2 = np.outer(g, np.abs(w3)) * (a2 > 0)
    d1 = (d2 @ np.abs(W2)) * (a1 > 0)
    s = np.empty(NPARAM)
    s[OFF_W1:OFF_B1] = d1.T @ np.abs(z)
    s[OFF_B1:OFF_W2] = d1.sum(axis=0)
    s[OFF_W2:OFF_B2] = (d2.T @ h1).reshape(-1)
    s[OFF_B2:OFF_W3] = d2.sum(axis=0)
    s[OFF_W3:OFF_B3] = h2.T @ g
    s[OFF_B3] = g.sum()
    return s
