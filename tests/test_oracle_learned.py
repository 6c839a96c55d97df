"""Pins the float64 oracle of the learned index's model (no GPU)."""
import numpy as np

from oracle import learned as L


def random_params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.5, L.NPARAM)
    p[L.OFF_B2:L.OFF_W3] = 0.3          # keep most layer-2 units active
    return p


def test_closed_form_network(inputs_mod):
    """w1 = e0, W2 = e1 e0^T, w3 = e1, biases 0: p(z) = max(0, z)."""
    p = np.zeros(L.NPARAM)
    p[L.OFF_W1 + 0] = 1.0
    p[L.OFF_W2 + L.H * 1 + 0] = 1.0      # row k=1, column j=0
    p[L.OFF_W3 + 1] = 1.0
    z = np.array([-0.5, 0.0, 0.25, 0.5, 1.0])
    assert np.array_equal(L.forward(p, z), np.maximum(z, 0.0))
    # exactly log-spaced table: z_i = i/(n-1), so the identity has zero loss
    n = 97
    table = 2.0 ** np.linspace(-10.0, 20.0, n)
    assert L.loss(p, table) < 1e-24
    # transposing W2 (a plausible layout mistake) changes the output
    q = p.copy()
    q[L.OFF_W2:L.OFF_B2] = p[L.OFF_W2:L.OFF_B2].reshape(L.H, L.H).T.reshape(-1)
    assert np.all(L.forward(q, z[2:]) == 0.0)


def test_gradient_matches_finite_differences(inputs_mod):
    table = inputs_mod.single_table(300)
    for seed in (1, 2):
        p = random_params(seed)
        loss, grad = L.loss_and_grad(p, table)
        assert abs(loss - L.loss(p, table)) <= 1e-12 * max(1.0, loss)
        h = 1e-6
        idx = np.concatenate([np.arange(0, 64, 5), np.arange(64, L.OFF_B2, 97),
                              np.arange(L.OFF_B2, L.NPARAM, 3)])
        for i in idx:
            e = np.zeros(L.NPARAM)
            e[i] = h
            fd = (L.loss(p + e, table) - L.loss(p - e, table)) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 + 1e-4 * abs(fd), (seed, i, fd, grad[i])


def test_input_normalisation(inputs_mod):
    table = inputs_mod.single_table(1000)
    z = L.model_input(table, table)
    assert z[0] == 0.0 and abs(z[-1] - 1.0) < 1e-15 and np.all(np.diff(z) >= 0)


# ---------------------------------------------------------------------------
# grad_scale (the tolerance of the device-gradient parity test): the size of
# each gradient's terms without cancellation.

def test_grad_scale_equals_gradient_without_cancellation(inputs_mod):
    """All weights and biases non-negative and the output above every target
    (b3 = 2 > 1 >= i/(n-1)): every term of every gradient sum is
    non-negative, so the terms' magnitudes sum to the gradient itself."""
    table = inputs_mod.single_table(300)
    rng = np.random.default_rng(4)
    p = np.abs(rng.normal(0.0, 0.5, L.NPARAM))
    p[L.OFF_B3] = 2.0
    _, grad = L.loss_and_grad(p, table)
    assert np.all(grad >= 0.0)
    assert np.array_equal(L.grad_scale(p, table), grad)


def test_grad_scale_hand_computed():
    """n = 3, table [1, 2, 4] (z = 0, 1/2, 1; targets 0, 1/2, 1), one active
    unit per layer: w1_0 = 1, b1_0 = 1/2, W2[0][0] = -2, b2_0 = 3,
    w3_0 = -1, b3 = 3/2.  Outputs -1/2, 1/2, 3/2; residuals -1/2, 0, 1/2;
    the second layer's unit is off at z = 1.  The b3 gradient cancels to 0;
    its scale is 2/3."""
    table = np.array([1.0, 2.0, 4.0])
    p = np.zeros(L.NPARAM)
    p[L.OFF_W1] = 1.0
    p[L.OFF_B1] = 0.5
    p[L.OFF_W2] = -2.0
    p[L.OFF_B2] = 3.0
    p[L.OFF_W3] = -1.0
    p[L.OFF_B3] = 1.5
    want = np.zeros(L.NPARAM)
    want[L.OFF_B1] = 2.0 / 3.0
    want[L.OFF_W2] = 1.0 / 6.0
    want[L.OFF_B2] = 1.0 / 3.0
    want[L.OFF_W3] = 2.0 / 3.0
    want[L.OFF_B3] = 2.0 / 3.0
    s = L.grad_scale(p, table)
    assert np.allclose(s, want, rtol=4 * np.finfo(float).eps, atol=0.0)
    _, grad = L.loss_and_grad(p, table)
    assert grad[L.OFF_B3] == 0.0 and abs(grad[L.OFF_W3] + 2.0 / 3.0) < 1e-15


def test_grad_scale_bounds_the_gradient(inputs_mod):
    table = inputs_mod.single_table(300)
    for seed in (1, 2, 3):
        p = random_params(seed)
        _, grad = L.loss_and_grad(p, table)
        s = L.grad_scale(p, table)
        assert np.all(np.abs(grad) <= s * (1 + 1e-12) + 1e-300)
