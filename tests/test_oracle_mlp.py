"""Pins of the FP64 MLP reference (oracle/mlp.py) against definitions that do not
go through its own code: GELU against x Phi(x) with the error function, the
backward pass against central differences of the loss, Adam's update against
its closed form for a constant gradient."""
import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp as R


def test_gelu_tanh_form_against_the_erf_definition():
    z = np.linspace(-6, 6, 1201)
    exact = 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))
    assert np.max(np.abs(R.gelu(z) - exact)) < 1e-3   # the tanh form's known approximation error
    assert R.gelu(np.array([0.0]))[0] == 0.0
    assert abs(R.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(R.gelu(np.array([-10.0]))[0]) < 1e-12


def test_gelu_grad_against_central_differences():
    z = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(R.gelu_grad(z) - fd)) < 1e-8
    assert abs(R.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    params = R.init_params(5, 7, 3, 2, rng)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    x = rng.standard_normal((9, 5))
    t = rng.standard_normal((9, 2))
    return params, x, t


def test_backward_against_central_differences():
    params, x, t = _tiny()
    y, cache = R.forward(params, x)
    grads = R.backward(params, cache, y, t)
    h = 1e-6
    worst = 0.0
    for l, (W, b) in enumerate(params):
        for k, P in enumerate((W, b)):
            G = grads[l][k]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                lp = R.loss(R.forward(params, x)[0], t)
                P[idx] = old - h
                lm = R.loss(R.forward(params, x)[0], t)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(G[idx] - fd) / max(1e-3, abs(fd)))
    assert worst < 1e-6


def test_a_dropped_term_in_backward_is_caught():
    """The finite-difference check above fails for a plausible mistake (gelu' dropped)."""
    params, x, t = _tiny(1)
    y, cache = R.forward(params, x)
    zs, hs = cache
    # gradient of the first layer's weights without the activation derivative
    n = y.shape[0]
    dy = 2.0 * (y - t) / (n * y.shape[1])
    dh = dy @ params[-1][0].T
    for l in range(len(params) - 2, 0, -1):
        dh = (dh * R.gelu_grad(zs[l])) @ params[l][0].T
    wrong = hs[0].T @ dh                      # gelu'(z_0) missing
    right = R.backward(params, cache, y, t)[0][0]
    assert np.max(np.abs(wrong - right)) > 1e-3


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2, so every step
    moves a parameter by lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    params = [(rng.standard_normal((3, 4)), rng.standard_normal(4))]
    grads = [(rng.standard_normal((3, 4)), rng.standard_normal(4))]
    opt = R.Adam(params, lr=0.01)
    p = params
    for _ in range(4):
        p = opt.step(p, grads)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, p, grads):
        assert np.allclose(W0 - W1, 4 * 0.01 * gW / (np.abs(gW) + 1e-8), rtol=1e-7, atol=1e-12)
        assert np.allclose(b0 - b1, 4 * 0.01 * gb / (np.abs(gb) + 1e-8), rtol=1e-7, atol=1e-12)


def test_training_reduces_the_loss():
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, size=(256, 4))
    t = np.sin(2 * x[:, :1]) + x[:, 1:2] * x[:, 2:3]
    params = R.init_params(4, 32, 2, 1, rng)
    opt = R.Adam(params, lr=3e-3)
    l0 = R.loss(R.forward(params, x)[0], t)
    for _ in range(300):
        y, cache = R.forward(params, x)
        params = opt.step(params, R.backward(params, cache, y, t))
    assert R.loss(R.forward(params, x)[0], t) < 0.1 * l0
