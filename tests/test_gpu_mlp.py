"""GPU parity of the library's BF16 matrix-core MLP (C ABI gplmm_mlp_*) against
the FP64 reference in oracle/mlp.py.

Tolerances: BF16 operands carry 8 significant bits (relative rounding 2^-9),
accumulation is FP32; through four products of width <= 128 the relative L2
error of the output and of the gradients stays near 1e-2, so the bounds are
3e-2 (forward) and 5e-2 (gradients).  The Adam step is FP32 arithmetic on the
GPU's own gradient and is compared with its closed form to 1e-5.
"""
import numpy as np
import pytest

from oracle import mlp as R

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def _unflat(flat, dims):
    out, p = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = flat[p:p + a * b].reshape(a, b).astype(np.float64)
        p += a * b
        out.append((W, flat[p:p + b].astype(np.float64)))
        p += b
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(seed, nin=13, nh=128, nl=3, nout=1, n=1000):
    rng = np.random.default_rng(seed)
    params = R.init_params(nin, nh, nl, nout, rng)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    flat = _flat(params)
    params = _unflat(flat, [nin] + [nh] * nl + [nout])   # the FP32 values the GPU holds
    x = rng.standard_normal((n, nin)).astype(np.float32)
    t = rng.standard_normal((n, nout)).astype(np.float32)
    return params, flat, x, t


def test_forward_gradient_and_adam_match_the_reference():
    torch = _torch()
    from paper_2510_22077_amd import Mlp
    params, flat, x, t = _case(0)
    m = Mlp(13, 128, 3, 1, max_batch=1024)
    assert m.num_params() == flat.size
    m.set_params(flat)
    assert np.array_equal(m.get_params(), flat)
    y = m.forward(x).cpu().numpy().astype(np.float64)
    yr, cache = R.forward(params, x.astype(np.float64))
    err = _rel(y, yr)
    print("forward rel err", err)
    assert err <= 3e-2
    loss, g = m.grad(x, t)
    gr = R.backward(params, cache, yr, t.astype(np.float64))
    assert abs(loss - R.loss(yr, t.astype(np.float64))) <= 3e-2 * R.loss(yr, t.astype(np.float64))
    gg = _unflat(g, [13, 128, 128, 128, 1])
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(gg, gr)):
        eW, eb = _rel(gW, rW), _rel(gb, rb)
        print("layer", l, "dW rel err", eW, "db rel err", eb)
        assert eW <= 5e-2 and eb <= 5e-2
    # one Adam step from zero moments: p -= lr g / (|g| + eps)
    m.adam(lr=1e-3)
    p1 = m.get_params().astype(np.float64)
    expect = flat.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert _rel(p1, expect) <= 1e-5
    m.close()


def test_ragged_batches_and_chunked_forward():
    """n not a multiple of 16 and larger than the batch capacity (chunked)."""
    torch = _torch()
    from paper_2510_22077_amd import Mlp
    params, flat, x, t = _case(1, nin=5, nh=32, nl=2, nout=3, n=1001)
    m = Mlp(5, 32, 2, 3, max_batch=300)
    m.set_params(flat)
    y = m.forward(x).cpu().numpy().astype(np.float64)
    yr, _ = R.forward(params, x.astype(np.float64))
    assert y.shape == (1001, 3)
    assert _rel(y, yr) <= 3e-2
    loss, g = m.grad(x[:299], t[:299])
    yr2, cache2 = R.forward(params, x[:299].astype(np.float64))
    gr = R.backward(params, cache2, yr2, t[:299].astype(np.float64))
    gg = _unflat(g, [5, 32, 32, 3])
    for (gW, gb), (rW, rb) in zip(gg, gr):
        assert _rel(gW, rW) <= 5e-2 and _rel(gb, rb) <= 5e-2
    m.close()


def test_training_on_the_gpu_reduces_the_loss():
    torch = _torch()
    from paper_2510_22077_amd import Mlp
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, size=(4096, 4)).astype(np.float32)
    t = (np.sin(2 * x[:, :1]) + x[:, 1:2] * x[:, 2:3]).astype(np.float32)
    params = R.init_params(4, 64, 3, 1, rng)
    m = Mlp(4, 64, 3, 1, max_batch=512)
    m.set_params(_flat(params))
    l0 = R.loss(R.forward(params, x.astype(np.float64))[0], t.astype(np.float64))
    last = m.train(x, t, epochs=30, batch=512, lr=3e-3)
    y = m.forward(x).cpu().numpy().astype(np.float64)
    l1 = R.loss(y, t.astype(np.float64))
    print("loss", l0, "->", l1, "(last epoch mean", last, ")")
    assert l1 < 0.05 * l0
    m.close()
