"""FP64 reference of the coarse-coefficient MLP: forward, backward, loss, Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps a feature vector to one coarse-operator coefficient:
  h_0 = x,  h_l = gelu(h_{l-1} W_l + b_l)  (l = 1..L hidden layers),
  y = h_L W_out + b_out,
with GELU in its tanh form, gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
Loss: mean squared error over the batch.  Optimiser: Adam (Kingma & Ba, 2015)
with bias correction.  Weights are row-major [fan_in, fan_out].
"""
import numpy as np

C_GELU = np.sqrt(2.0 / np.pi)
A_GELU = 0.044715


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + A_GELU * z ** 3)))


def gelu_grad(z):
    u = C_GELU * (z + A_GELU * z ** 3)
    t = np.tanh(u)
    du = C_GELU * (1.0 + 3.0 * A_GELU * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def init_params(nin, nhidden, nlayers, nout, rng):
    """He-style uniform init; returns a list [(W, b), ...] of nlayers + 1 layers."""
    dims = [nin] + [nhidden] * nlayers + [nout]
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / a)
        params.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
    return params


def forward(params, x):
    """Returns (y, cache) with cache = (pre-activations z_l, activations h_l)."""
    hs = [x]
    zs = []
    h = x
    for W, b in params[:-1]:
        z = h @ W + b
        zs.append(z)
        h = gelu(z)
        hs.append(h)
    W, b = params[-1]
    y = h @ W + b
    return y, (zs, hs)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of the MSE loss: list [(dW, db), ...] aligned with params."""
    zs, hs = cache
    n = y.shape[0]
    dy = 2.0 * (y - t) / (n * y.shape[1])
    grads = [None] * len(params)
    W, _ = params[-1]
    grads[-1] = (hs[-1].T @ dy, dy.sum(axis=0))
    dh = dy @ W.T
    for l in range(len(params) - 2, -1, -1):
        dz = dh * gelu_grad(zs[l])
        grads[l] = (hs[l].T @ dz, dz.sum(axis=0))
        dh = dz @ params[l][0].T
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for k, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][k] + (1.0 - self.b1) * g
                v = self.b2 * self.v[i][k] + (1.0 - self.b2) * g * g
                mm = list(self.m[i]); mm[k] = m; self.m[i] = tuple(mm)
                vv = list(self.v[i]); vv[k] = v; self.v[i] = tuple(vv)
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out
