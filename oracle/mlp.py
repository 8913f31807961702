"""CPU oracle for the learned per-element eddy-viscosity closure network.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): plain numpy in float64, written from the
definitions below, and shared with nothing in the HIP library.

The network (the closure's reading; the paper names "LES sub-grid scale models" without one):
  x_hat = (x - mean) / std                      input standardisation, fixed per model
  h1 = tanh(W1 x_hat + b1)                      H = 64 units
  h2 = tanh(W2 h1 + b2)                         H = 64 units
  y  = softplus(w3 . h2 + b3)                   y = nu_t / nu_scale >= 0
Weights W1, W2, w3 are used rounded to bfloat16 (round to nearest, ties to even) from their
float32 master copies; biases, standardisation and accumulation are wider. Training minimises
L = mean_n (y_n - t_n)^2 with Adam (Kingma and Ba, 2015) on the float32 masters; the gradient
with respect to a master is the gradient with respect to its rounded copy.

Flat parameter layout (float32): W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3[1].
"""
from __future__ import annotations

import numpy as np

H = 64


def n_params(F: int) -> int:
    return H * F + H + H * H + H + H + 1


def unpack(theta: np.ndarray, F: int) -> dict:
    theta = np.asarray(theta)
    assert theta.shape == (n_params(F),)
    o = 0
    out = {}
    for name, shape in (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)),
                        ("b3", (1,))):
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[k]).ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32. Finite inputs only."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    assert np.all(np.isfinite(x))
    b = x.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def effective(theta: np.ndarray, F: int) -> dict:
    """float64 copies of the parameters as the network uses them (weights rounded to bf16)."""
    d = unpack(np.asarray(theta, dtype=np.float32), F)
    return {k: (bf16_round(v) if k in ("W1", "W2", "w3") else v).astype(np.float64) for k, v in d.items()}


def init_params(F: int, seed: int) -> np.ndarray:
    """Seeded uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) initialisation, float32."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, fan_in, shape in (("W1", F, (H, F)), ("b1", F, (H,)), ("W2", H, (H, H)), ("b2", H, (H,)),
                                ("w3", H, (H,)), ("b3", H, (1,))):
        lim = 1.0 / np.sqrt(fan_in)
        d[name] = rng.uniform(-lim, lim, size=shape)
    return pack(d).astype(np.float32)


def softplus(z):
    return np.logaddexp(0.0, z)


def forward(eff: dict, X: np.ndarray, mean: np.ndarray, std: np.ndarray, keep: bool = False):
    """y [N] for inputs X [N][F]; with keep=True also the intermediate values."""
    Xh = (np.asarray(X, np.float64) - np.asarray(mean, np.float64)) / np.asarray(std, np.float64)
    h1 = np.tanh(Xh @ eff["W1"].T + eff["b1"])
    h2 = np.tanh(h1 @ eff["W2"].T + eff["b2"])
    z = h2 @ eff["w3"] + eff["b3"][0]
    y = softplus(z)
    if keep:
        return y, {"Xh": Xh, "h1": h1, "h2": h2, "z": z}
    return y


def loss_and_grad(theta: np.ndarray, X, t, mean, std):
    """L = mean (y - t)^2 and dL/dtheta (float64, flat layout), by the chain rule."""
    F = np.asarray(X).shape[1]
    eff = effective(theta, F)
    y, c = forward(eff, X, mean, std, keep=True)
    N = y.shape[0]
    t = np.asarray(t, np.float64)
    L = np.mean((y - t) ** 2)
    dz = 2.0 * (y - t) / N / (1.0 + np.exp(-c["z"]))  # softplus'(z) = logistic(z)
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, eff["w3"]) * (1.0 - c["h2"] ** 2)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ eff["W2"]) * (1.0 - c["h1"] ** 2)
    g["W1"] = da1.T @ c["Xh"]
    g["b1"] = da1.sum(axis=0)
    return L, pack(g)


class Adam:
    """Adam on float32 master parameters; moments kept in float64 here, masters rounded to
    float32 after each update as the library stores them."""

    def __init__(self, theta, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = np.asarray(theta, dtype=np.float32).copy()
        self.m = np.zeros(self.theta.shape)
        self.v = np.zeros(self.theta.shape)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.theta = (self.theta.astype(np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps)).astype(np.float32)
        return self.theta
