"""fp64 CPU reference of the cost-model MLP (test infrastructure only).

A 16 -> 64 -> 64 -> 2 multilayer perceptron with ReLU hidden layers, inputs
standardised by (x - mean_x) / std_x, targets by (t - mean_y) / std_y, loss =
mean over samples and outputs of the squared error in standardised units, and
Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015) with
bias correction.  Forward and backward are written out layer by layer (the
chain rule by hand); the tests pin them to finite differences and to an
independent automatic-differentiation library.

Parameter vector layout (row-major W[out][in]): W1[64][16] b1[64] W2[64][64]
b2[64] W3[2][64] b3[2]; normalisation vector: mean_x[16] std_x[16] mean_y[2]
std_y[2].
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 16, 64, 2
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)), ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
NNORM = 2 * IN + 2 * OUT


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def split_norm(norm):
    norm = np.asarray(norm, dtype=np.float64)
    return norm[:IN], norm[IN:2 * IN], norm[2 * IN:2 * IN + OUT], norm[2 * IN + OUT:]


def forward(p, norm, X):
    """Raw-scale predictions [B, 2] and the intermediate values."""
    w = unpack(p)
    mx, sx, my, sy = split_norm(norm)
    xn = (np.asarray(X, np.float64) - mx) / sx
    z1 = xn @ w["W1"].T + w["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ w["W2"].T + w["b2"]
    a2 = np.maximum(z2, 0.0)
    yn = a2 @ w["W3"].T + w["b3"]
    return yn * sy + my, dict(xn=xn, z1=z1, a1=a1, z2=z2, a2=a2, yn=yn)


def loss_and_grad(p, norm, X, T):
    """Loss and its gradient w.r.t. the parameter vector."""
    w = unpack(p)
    mx, sx, my, sy = split_norm(norm)
    _, c = forward(p, norm, X)
    B = len(X)
    tn = (np.asarray(T, np.float64) - my) / sy
    e = c["yn"] - tn
    loss = float(np.sum(e * e) / (B * OUT))
    dy = 2.0 * e / (B * OUT)                      # d loss / d yn
    g = {"W3": dy.T @ c["a2"], "b3": dy.sum(0)}
    da2 = dy @ w["W3"]
    dz2 = da2 * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["a1"]
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ w["W2"]
    dz1 = da1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["xn"]
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(p, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    g = np.asarray(grad, np.float64) + weight_decay * np.asarray(p, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
