"""FP64 reference of the learned-R network -- TEST INFRASTRUCTURE ONLY.

The network maps the 27 features of a query (oracle.features) to a prediction
of the nearest-neighbour statistic R of Eq. 4:

    x  = bf16(feat)                       27
    a1 = bf16(W1) x + b1,  h1 = bf16(gelu(a1))    64
    a2 = bf16(W2) h1 + b2, h2 = bf16(gelu(a2))    64
    y  = bf16(W3) h2 + b3                         1

with gelu(u) = u / 2 * (1 + tanh(sqrt(2 / pi) (u + 0.044715 u^3))) and the
training loss L = mean_b (y_b - t_b)^2.  Parameters are one float32 vector:
W1 (64 x 27, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (64), b3 (1).
bf16() rounds to the nearest bfloat16 (ties to even) after rounding to float32;
those are the points where the GPU kernels round their operands.  Everything
else is float64 here.  The gradient treats every rounding as the identity
(the straight-through gradient the GPU also computes).  With rounding=False
the network is smooth, which lets the tests check the analytic gradient by
finite differences.
"""
import numpy as np

N_IN, N_H = 27, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
C_GELU = np.sqrt(2.0 / np.pi)


def unpack(params):
    out, o = {}, 0
    p = np.asarray(params, np.float64)
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to float32, then to the nearest bfloat16 (ties to even); returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(u):
    return 0.5 * u * (1.0 + np.tanh(C_GELU * (u + 0.044715 * u ** 3)))


def gelu_grad(u):
    t = np.tanh(C_GELU * (u + 0.044715 * u ** 3))
    return 0.5 * (1.0 + t) + 0.5 * u * (1.0 - t * t) * C_GELU * (1.0 + 3 * 0.044715 * u * u)


def forward(params, feat, rounding=True):
    """-> (y [B], cache) for features [B, 27]."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    P = unpack(params)
    x = r(feat)
    a1 = x @ r(P["W1"]).T + P["b1"]
    h1 = r(gelu(a1))
    a2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(gelu(a2))
    y = h2 @ r(P["W3"]) + P["b3"][0]
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, y=y, W2=r(P["W2"]), W3=r(P["W3"]))


def loss_and_grad(params, feat, target, rounding=True):
    """Mean squared error over the batch and its gradient with respect to the parameter vector."""
    y, c = forward(params, feat, rounding)
    t = np.asarray(target, np.float64)
    B = y.shape[0]
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / B
    g = {}
    g["W3"] = dy @ c["h2"]
    g["b3"] = np.array([dy.sum()])
    da2 = np.outer(dy, c["W3"]) * gelu_grad(c["a2"])
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ c["W2"]) * gelu_grad(c["a1"])
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)
