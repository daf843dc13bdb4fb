"""FP64 reference of the access-path chooser's network (test infrastructure).

A 6 -> 64 -> 64 -> 16 perceptron with ReLU; a layer computes
out[j] = b[j] + sum_i in[i] W[i][j].  The loss is the masked mean squared
error sum(mask (y - t)^2) / sum(mask) over predicted and measured log-times;
gradients follow from the chain rule (ReLU passes the gradient where its
input was positive); Adam is Kingma & Ba's update with bias correction.
Parameters are one flat vector: W1[6][64], b1[64], W2[64][64], b2[64],
W3[64][16], b3[16].  Pinned by tests/test_oracle_mlp.py.
"""

import numpy as np

NI, NH, NO = 6, 64, 16
SHAPES = [("W1", (NI, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NO)),
          ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(p, x):
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ w["W1"] + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (z1, h1, z2, h2)


def loss(p, x, t, mask):
    y, _ = forward(p, x)
    m = np.asarray(mask, dtype=np.float64)
    e = m * (y - np.asarray(t, dtype=np.float64))
    return float((e * e).sum() / m.sum())


def grad(p, x, t, mask):
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(p, x)
    m = np.asarray(mask, dtype=np.float64)
    count = m.sum()
    e = m * (y - np.asarray(t, dtype=np.float64))
    dy = 2.0 * e / count
    d2 = (dy @ w["W3"].T) * (z2 > 0)
    d1 = (d2 @ w["W2"].T) * (z1 > 0)
    g = {"W3": h2.T @ dy, "b3": dy.sum(0), "W2": h1.T @ d2, "b2": d2.sum(0),
         "W1": x.T @ d1, "b1": d1.sum(0)}
    return pack(g), float((e * e).sum() / count)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
