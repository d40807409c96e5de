"""Plain fp64 reference of the learned policy's scoring network (test
infrastructure only).

Network: x (16) -> h1 = relu(x W1 + b1) (128) -> h2 = relu(h1 W2 + b2) (128)
-> y = h2 w3 + b3.  Parameters in one flat vector in the order W1[16][128],
b1, W2[128][128], b2, w3, b3 (row-major).  Loss (1/R) sum_r (y_r - t_r)^2.
The gradient is backpropagation written out layer by layer; the tests pin it
with central finite differences.
"""
import numpy as np

IN, HID = 16, 128
NPARAM = IN * HID + HID + HID * HID + HID + HID + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NPARAM,)
    o = 0
    W1 = w[o:o + IN * HID].reshape(IN, HID); o += IN * HID
    b1 = w[o:o + HID]; o += HID
    W2 = w[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = w[o:o + HID]; o += HID
    w3 = w[o:o + HID]; o += HID
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def forward(w, x):
    W1, b1, W2, b2, w3, b3 = unpack(w)
    x = np.asarray(x, dtype=np.float64).reshape(-1, IN)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ w3 + b3


def loss(w, x, t):
    y = forward(w, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(w, x, t):
    """(gradient of loss w.r.t. the flat parameters, loss)."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    x = np.asarray(x, dtype=np.float64).reshape(-1, IN)
    t = np.asarray(t, dtype=np.float64)
    R = x.shape[0]
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - t) / R
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    da2 = np.outer(dy, w3) * (a2 > 0)
    gW2 = h1.T @ da2
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2.T) * (a1 > 0)
    gW1 = x.T @ da1
    gb1 = da1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return g, float(np.mean((y - t) ** 2))


def init(seed):
    """A seeded parameter vector for tests (not the library's initialisation)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(NPARAM)
    o = 0
    w[o:o + IN * HID] = rng.uniform(-1, 1, IN * HID) / np.sqrt(IN); o += IN * HID
    w[o:o + HID] = rng.uniform(-0.1, 0.1, HID); o += HID
    w[o:o + HID * HID] = rng.uniform(-1, 1, HID * HID) / np.sqrt(HID); o += HID * HID
    w[o:o + HID] = rng.uniform(-0.1, 0.1, HID); o += HID
    w[o:o + HID] = rng.uniform(-1, 1, HID) / np.sqrt(HID); o += HID
    w[o] = 0.05
    return w
