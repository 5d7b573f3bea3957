"""Gradient-corrector network, FP64 reference: forward pass, MSE loss, its
gradient by hand-written backpropagation, and Adam.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

The paper motivates a correction of the near-surface velocity gradients of
the immersed boundary method (Sec. 3.2.1 and Sec. 4) without
specifying one. Reading: a multilayer perceptron 85 -> 64 -> 64 -> 9 with
SiLU activations,
    z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, h2 = silu(z2),
    y = W3 h2 + b3,
silu(z) = z sigmoid(z), trained on the mean squared error over the batch
and the 9 outputs, L = mean((y - t)^2), with Adam (Kingma & Ba 2015):
    m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Parameters are one vector: W1 (64x85, [out][in]), b1, W2, b2, W3 (9x64), b3.
Batches are rows: X (B, 85), targets T (B, 9).
"""
import numpy as np

N_IN, N_HID, N_OUT = 85, 64, 9
SHAPES = ((N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,))
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 10,249


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    """d/dz [z s(z)] = s(z) + z s(z) (1 - s(z))."""
    s = sigmoid(z)
    return s + z * s * (1.0 - s)


def forward(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(T, np.float64)) ** 2))


def grad(theta, X, T):
    """(loss, dL/dtheta) by backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    T = np.asarray(T, np.float64)
    B = X.shape[0]
    dy = 2.0 * (y - T) / (B * N_OUT)
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dz2 = (dy @ W3) * silu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * silu_grad(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return float(np.mean((y - T) ** 2)), pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
