"""fp64 reference of the per-level variant scheduler (test infrastructure).

The paper fixes the worker at one warp per vertex and argues (Sec. 4.3.1) that
a finer worker only pays when the graph sits in GPU memory and degrees are
low, while Sec. 5.3.1 shows that alignment pays least on uniformly
low-degree graphs: no single access variant wins on every frontier.  The
scheduler is a small network that maps 16 frontier features to one of 6
result-identical variants.  This module is its plain definition:

    h1 = relu(W1 x + b1)      W1: 64x16
    h2 = relu(W2 h1 + b2)     W2: 64x64
    z  = W3 h2 + b3           W3: 6x64
    loss = mean_b [ logsumexp(z_b) - z_b[y_b] ]   (softmax cross-entropy)

Parameters are one flat vector in the order W1, b1, W2, b2, W3, b3
(row-major, 5638 values).  Adam follows Kingma & Ba (2015), Algorithm 1.
"""
import numpy as np

N_IN, N_H, N_OUT = 16, 64, 6
SHAPES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta):
    out, k = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[k:k + n], dtype=np.float64).reshape(s))
        k += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X):
    """Returns (logits z [B,6], cache) for inputs X [B,16]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (X, a1, h1, a2, h2)


def loss(theta, X, y):
    z, _ = forward(theta, X)
    m = z.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(z - m).sum(axis=1))
    return float(np.mean(lse - z[np.arange(z.shape[0]), y]))


def backward(theta, X, y):
    """Analytic gradient of ``loss`` with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    B = z.shape[0]
    m = z.max(axis=1, keepdims=True)
    p = np.exp(z - m)
    p /= p.sum(axis=1, keepdims=True)
    dz = p.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(theta, X):
    z, _ = forward(theta, X)
    return np.argmax(z, axis=1)
