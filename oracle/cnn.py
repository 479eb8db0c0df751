"""FP64 NumPy oracle of the warm-start network (test infrastructure only).

The network is not from the paper: it predicts a starting point u0 for the paper's PCG from
the noisy image and the parameters.  Architecture: five 3x3 convolutions with zero "same"
padding, widths in -> 32 -> 32 -> 32 -> 32 -> 1, ReLU between layers, no activation at the end;
input channels (f, log alpha, log sigma_1..L) with the scalars broadcast as constant maps;
output u0 = f + residual.  Loss: mean squared error against the reference solution.  Training
step: Adam with bias correction.

Convolution convention (cross-correlation, as in deep-learning libraries):
    y[co, i, j] = b[co] + sum_ci sum_{a,c in -1..1} w[co, ci, a+1, c+1] x[ci, i+a, j+c]
with x = 0 outside the image.  Parameters are kept as a flat FP64 vector in the order
(W_1, b_1, ..., W_5, b_5), each W_k of shape (cout, cin, 3, 3).

Pins (tests): the forward pass against scipy.signal.correlate2d summed over channels,
the backward passes against central finite differences, one Adam step against its closed
form, and the full-network gradient against finite differences.
"""
from __future__ import annotations

import numpy as np

WIDTH = 32
DEPTH = 5


def layer_shapes(cin: int, width: int = WIDTH, depth: int = DEPTH):
    shapes = []
    c = cin
    for k in range(depth):
        co = 1 if k == depth - 1 else width
        shapes.append((co, c))
        c = co
    return shapes


def param_count(cin: int) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(cin))


def unpack(theta: np.ndarray, cin: int):
    out = []
    o = 0
    for co, ci in layer_shapes(cin):
        w = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((w, b))
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x (cin, H, W), w (cout, cin, 3, 3), b (cout,) -> (cout, H, W)."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], H, W)) + b[:, None, None]
    for a in range(3):
        for c in range(3):
            patch = xp[:, a:a + H, c:c + W]                     # x[ci, i + a - 1, j + c - 1]
            y += np.einsum("oc,chw->ohw", w[:, :, a, c], patch)
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to x, w and b."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            patch = xp[:, a:a + H, c:c + W]
            dw[:, :, a, c] = np.einsum("ohw,chw->oc", dy, patch)
            dxp[:, a:a + H, c:c + W] += np.einsum("oc,ohw->chw", w[:, :, a, c], dy)
    db = dy.sum(axis=(1, 2))
    return dxp[:, 1:-1, 1:-1], dw, db


def inputs(f: np.ndarray, cond) -> np.ndarray:
    """Channels (f, cond_0, cond_1, ...) of one image; cond = (log alpha, log sigma_1..L)."""
    H, W = f.shape
    x = np.empty((1 + len(cond), H, W))
    x[0] = f
    for k, c in enumerate(cond):
        x[1 + k] = c
    return x


def forward(theta: np.ndarray, f: np.ndarray, cond):
    """Returns (u0, cache) for one image."""
    x = inputs(f, cond)
    layers = unpack(theta, x.shape[0])
    acts = [x]
    pre = []
    h = x
    for k, (w, b) in enumerate(layers):
        z = conv3x3(h, w, b)
        pre.append(z)
        h = np.maximum(z, 0.0) if k < len(layers) - 1 else z
        acts.append(h)
    return f + h[0], (acts, pre, layers)


def loss_and_grad(theta: np.ndarray, batch):
    """batch = [(f, cond, target)]; loss = mean over all pixels of (u0 - target)^2."""
    count = sum(f.size for f, _, _ in batch)
    loss = 0.0
    grad = np.zeros_like(theta)
    for f, cond, target in batch:
        u0, (acts, pre, layers) = forward(theta, f, cond)
        e = u0 - target
        loss += float(np.sum(e * e)) / count
        d = (2.0 / count * e)[None]                  # d loss / d (last pre-activation)
        grads = []
        for k in range(len(layers) - 1, -1, -1):
            w, _ = layers[k]
            dx, dw, db = conv3x3_backward(acts[k], w, d)
            grads.append((dw, db))
            if k > 0:
                d = dx * (pre[k - 1] > 0.0)
        o = 0
        for dw, db in reversed(grads):
            grad[o:o + dw.size] += dw.ravel()
            o += dw.size
            grad[o:o + db.size] += db
            o += db.size
    return loss, grad


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
