"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE).

A multilayer perceptron n_in -> width (SiLU) x depth -> 1 trained on the mean
squared error.  Flat parameter vector: for each layer, W [out][in] row-major
then b [out] (the layout the HIP kernels use).  SiLU(z) = z sigma(z),
SiLU'(z) = sigma(z) (1 + z (1 - sigma(z))).  AdamW with decoupled weight decay
(Loshchilov and Hutter): w <- w - lr (m_hat / (sqrt(v_hat) + eps) + wd w).
"""
import numpy as np


def layer_shapes(n_in=5, width=128, depth=3):
    shapes, prev = [], n_in
    for _ in range(depth):
        shapes.append((width, prev))
        prev = width
    shapes.append((1, prev))
    return shapes


def num_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(params, shapes):
    out, k = [], 0
    for o, i in shapes:
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    return out


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X, shapes):
    layers = unpack(np.asarray(params, np.float64), shapes)
    H = np.asarray(X, np.float64)
    cache = [H]
    for W, b in layers[:-1]:
        Z = H @ W.T + b
        H = Z * _sig(Z)
        cache.append((Z, H))
    W, b = layers[-1]
    y = (H @ W.T + b)[:, 0]
    return y, cache


def loss_and_grad(params, X, y, shapes):
    """L = mean((f(x) - y)^2) and dL/dparams (flat, same layout)."""
    layers = unpack(np.asarray(params, np.float64), shapes)
    yhat, cache = forward(params, X, shapes)
    B = len(y)
    g = 2.0 * (yhat - np.asarray(y, np.float64)) / B
    grads = []
    H_last = cache[-1][1] if len(cache) > 1 else cache[0]
    W, b = layers[-1]
    grads.append((g[:, None] * H_last).sum(0)[None, :].ravel().tolist() + [g.sum()])
    dH = g[:, None] * W[0][None, :]
    for li in range(len(layers) - 2, -1, -1):
        Z, _ = cache[li + 1]
        Hprev = cache[li][1] if li > 0 else cache[0]
        s = _sig(Z)
        dZ = dH * s * (1.0 + Z * (1.0 - s))
        W, b = layers[li]
        grads.append(list((dZ.T @ Hprev).ravel()) + list(dZ.sum(0)))
        dH = dZ @ W
    flat = []
    for gl in reversed(grads):
        flat.extend(gl)
    return float(np.mean((yhat - y) ** 2)), np.array(flat)


def adamw_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    params = params - lr * (mh / (np.sqrt(vh) + eps) + wd * params)
    return params, m, v


def init_params(shapes, seed=0):
    """Uniform(+-1/sqrt(fan_in)) weights and biases from numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for o, i in shapes:
        bound = 1.0 / np.sqrt(i)
        out.append(rng.uniform(-bound, bound, o * i))
        out.append(rng.uniform(-bound, bound, o))
    return np.concatenate(out)
