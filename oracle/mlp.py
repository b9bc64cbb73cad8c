"""FP64 oracle of the process-rate surrogate network -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product never imports it and shares no code with it.

Network: 12 inputs -> three hidden layers of 128 units with the SiLU
activation silu(z) = z / (1 + exp(-z)) -> 12 linear outputs.
Parameters are one flat vector in the order W1 (12x128, row = input),
b1 (128), W2 (128x128), b2, W3 (128x128), b3, W4 (128x12), b4 (12):
36,236 values.  Layer l computes z_l = a_{l-1} W_l + b_l.

Loss: masked mean squared error
    L = sum_ij m_ij (y_ij - t_ij)^2 / max(1, sum_ij m_ij).
Gradients follow the chain rule layer by layer (dL/dW_l = a_{l-1}^T dL/dz_l,
dL/db_l = column sums of dL/dz_l, dL/da_{l-1} = dL/dz_l W_l^T,
dL/dz_l = dL/da_l * silu'(z_l) with silu'(z) = s (1 + z (1 - s)), s the
logistic function).
Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

SIZES = (12, 128, 128, 128, 12)


def layer_shapes():
    out = []
    for i in range(4):
        out.append(((SIZES[i], SIZES[i + 1]), (SIZES[i + 1],)))
    return out


N_PARAMS = sum(a * b + b for (a, b), _ in layer_shapes())


def unpack(theta: np.ndarray):
    """Flat vector -> [(W1, b1), ..., (W4, b4)] views."""
    out, o = [], 0
    for (a, b), _ in layer_shapes():
        W = theta[o:o + a * b].reshape(a, b); o += a * b
        bb = theta[o:o + b]; o += b
        out.append((W, bb))
    assert o == theta.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """Returns (y, cache) with cache = list of (a_in, z) per layer."""
    a = np.asarray(X, dtype=np.float64)
    cache = []
    layers = unpack(np.asarray(theta, dtype=np.float64))
    for i, (W, b) in enumerate(layers):
        z = a @ W + b
        cache.append((a, z))
        a = silu(z) if i < 3 else z
    return a, cache


def loss(theta, X, T, M):
    y, _ = forward(theta, X)
    return float(np.sum(M * (y - T) ** 2) / max(1.0, float(np.sum(M))))


def loss_and_grad(theta, X, T, M):
    theta = np.asarray(theta, dtype=np.float64)
    y, cache = forward(theta, X)
    denom = max(1.0, float(np.sum(M)))
    L = float(np.sum(M * (y - T) ** 2) / denom)
    layers = unpack(theta)
    grads = []
    dz = 2.0 * M * (y - T) / denom
    for i in range(3, -1, -1):
        a_in, z = cache[i]
        W, _ = layers[i]
        gW = a_in.T @ dz
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if i > 0:
            da = dz @ W.T
            dz = da * dsilu(cache[i - 1][1])
    grads.reverse()
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, g


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  bfloat16 keeps the top 16 bits of the binary32 encoding."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out)


def forward_bf16(theta, X):
    """Inference with bfloat16 weights and activations and float32
    accumulation, with the activations carried scaled by s = -log2(e) (the
    base-2 exponent of the logistic function): with z_l = a_{l-1} W_l + b_l
    and silu(z) = z / (1 + e^-z),

        c_0 = bf16(s x),
        u_l = c_{l-1} bf16(W_l) + s b_l   (= s z_l up to rounding),
        c_l = bf16(u_l / (1 + 2^u_l))     (= s silu(z_l), as 2^(s z) = e^-z),
        y   = -ln(2) (c_3 bf16(W_4) + s b_4)   (= z_4, as -ln(2) s = 1).

    Every layer input and every weight is rounded to bfloat16; products,
    sums and the scalings are formed in float32."""
    s = np.float32(-1.4426950408889634)
    c = bf16_round(s * np.asarray(X, dtype=np.float32))
    layers = unpack(np.asarray(theta, dtype=np.float64))
    for i, (W, b) in enumerate(layers):
        Wb = bf16_round(W.astype(np.float32))
        u = (c.astype(np.float32) @ Wb).astype(np.float32) + s * b.astype(np.float32)
        if i < 3:
            with np.errstate(over="ignore"):          # 2^u = inf gives c = 0
                c = bf16_round(u / (np.float32(1.0) + np.exp2(u)))
        else:
            return np.float32(-0.6931471805599453) * u
