"""Oracle (test infrastructure only): the learned pressure-stage correction.

A small 3-D convolutional network maps the normalised pressure residual and
log-permeability of every cell to a pressure correction:

    c = s * N([r_p / s, (ln k - mu) / sigma]),   s = RMS(r_p),

with N four zero-padded "same" 3x3x3 convolutions, channels 2 -> 16 -> 16 ->
16 -> 1, biases, and ReLU after the first three.  The correction is trained
on pairs (r_p, e) with e = A_pp^{-1} r_p - V(r_p), the error that one AMG
V-cycle leaves, by mean-squared error on e / s (or by the A_pp-weighted
error, the residual the correction would leave) and Adam.  In CPR the
V-cycle result is corrected by the multiple of c that minimises the pressure
residual ||r_p - A_pp x||, when that multiple is positive; otherwise the
plain V-cycle result is used.

Everything here is plain numpy: FP64 forward and backward, and a BF16
emulation in which the weights, each layer's input and each backward operand
are rounded to BF16 and products are summed exactly and rounded to FP32 (the
precision of a BF16 matrix-core product with FP32 accumulation).

Tensors are (nz, ny, nx, channels).  Tap t of a 3x3x3 kernel has offset
(dz, dy, dx) = (t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1); a layer's weights
are W[t, c_in, c_out].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 16, 16, 16, 1)
TAPS = [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def bf16(x) -> np.ndarray:
    """Round to BF16 (8 significant bits, ties to even) from the FP32 value,
    returned as float32."""
    f = np.asarray(x, dtype=np.float32)
    m, e = np.frexp(f)                       # f = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(f) & (f != 0), r, f).astype(np.float32)


def _shifted(X: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """S[v] = X[v + (dz, dy, dx)], zero outside the grid."""
    P = np.pad(X, ((1, 1), (1, 1), (1, 1), (0, 0)))
    nz, ny, nx = X.shape[:3]
    return P[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def conv(X: np.ndarray, W: np.ndarray, b=None) -> np.ndarray:
    """Z[v, o] = b[o] + sum_t sum_c X[v + off(t), c] W[t, c, o] (FP64 sums)."""
    X = np.asarray(X, dtype=np.float64)
    Z = np.zeros(X.shape[:3] + (W.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        Z += _shifted(X, dz, dy, dx) @ np.asarray(W[t], dtype=np.float64)
    if b is not None:
        Z += np.asarray(b, dtype=np.float64)
    return Z


def conv_input_grad(dZ: np.ndarray, W: np.ndarray) -> np.ndarray:
    """dX[u, c] = sum_t sum_o dZ[u - off(t), o] W[t, c, o]."""
    dZ = np.asarray(dZ, dtype=np.float64)
    dX = np.zeros(dZ.shape[:3] + (W.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        dX += _shifted(dZ, -dz, -dy, -dx) @ np.asarray(W[t], dtype=np.float64).T
    return dX


def conv_weight_grad(X: np.ndarray, dZ: np.ndarray):
    """dW[t, c, o] = sum_v X[v + off(t), c] dZ[v, o];  db[o] = sum_v dZ[v, o]."""
    X = np.asarray(X, dtype=np.float64)
    dZ = np.asarray(dZ, dtype=np.float64)
    co = dZ.shape[3]
    D = dZ.reshape(-1, co)
    dW = np.stack([_shifted(X, dz, dy, dx).reshape(-1, X.shape[3]).T @ D for (dz, dy, dx) in TAPS])
    return dW, D.sum(axis=0)


def forward(params, X, emulate_bf16: bool = False):
    """Returns the output (nz, ny, nx, 1) and the per-layer cache.  params is a
    list of (W, b) per layer."""
    cache = []
    A = np.asarray(X, dtype=np.float64)
    nl = len(params)
    for l, (W, b) in enumerate(params):
        if emulate_bf16:
            Ain = bf16(A).astype(np.float64)
            Z = conv(Ain, bf16(W).astype(np.float64))
            Z = (Z.astype(np.float32) + np.asarray(b, dtype=np.float32)).astype(np.float64)
        else:
            Ain = A
            Z = conv(Ain, W, b)
        cache.append((Ain, Z))
        A = np.maximum(Z, 0.0) if l < nl - 1 else Z
    return A, cache


def mse(Y, T) -> float:
    d = np.asarray(Y, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    return float(np.mean(d * d))


def backward(params, cache, Y, T, emulate_bf16: bool = False):
    """Gradients of mse(Y, T) with respect to every (W, b)."""
    M = np.asarray(Y).size
    dZ = 2.0 * (np.asarray(Y, dtype=np.float64) - np.asarray(T, dtype=np.float64)) / M
    return _backprop(params, cache, dZ, emulate_bf16)


def _backprop(params, cache, dZ, emulate_bf16: bool):
    """Weight and bias gradients from the output gradient dZ (nz, ny, nx, 1)."""
    if emulate_bf16:
        dZ = dZ.astype(np.float32).astype(np.float64)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        Ain, Z = cache[l]
        if emulate_bf16:
            dZq = bf16(dZ).astype(np.float64)
            dW, db = conv_weight_grad(Ain, dZq)
            grads[l] = (dW.astype(np.float32).astype(np.float64), db.astype(np.float32).astype(np.float64))
            if l > 0:
                dX = conv_input_grad(dZq, bf16(W).astype(np.float64)).astype(np.float32).astype(np.float64)
                dZ = dX * (cache[l - 1][1] > 0)
        else:
            grads[l] = conv_weight_grad(Ain, dZ)
            if l > 0:
                dZ = conv_input_grad(dZ, W) * (cache[l - 1][1] > 0)
    return grads


# 7-point stencil slots of a pressure matrix: (dz, dy, dx) of the coupled cell
SLOTS = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]


def stencil_apply(coef: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """(A y)_i = sum_s coef[s, i] y[i + off(s)] on a (nz, ny, nx) volume,
    couplings that leave the volume dropped (coef: (7, nz, ny, nx))."""
    Y = np.asarray(Y, dtype=np.float64)
    out = np.zeros(Y.shape)
    for s, (dz, dy, dx) in enumerate(SLOTS):
        out += np.asarray(coef[s], dtype=np.float64) * _shifted(Y[..., None], dz, dy, dx)[..., 0]
    return out


def interior_mask(shape) -> np.ndarray:
    """Voxels whose six neighbours all lie in the volume."""
    m = np.zeros(shape, dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def weighted_loss(Y, coef, T) -> float:
    """Mean over interior voxels of (A (y - t))^2: the error of the correction
    measured by the pressure residual it would leave, on the voxels whose
    stencil lies inside the volume."""
    d = np.asarray(Y, dtype=np.float64).reshape(np.shape(T)) - np.asarray(T, dtype=np.float64)
    m = interior_mask(np.shape(T))
    R = stencil_apply(coef, d)[m]
    return float(np.mean(R * R))


def weighted_loss_grad(Y, coef, T) -> np.ndarray:
    """d weighted_loss / d y = (2 / M) A^T (mask . A (y - t)), M interior voxels."""
    shape = np.shape(T)
    d = np.asarray(Y, dtype=np.float64).reshape(shape) - np.asarray(T, dtype=np.float64)
    m = interior_mask(shape)
    R = np.where(m, stencil_apply(coef, d), 0.0)
    g = np.zeros(shape)
    for s, (dz, dy, dx) in enumerate(SLOTS):
        # (A^T R)_j gets coef[s, i] R_i from i = j - off(s)
        g += _shifted((np.asarray(coef[s], dtype=np.float64) * R)[..., None], -dz, -dy, -dx)[..., 0]
    return 2.0 * g / max(int(m.sum()), 1)


def backward_weighted(params, cache, Y, coef, T, emulate_bf16: bool = False):
    """Gradients of weighted_loss(Y, coef, T) with respect to every (W, b)."""
    dY = weighted_loss_grad(Y, coef, T)[..., None]
    return _backprop(params, cache, dY, emulate_bf16)


class Adam:
    """Adam (Kingma and Ba) with bias correction, on FP64 copies of the
    parameters."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros(np.shape(W)), np.zeros(np.shape(b))] for W, b in params]
        self.v = [[np.zeros(np.shape(W)), np.zeros(np.shape(b))] for W, b in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for q, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.m[l][q] = self.b1 * self.m[l][q] + (1 - self.b1) * g
                v = self.v[l][q] = self.b2 * self.v[l][q] + (1 - self.b2) * g * g
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(np.asarray(p, dtype=np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps))
            out.append(tuple(new))
        return out


def normalise_inputs(rp: np.ndarray, logk: np.ndarray, shape):
    """Network input (nz, ny, nx, 2) and the scale s = RMS(r_p)."""
    s = float(np.sqrt(np.mean(np.asarray(rp, dtype=np.float64) ** 2)))
    s = s if s > 0 else 1.0
    lk = np.asarray(logk, dtype=np.float64)
    sd = float(lk.std())
    z = (lk - lk.mean()) / (sd if sd > 0 else 1.0)
    X = np.stack([np.asarray(rp, dtype=np.float64).reshape(shape) / s, z.reshape(shape)], axis=-1)
    return X, s


def judge(App, rp, v, c):
    """The V-cycle result v corrected by the multiple alpha c of the network's
    correction that minimises ||r_p - A_pp (v + alpha c)||: alpha =
    <u, A_pp c> / ||A_pp c||^2 with u = r_p - A_pp v.  The correction is kept
    when alpha > 0 (the residual then falls by the factor sqrt(1 - cos^2) of
    the angle between u and A_pp c); otherwise (alpha <= 0, or A_pp c = 0)
    the plain V-cycle result is used.  Returns (x, alpha)."""
    u = rp - App @ v
    w = App @ c
    q = float(w @ w)
    p = float(u @ w)
    if q > 0.0 and p > 0.0:
        a = p / q
        return v + a * c, a
    return v, 0.0
