"""Pins of the oracle's learned pressure-stage network (CPU only): the
convolution against scipy's n-dimensional correlation, the analytic gradients
against central finite differences, Adam against torch's optimiser, the BF16
rounding against torch's conversion, and the judge's fallback."""
import numpy as np
import pytest

import bo_casegen as cg
from oracle import cnn as N


def rand_params(seed, chans=(2, 4, 4, 3, 1), scale=0.3):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((27, chans[l], chans[l + 1])) * scale, rng.standard_normal(chans[l + 1]) * 0.1)
            for l in range(len(chans) - 1)]


def test_conv_matches_scipy_correlate():
    from scipy.signal import correlate
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5, 6, 7, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    Z = N.conv(X, W, b)
    for o in range(2):
        ref = np.full(X.shape[:3], b[o])
        for c in range(3):
            ker = W[:, c, o].reshape(3, 3, 3)   # tap t -> (dz+1, dy+1, dx+1)
            ref += correlate(X[..., c], ker, mode="same")
        assert np.allclose(Z[..., o], ref, rtol=1e-13, atol=1e-13)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((4, 5, 3, 2))
    T = rng.standard_normal((4, 5, 3, 1))
    params = rand_params(3)
    Y, cache = N.forward(params, X)
    grads = N.backward(params, cache, Y, T)
    h = 1e-6
    for l in range(4):
        for which in (0, 1):
            p = params[l][which]
            g = grads[l][which]
            for idx in [tuple(rng.integers(0, s) for s in p.shape) for _ in range(6)]:
                old = p[idx]
                p[idx] = old + h
                lp = N.mse(N.forward(params, X)[0], T)
                p[idx] = old - h
                lm = N.mse(N.forward(params, X)[0], T)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-3), (l, which, idx, fd, g[idx])


def test_input_gradient_chain_matches_finite_differences():
    """conv_input_grad is the adjoint of conv: <conv(X), D> = <X, conv^T(D)>."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 3, 5, 3))
    W = rng.standard_normal((27, 3, 2))
    D = rng.standard_normal((4, 3, 5, 2))
    lhs = np.sum(N.conv(X, W) * D)
    rhs = np.sum(X * N.conv_input_grad(D, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    params = rand_params(6)
    opt = N.Adam(params, lr=1e-2)
    tparams = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for W, b in params for p in (W, b)]
    topt = torch.optim.Adam(tparams, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    cur = params
    for _ in range(5):
        grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in cur]
        cur = opt.step(cur, grads)
        for tp, g in zip(tparams, [g for pair in grads for g in pair]):
            tp.grad = torch.tensor(g, dtype=torch.float64)
        topt.step()
    ours = [p for pair in cur for p in pair]
    for a, t in zip(ours, tparams):
        assert np.allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(7)
    v = (rng.standard_normal(5000) * np.exp2(rng.integers(-30, 30, 5000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(N.bf16(v), ref)


def test_bf16_emulation_close_to_fp64():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((6, 7, 8, 2))
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in cg.cnn_init(11)]
    Y64, _ = N.forward(params, X)
    Y16, _ = N.forward(params, X, emulate_bf16=True)
    e = np.linalg.norm(Y16 - Y64) / np.linalg.norm(Y64)
    assert 1e-5 < e <= 2.0**-5, e


def test_zero_last_layer_gives_zero_correction_and_judge_falls_back():
    import scipy.sparse as sp
    rng = np.random.default_rng(9)
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in cg.cnn_init(12)]
    params[-1] = (np.zeros_like(params[-1][0]), np.zeros_like(params[-1][1]))
    X = rng.standard_normal((3, 4, 5, 2))
    Y, _ = N.forward(params, X)
    assert not np.any(Y)
    A = sp.diags([np.full(60, 4.0), np.full(59, -1.0), np.full(59, -1.0)], [0, -1, 1]).tocsr()
    rp = rng.standard_normal(60)
    v = rng.standard_normal(60)
    x, used = N.judge(A, rp, v, Y.ravel())
    assert not used and np.array_equal(x, v)
    x, used = N.judge(A, rp, v, 0.5 * (np.linalg.solve(A.toarray(), rp) - v))
    assert used
