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
    x, alpha = N.judge(A, rp, v, Y.ravel())
    assert alpha == 0.0 and np.array_equal(x, v)
    # half the exact error: the minimal-residual multiple is exactly 2 and the
    # corrected result is the exact solution
    xs = np.linalg.solve(A.toarray(), rp)
    x, alpha = N.judge(A, rp, v, 0.5 * (xs - v))
    assert alpha == pytest.approx(2.0, rel=1e-12)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    # a correction pointing the wrong way is never used
    x, alpha = N.judge(A, rp, v, -(xs - v))
    assert alpha == 0.0 and np.array_equal(x, v)
    # any other correction: the residual after the judge never exceeds the
    # V-cycle's, and equals the closed-form minimum over alpha
    c = rng.standard_normal(60)
    x, alpha = N.judge(A, rp, v, c)
    u, w = rp - A @ v, A @ c
    best = np.sqrt(max(u @ u - max(u @ w, 0.0) ** 2 / (w @ w), 0.0))
    assert np.linalg.norm(rp - A @ x) == pytest.approx(best, rel=1e-10)
    assert np.linalg.norm(rp - A @ x) <= np.linalg.norm(u)


def test_weighted_loss_gradient_matches_finite_differences():
    """The A_pp-weighted loss (the residual a correction would leave, on the
    voxels whose stencil lies inside the crop): its gradient with respect to
    the network output against central differences, and with respect to the
    weights through the same back-propagation as the MSE."""
    rng = np.random.default_rng(10)
    shape = (4, 5, 6)
    coef = rng.standard_normal((7,) + shape)
    coef[3] = 6.0 + np.abs(coef[3])
    Y = rng.standard_normal(shape + (1,))
    T = rng.standard_normal(shape)
    g = N.weighted_loss_grad(Y, coef, T)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (3, 4, 5), (2, 1, 0), (1, 1, 1)]:
        Yp, Ym = Y.copy(), Y.copy()
        Yp[idx + (0,)] += h
        Ym[idx + (0,)] -= h
        fd = (N.weighted_loss(Yp, coef, T) - N.weighted_loss(Ym, coef, T)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-9)
    # the loss is the MSE of A (y - t) on interior voxels: zero at y = t, and
    # with unit diagonal coefficients and no couplings it is the interior MSE
    assert N.weighted_loss(T[..., None], coef, T) == 0.0
    I = np.zeros((7,) + shape)
    I[3] = 1.0
    m = N.interior_mask(shape)
    assert N.weighted_loss(Y, I, T) == pytest.approx(np.mean((Y[..., 0] - T)[m] ** 2), rel=1e-14)
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in cg.cnn_init(13, last_scale=1.0)]
    X = rng.standard_normal(shape + (2,))
    Yn, cache = N.forward(params, X)
    grads = N.backward_weighted(params, cache, Yn, coef, T)
    l, q, pos = 3, 0, (5, 2, 0)
    Wp = [(W.copy(), b.copy()) for W, b in params]
    Wm = [(W.copy(), b.copy()) for W, b in params]
    Wp[l][q][pos] += h
    Wm[l][q][pos] -= h
    fd = (N.weighted_loss(N.forward(Wp, X)[0], coef, T) - N.weighted_loss(N.forward(Wm, X)[0], coef, T)) / (2 * h)
    assert fd == pytest.approx(grads[l][q][pos], rel=1e-5)
