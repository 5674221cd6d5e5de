"""Pins of the numpy neural-field oracle: finite differences, library routines."""
import math

import numpy as np
import pytest
import torch

import crp_inputs as I
from oracle import nf_oracle as N


def small_net(seed=0, width=16, depth=3, nfeat=5):
    rng = np.random.default_rng(seed)
    F = rng.integers(-4, 5, size=(nfeat, 3))
    ws, bs = [], []
    fan = 2 * nfeat
    for _ in range(depth):
        ws.append(rng.standard_normal((width, fan)) / math.sqrt(fan))
        bs.append(rng.standard_normal(width) * 0.1)
        fan = width
    ws.append(rng.standard_normal((3, fan)) / math.sqrt(fan))
    bs.append(rng.standard_normal(3) * 0.1)
    return F, ws, bs


def test_forward_backward_central_differences():
    F, ws, bs = small_net()
    rng = np.random.default_rng(1)
    x = rng.random((40, 3))
    y = rng.standard_normal((40, 3))
    out, cache = N.forward(ws, bs, x, F)
    gW, gb = N.backward(ws, cache, N.mse_grad(out, y))
    h = 1e-6
    for k in range(len(ws)):
        for (i, j) in [(0, 0), (1, 2), (ws[k].shape[0] - 1, ws[k].shape[1] - 1)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[k][i, j] += h
            wm[k][i, j] -= h
            fd = (N.mse_loss(N.forward(wp, bs, x, F)[0], y) -
                  N.mse_loss(N.forward(wm, bs, x, F)[0], y)) / (2 * h)
            assert abs(fd - gW[k][i, j]) <= 1e-6 * max(abs(fd), 1e-3)
        for i in (0, bs[k].shape[0] - 1):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[k][i] += h
            bm[k][i] -= h
            fd = (N.mse_loss(N.forward(ws, bp, x, F)[0], y) -
                  N.mse_loss(N.forward(ws, bm, x, F)[0], y)) / (2 * h)
            assert abs(fd - gb[k][i]) <= 1e-6 * max(abs(fd), 1e-3)


def test_forward_matches_torch_float64():
    F, ws, bs = small_net(2)
    x = np.random.default_rng(3).random((64, 3))
    out, _ = N.forward(ws, bs, x, F)
    xt = torch.tensor(x)
    ang = 2 * math.pi * xt @ torch.tensor(F, dtype=torch.float64).T
    a = torch.cat([torch.cos(ang), torch.sin(ang)], 1)
    for k, (w, b) in enumerate(zip(ws, bs)):
        a = torch.nn.functional.linear(a, torch.tensor(w), torch.tensor(b))
        if k < len(ws) - 1:
            a = torch.relu(a)
    assert np.allclose(out, a.numpy(), rtol=1e-13, atol=1e-13)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    v = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-8, 8, 100000)).astype(np.float32)
    v = np.concatenate([v, np.float32([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125])])
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.round_bf16(v.astype(np.float64)), ref)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = [rng.standard_normal((4, 3)), rng.standard_normal(4)]
    grads = [[rng.standard_normal(p.shape) for p in p0] for _ in range(5)]
    tp = [torch.tensor(p, requires_grad=True) for p in p0]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    params = [p.copy() for p in p0]
    m = [np.zeros_like(p) for p in p0]
    v = [np.zeros_like(p) for p in p0]
    for t, g in enumerate(grads, start=1):
        for tt, gg in zip(tp, g):
            tt.grad = torch.tensor(gg)
        opt.step()
        params, m, v = N.adam_step(params, g, m, v, t, 1e-2)
    for a, b in zip(params, tp):
        assert np.allclose(a, b.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_embedding_is_periodic_and_unit():
    F = I.nf_frequencies()
    assert F.shape == (64, 3) and F.dtype == np.int32
    mag = np.sqrt((F.astype(float) ** 2).sum(1))
    assert mag.min() >= 2 and mag.max() <= 16
    rng = np.random.default_rng(6)
    x = rng.random((100, 3))
    g0 = N.embed(x, F)
    g1 = N.embed(x + rng.integers(-3, 4, (100, 3)), F)
    assert np.allclose(g0, g1, atol=1e-11)
    assert np.allclose(g0[:, :64] ** 2 + g0[:, 64:] ** 2, 1.0)


def test_normalized_position_wraps():
    p = np.array([[-1.0, 0.0, 10.5], [3.0, 7.0, -0.25]])
    xh = N.normalized_position(p, (2, 2, 2), 2.0)
    assert np.allclose(xh, [[0.75, 0.0, 0.625], [0.75, 0.75, 0.9375]])


def test_flat_initial_parameters_follow_the_oracle_layout():
    """The input module's flat initial vector (used by the benchmark) is the
    oracle's flattening of the same weights."""
    import crp_inputs as I
    from oracle import nf_oracle as NO
    ws, bs = I.nf_init_weights(509)
    assert np.array_equal(I.nf_init_flat(509), NO.flatten(ws, bs).astype(np.float32))
