"""Pins for the oracle's learned-preconditioner pieces.

Forward and backward are checked against torch's CPU convolution and
autograd in float64 (library routines), the backward also against central
finite differences, the bfloat16 rounding against torch's own cast, and Adam
against its closed form on the first step.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2406_19754_amd import problems as P

C = 16


def split(p):
    if not isinstance(p, torch.Tensor):
        p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    o = 0
    out = []
    for shape in [(C, 1, 3, 3, 3), (C,), (C, C, 3, 3, 3), (C,), (1, C, 3, 3, 3), (1,)]:
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    assert o == p.numel()
    return out


def torch_net(p, u, rnd):
    W1, b1, W2, b2, W3, b3 = split(p)
    bf = (lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)) if rnd else (lambda t: t)
    if rnd:
        W1, W2, W3 = bf(W1), bf(W2), bf(W3)
    x = bf(u)[:, None]
    h1 = bf(F.gelu(F.conv3d(x, W1, b1, padding=1)))
    h2 = bf(F.gelu(F.conv3d(h1, W2, b2, padding=1)))
    return F.conv3d(h2, W3, b3, padding=1)[:, 0]


def rand_params(seed, scale=1.0):
    p = P.net_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    p += 0.05 * rng.standard_normal(p.size)     # non-zero biases too
    return p * scale


def test_bf16_rounding_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-5, 5, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1e-40, 3.4e38, -2.5]])
    ref = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16(x), ref)


@pytest.mark.parametrize("rnd", [False, True])
def test_forward_matches_torch_conv3d(rnd):
    p = rand_params(1)
    u = np.random.default_rng(2).standard_normal((2, 5, 6, 7))
    out = oracle.net_forward(p, u, round_bf16=rnd)
    ref = torch_net(p, torch.tensor(u), rnd).numpy()
    if rnd:
        # identical operands; only the bf16 decision on intermediate sums can differ
        assert np.abs(out - ref).max() <= 2e-2 * np.abs(ref).max()
        assert np.mean(np.abs(out - ref) <= 1e-12 * np.abs(ref).max()) > 0.9
    else:
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_backward_matches_autograd_and_finite_differences():
    p = rand_params(3, scale=0.7)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((2, 6, 6, 6))
    y = rng.standard_normal((2, 6, 6, 6))
    margin = 1
    loss, g = oracle.net_loss_grad(p, u, y, margin, round_bf16=False)
    # autograd reference
    pt = torch.tensor(p, requires_grad=True)
    out = torch_net(pt, torch.tensor(u), False)
    sl = (slice(None),) + (slice(margin, -margin),) * 3
    lt = ((out[sl] - torch.tensor(y)[sl]) ** 2).mean()
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * abs(loss)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=0, atol=1e-10 * np.abs(g).max())
    # central finite differences on a sample of parameters from every group
    idx = np.concatenate([rng.choice(432, 8, replace=False), 432 + rng.choice(16, 3, replace=False),
                          448 + rng.choice(6912, 12, replace=False), 7360 + rng.choice(16, 3, replace=False),
                          7376 + rng.choice(432, 8, replace=False), [7808]])
    h = 1e-5
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = oracle.net_loss_grad(pp, u, y, margin, round_bf16=False)
        lm, _ = oracle.net_loss_grad(pm, u, y, margin, round_bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_backward_with_rounding_is_straight_through():
    p = rand_params(5, scale=0.7)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((1, 5, 5, 5))
    y = rng.standard_normal((1, 5, 5, 5))
    l0, g0 = oracle.net_loss_grad(p, u, y, 1, round_bf16=False)
    l1, g1 = oracle.net_loss_grad(p, u, y, 1, round_bf16=True)
    assert abs(l1 - l0) <= 0.05 * l0
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(7)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m1, v1 = oracle.adam_step(p0, m, v, g, 1, lr=1e-3)
    # bias-corrected moments equal g and g^2 on the first step
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected moments at g, g^2
    p2, _, _ = oracle.adam_step(p1, m1, v1, g, 2, lr=1e-3)
    np.testing.assert_allclose(p2, p1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_net_apply_is_scale_equivariant_and_zero_net_falls_back():
    n = 8
    p = rand_params(8, scale=0.5)
    r = np.random.default_rng(9).standard_normal(n ** 3)
    z1 = oracle.net_apply(p, r, (n, n, n))
    z2 = oracle.net_apply(p, 7.0 * r, (n, n, n))
    np.testing.assert_allclose(z2, 7.0 * z1, rtol=1e-13, atol=1e-13 * np.abs(z2).max())
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(n ** 3, 1)
    zero = np.zeros(oracle.net_param_count())
    f = h.fcg(b, rtol=1e-6, params=zero, dims=(n, n, n))
    base = h.fcg(b, rtol=1e-6)
    assert f["status"] == oracle.OK and f["fallbacks"] >= 1
    # z = 0 fails z.r > 0 every time: two such steps in a row switch the
    # network off, later scheduled steps count as fallbacks without it
    assert f["net_evals"] == 2 and f["fallbacks"] == f["iters"] // 2
    # every network step fell back, so the iterates are the plain V-cycle ones
    assert f["iters"] == base["iters"]
    np.testing.assert_allclose(f["x"], base["x"], rtol=0, atol=1e-12 * np.abs(base["x"]).max())
