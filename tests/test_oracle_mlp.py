"""Pins of the prefetch network's oracle (oracle/or_mlp.c) on the CPU.

- one layer with one output is logistic regression: loss and gradient in
  closed form;
- the unrounded network against PyTorch autograd in float64 (an independent
  implementation of the same forward and backward);
- central finite differences of the oracle's own loss;
- the bf16-rounded forward against the same network evaluated by PyTorch
  with its own round-to-nearest-even bf16 casts at the same points;
- Adam against torch.optim.Adam.
"""
import math

import numpy as np
import pytest
import torch

import oracle


def _rand_params(dims, rng, scale=0.5):
    return (rng.standard_normal(oracle.mlp_n_params(dims)) * scale).astype(np.float32)


def _split(params, dims):
    out, o = [], 0
    for l in range(len(dims) - 1):
        din, dout = dims[l], dims[l + 1]
        W = params[o:o + din * dout].reshape(din, dout)
        o += din * dout
        b = params[o:o + dout]
        o += dout
        out.append((W, b))
    return out


def test_logistic_regression_closed_form():
    w = np.array([0.75, -1.25, 0.5], np.float32)     # W [2][1] then b [1]
    x = np.array([[2.0, 1.0]], np.float32)
    for y in (0.0, 1.0):
        loss, g, z = oracle.mlp_backward(w, [2, 1], x, np.array([[y]], np.float32), bf16=False)
        zz = 0.75 * 2.0 - 1.25 * 1.0 + 0.5
        s = 1.0 / (1.0 + math.exp(-zz))
        assert z[0, 0] == pytest.approx(zz, abs=1e-15)
        assert loss == pytest.approx(-(y * math.log(s) + (1 - y) * math.log(1 - s)), rel=1e-14)
        assert np.allclose(g, [(s - y) * 2.0, (s - y) * 1.0, s - y], rtol=1e-14, atol=0)


@pytest.mark.parametrize("dims,B", [([7, 6, 5, 4], 3), ([12, 8, 8, 8, 16], 5)])
def test_against_autograd(dims, B):
    rng = np.random.default_rng(1)
    p = _rand_params(dims, rng)
    x = rng.standard_normal((B, dims[0])).astype(np.float32)
    y = (rng.random((B, dims[-1])) < 0.3).astype(np.float32)
    loss, g, z = oracle.mlp_backward(p, dims, x, y, bf16=False)
    ts = [(torch.tensor(W, dtype=torch.float64, requires_grad=True), torch.tensor(b, dtype=torch.float64,
                                                                               requires_grad=True))
          for W, b in _split(p, dims)]
    h = torch.tensor(x, dtype=torch.float64)
    for l, (W, b) in enumerate(ts):
        h = h @ W + b
        if l + 1 < len(ts):
            h = torch.relu(h)
    tl = torch.nn.functional.binary_cross_entropy_with_logits(h, torch.tensor(y, dtype=torch.float64))
    tl.backward()
    tg = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy()]) for W, b in ts])
    assert np.allclose(z, h.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-14)


def test_finite_differences():
    dims, B = [6, 5, 4, 3], 4
    rng = np.random.default_rng(2)
    p = _rand_params(dims, rng)
    x = rng.standard_normal((B, dims[0])).astype(np.float32)
    y = (rng.random((B, dims[-1])) < 0.5).astype(np.float32)
    _, g, _ = oracle.mlp_backward(p, dims, x, y, bf16=False)
    h = 2.0 ** -12
    for i in rng.choice(p.size, 40, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += np.float32(h)
        pm[i] -= np.float32(h)
        hp, hm = float(pp[i]) - float(p[i]), float(p[i]) - float(pm[i])   # the steps float32 can take
        lp = oracle.mlp_backward(pp, dims, x, y, bf16=False)[0]
        lm = oracle.mlp_backward(pm, dims, x, y, bf16=False)[0]
        fd = (lp - lm) / (hp + hm)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_bf16_forward_against_torch_casts():
    dims, B = [20, 16, 16, 12], 6
    rng = np.random.default_rng(3)
    p = _rand_params(dims, rng)
    x = rng.standard_normal((B, dims[0])).astype(np.float32)
    z = oracle.mlp_forward(p, dims, x, bf16=True)

    def bf(a):
        return torch.as_tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64)

    h = bf(x)
    layers = _split(p, dims)
    for l, (W, b) in enumerate(layers):
        h = h @ bf(W) + torch.tensor(b, dtype=torch.float64)
        if l + 1 < len(layers):
            # the oracle takes a double activation to float32, then to bf16
            h = bf(torch.relu(h).to(torch.float32).numpy())
    assert np.allclose(z, h.numpy(), rtol=1e-6, atol=1e-6)
    # the rounded network stays close to the unrounded one
    z0 = oracle.mlp_forward(p, dims, x, bf16=False)
    assert np.abs(z - z0).max() < 0.05 * np.abs(z0).max()


def test_adam_against_torch():
    rng = np.random.default_rng(4)
    n = 257
    w0 = rng.standard_normal(n).astype(np.float32)
    w, m, v = w0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)
    tw = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(n)
        oracle.adam(w, m, v, g, 1e-2, 0.9, 0.999, 1e-8, t)
        tw.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        assert np.allclose(w, tw.detach().numpy(), rtol=1e-6, atol=1e-7), t
