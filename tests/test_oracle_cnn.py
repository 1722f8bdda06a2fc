"""Pins of the network oracle: bf16 rounding, manual backward vs autograd,
finite differences, and the Gaussian NLL gradient."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C

import cnn_cases


def test_parameter_count():
    # 6 convolutions 286432 + dense 33024 + dense 7196
    assert C.n_params() == 326652


def test_bf16_rounding_nearest_even():
    x = torch.tensor([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e38, 1e-40],
                     dtype=torch.float64)
    r = C.bf16(x).numpy()
    # ties to even: 1 + 2^-8 -> 1 ; 1 + 3*2^-8 -> 1 + 2^-6 ; below half -> down
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == 1.0 and r[4] == -2.5
    ref = torch.tensor(x.numpy(), dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(r, ref)
    y = torch.randn(10000, dtype=torch.float64) * 10
    np.testing.assert_array_equal(C.bf16(y).numpy(),
                                  y.to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy())


def _rand(seed, B=3):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=0.04, size=C.n_params())
    img = rng.normal(size=(B, 64, 64))
    tgt = rng.normal(size=(B, C.NT))
    return p, img, tgt


def test_manual_backward_equals_autograd_without_rounding():
    p, img, tgt = _rand(1)
    L, g, out = C.loss_and_grad(p, img, tgt, rounding=False)
    pt = torch.tensor(p, requires_grad=True)
    P = {}
    o = 0
    for name, shape in C.layout():
        n = int(np.prod(shape))
        P[name] = pt[o:o + n].reshape(shape)
        o += n
    x = torch.tensor(img)[:, None]
    for l, s in enumerate(C.STRIDES):
        x = torch.relu(torch.nn.functional.conv2d(x, P[f"conv{l}.w"].permute(0, 3, 1, 2), P[f"conv{l}.b"],
                                                  stride=s, padding=1))
    h = torch.relu(x.mean(dim=(2, 3)) @ P["fc1.w"].T + P["fc1.b"])
    out2 = h @ P["fc2.w"].T + P["fc2.b"]
    z = torch.tensor(tgt)
    mu, sv = out2[:, :C.NT], out2[:, C.NT:]
    L2 = (0.5 * (z - mu) ** 2 * torch.exp(-sv) + 0.5 * sv).sum() / img.shape[0]
    L2.backward()
    assert abs(L - float(L2)) < 1e-12 * abs(L)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_loss_gradient_finite_differences():
    p, img, tgt = _rand(2, B=2)
    L, g, _ = C.loss_and_grad(p, img, tgt, rounding=False)
    rng = np.random.default_rng(3)
    for j in rng.choice(len(p), 12, replace=False).tolist() + [len(p) - 1, len(p) - 30]:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (C.loss_and_grad(pp, img, tgt, False)[0] - C.loss_and_grad(pm, img, tgt, False)[0]) / (2 * h)
        # truncation O(h^2) plus round-off of the loss difference, ~ 1e-16 |L| / h
        assert abs(fd - g[j]) <= 1e-6 * abs(g[j]) + 1e-9 * max(1.0, abs(L)), (j, fd, g[j])


def test_nll_stationarity_conditions():
    # d/ds = 0 at s = log (z - mu)^2 for any mu; d/dmu = 0 at mu = z for any s
    z = np.full((2, C.NT), 0.3)
    out = torch.zeros((2, C.OUT), dtype=torch.float64)
    out[:, :C.NT] = 0.8
    out[:, C.NT:] = float(np.log(0.25))
    _, d = C.nll(out, z)
    assert torch.abs(d[:, C.NT:]).max() < 1e-15
    assert torch.all(d[:, :C.NT] > 0)            # mu above z: gradient pushes it down
    out[:, :C.NT] = 0.3
    out[:, C.NT:] = 1.7
    _, d = C.nll(out, z)
    assert torch.abs(d[:, :C.NT]).max() < 1e-15


def _finest_unit(t):
    a = t.abs()
    a = a[a > 0]
    return float((2.0 ** (torch.floor(torch.log2(a)) - 7)).min())


@pytest.mark.parametrize("batch", [cnn_cases.EXACT_BATCH, 64, 256])
def test_exact_fixture_partial_sums_fit_fp32(batch):
    """The sparse-integer fixture used for the bitwise kernel comparison:
    every forward and data-gradient sum, bounded by the sum of absolute
    terms, stays below 2^24 times the finest unit of its bf16 operands, so
    any summation order gives the exact value in fp32."""
    import torch.nn.functional as F
    p, img, tgt = cnn_cases.exact_case(batch)
    P = C.unflatten(p)
    out, c = C.forward(p, img)
    acts = c["acts"]
    for l, s in enumerate(C.STRIDES):
        x = acts[l]
        w = C.bf16(P[f"conv{l}.w"]).permute(0, 3, 1, 2)
        bound = F.conv2d(x.abs(), w.abs(), None, stride=s, padding=1)
        assert float(bound.max()) < 2.0 ** 24 * _finest_unit(x), l
    _, dout = C.nll(out, tgt)
    dout = C.bf16(dout)
    w2, w1 = C.bf16(P["fc2.w"]), C.bf16(P["fc1.w"])
    assert float((dout.abs() @ w2.abs()).max()) < 2.0 ** 24 * _finest_unit(dout)
    dh = C.bf16((dout @ w2) * (c["hidden"] > 0))
    assert float((dh.abs() @ w1.abs()).max()) < 2.0 ** 24 * _finest_unit(dh)
    a6 = acts[-1]
    dz = C.bf16(((dh @ w1)[:, :, None, None] / 64).expand_as(a6) * (a6 > 0))
    for l in range(len(C.STRIDES) - 1, 0, -1):
        xin = acts[l]
        w = C.bf16(P[f"conv{l}.w"]).permute(0, 3, 1, 2)
        bound = torch.nn.grad.conv2d_input(xin.shape, w.abs(), dz.abs(), stride=C.STRIDES[l], padding=1)
        assert float(bound.max()) < 2.0 ** 24 * _finest_unit(dz), l
        dz = C.bf16(torch.nn.grad.conv2d_input(xin.shape, w, dz, stride=C.STRIDES[l], padding=1) * (xin > 0))
    assert float(dz.abs().max()) > 0
