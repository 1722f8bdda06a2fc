"""Float64 CPU oracle of the learned initializer's network.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg); shares no
code with the HIP kernels and imports nothing from the product.

The network (not from the paper; the initializer proposes starting particles
for the multi-start MAP stage of Sec. 3): input 64x64 (one channel); six
3x3 convolutions, padding 1, ReLU, channels 32-32-64-64-128-128, strides
1-2-1-2-1-2; global average pooling; dense 128 -> 256 (ReLU) -> 28
(14 means and 14 log-variances).  Loss: mean over the batch of
sum_k [(z_k - mu_k)^2 exp(-s_k) + s_k] / 2.

Arithmetic: every contraction in float64 (torch conv2d / conv2d_input /
conv2d_weight and matmul as library primitives) on operands rounded to bf16
(round to nearest even) at the points where the GPU kernels round: inputs,
weights, each layer's output, the pooled features, the hidden layer, the
output gradient, and the gradients passed between layers.  ``rounding=False``
turns every rounding off (then the manual backward equals autograd).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64
CHANNELS = [32, 32, 64, 64, 128, 128]
STRIDES = [1, 2, 1, 2, 1, 2]
C6, H1, NT = 128, 256, 14
OUT = 2 * NT


def layout() -> List[Tuple[str, Tuple[int, ...]]]:
    """(name, shape) of the flat parameter vector, in order."""
    out = []
    cin = 1
    for l, c in enumerate(CHANNELS):
        out.append((f"conv{l}.w", (c, 3, 3, cin)))
        out.append((f"conv{l}.b", (c,)))
        cin = c
    out += [("fc1.w", (H1, C6)), ("fc1.b", (H1,)), ("fc2.w", (OUT, H1)), ("fc2.b", (OUT,))]
    return out


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in layout()))


def unflatten(flat) -> Dict[str, torch.Tensor]:
    flat = torch.as_tensor(np.asarray(flat, dtype=np.float64))
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d: Dict[str, torch.Tensor]) -> np.ndarray:
    return np.concatenate([d[name].reshape(-1).numpy() for name, _ in layout()])


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    f = x.to(torch.float32).contiguous()
    u = f.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = torch.where(torch.isnan(f), u, r)
    r32 = torch.where(r >= 2 ** 31, r - 2 ** 32, r).to(torch.int32)
    return r32.view(torch.float32).to(DT)


def _r(x, on):
    return bf16(x) if on else x


def forward(params, img_bf16, rounding: bool = True):
    """Network output [B, 28] (float64) and the cached activations.

    img_bf16: [B, 64, 64] (values already bf16, e.g. from ``bf16``).
    """
    P = unflatten(params)
    x = torch.as_tensor(np.asarray(img_bf16, dtype=np.float64))[:, None]     # NCHW
    acts = [x]
    for l, s in enumerate(STRIDES):
        w = _r(P[f"conv{l}.w"], rounding).permute(0, 3, 1, 2)                  # [co, ci, 3, 3]
        z = F.conv2d(acts[-1], w, P[f"conv{l}.b"], stride=s, padding=1)
        acts.append(_r(torch.relu(z), rounding))
    pooled = _r(acts[-1].mean(dim=(2, 3)), rounding)
    hid = _r(torch.relu(pooled @ _r(P["fc1.w"], rounding).T + P["fc1.b"]), rounding)
    out = hid @ _r(P["fc2.w"], rounding).T + P["fc2.b"]
    return out, {"acts": acts, "pooled": pooled, "hidden": hid}


def nll(out, target):
    """Mean over the batch of sum_k [(z - mu)^2 e^{-s} + s] / 2 and its gradient."""
    out = torch.as_tensor(out, dtype=DT)
    z = torch.as_tensor(np.asarray(target, dtype=np.float64))
    mu, s = out[:, :NT], out[:, NT:]
    B = out.shape[0]
    e = torch.exp(-s)
    L = (0.5 * (z - mu) ** 2 * e + 0.5 * s).sum() / B
    d = torch.cat([-(z - mu) * e / B, 0.5 * (1 - (z - mu) ** 2 * e) / B], dim=1)
    return float(L), d


def loss_and_grad(params, img_bf16, target, rounding: bool = True):
    """Loss and gradient w.r.t. the flat parameters (manual backward)."""
    P = unflatten(params)
    out, c = forward(params, img_bf16, rounding)
    L, dout = nll(out, target)
    dout = _r(dout, rounding)
    g: Dict[str, torch.Tensor] = {}
    hid, pooled, acts = c["hidden"], c["pooled"], c["acts"]
    g["fc2.w"] = dout.T @ hid
    g["fc2.b"] = dout.sum(0)
    dh = _r((dout @ _r(P["fc2.w"], rounding)) * (hid > 0), rounding)
    g["fc1.w"] = dh.T @ pooled
    g["fc1.b"] = dh.sum(0)
    dpool = dh @ _r(P["fc1.w"], rounding)                                      # not rounded
    a6 = acts[-1]
    hw = a6.shape[2] * a6.shape[3]
    dz = _r((dpool[:, :, None, None] / hw).expand_as(a6) * (a6 > 0), rounding)
    for l in range(len(STRIDES) - 1, -1, -1):
        xin = acts[l]
        w = _r(P[f"conv{l}.w"], rounding).permute(0, 3, 1, 2)
        gw = torch.nn.grad.conv2d_weight(xin, w.shape, dz, stride=STRIDES[l], padding=1)
        g[f"conv{l}.w"] = gw.permute(0, 2, 3, 1)
        g[f"conv{l}.b"] = dz.sum(dim=(0, 2, 3))
        if l > 0:
            dx = torch.nn.grad.conv2d_input(xin.shape, w, dz, stride=STRIDES[l], padding=1)
            dz = _r(dx * (xin > 0), rounding)
    return L, flatten(g), out.numpy()


def asinh_transform(img, sigma: float) -> np.ndarray:
    """Network input: asinh(x / (3 sigma)) rounded to bf16."""
    x = torch.as_tensor(np.asarray(img, dtype=np.float64))
    return bf16(torch.asinh(x / (3.0 * sigma))).numpy()
