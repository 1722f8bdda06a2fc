"""Seeded inputs for the learned initializer's network tests (no arithmetic
of the method): sparse {-1, 0, 1} weights and quarter-integer images, for
which every partial sum of the network is exact in fp32."""
import numpy as np

from oracle import cnn_oracle as C

EXACT_BATCH = 8
EXACT_DENSITY = 0.02


def sparse_int_params(seed, density=EXACT_DENSITY):
    """Weights in {-1, 0, 1} (sparse), zero biases, zero log-variance rows."""
    rng = np.random.default_rng(seed)
    p = np.zeros(C.n_params())
    o = 0
    for name, shape in C.layout():
        n = int(np.prod(shape))
        if name.endswith(".w"):
            w = rng.choice([-1.0, 0.0, 1.0], size=n, p=[density / 2, 1 - density, density / 2]).reshape(shape)
            if name == "fc2.w":
                w[C.NT:] = 0.0
            p[o:o + n] = w.reshape(-1)
        o += n
    return p


def exact_case(batch=EXACT_BATCH):
    rng = np.random.default_rng(11 if batch == EXACT_BATCH else 11 + batch)
    img = rng.integers(0, 5, size=(batch, 64, 64)) * 0.25
    tgt = rng.integers(-4, 5, size=(batch, C.NT)) * 0.25
    return sparse_int_params(12), img, tgt


def gradient_term_scale(params, img, target):
    """Per parameter entry, the sum of the absolute values of the terms whose
    sum is that entry of the loss gradient (weight gradients: |input| times
    |upstream gradient| summed over the batch and positions; biases: the sum
    of |upstream gradient|), with the oracle's own activations and upstream
    gradients.  On the exact fixture those intermediates are exact on both
    sides, so the only difference left is the float rounding of these final
    sums, bounded relative to this scale."""
    import torch
    P = C.unflatten(params)
    out, c = C.forward(params, img)
    _, dout = C.nll(out, target)
    dout = C.bf16(dout)
    hid, pooled, acts = c["hidden"], c["pooled"], c["acts"]
    W = lambda k: C.bf16(P[k])
    env = {"fc2.w": dout.abs().T @ hid.abs(), "fc2.b": dout.abs().sum(0)}
    dh = C.bf16((dout @ W("fc2.w")) * (hid > 0))
    env["fc1.w"] = dh.abs().T @ pooled.abs()
    env["fc1.b"] = dh.abs().sum(0)
    dpool = dh @ W("fc1.w")
    a6 = acts[-1]
    dz = C.bf16((dpool[:, :, None, None] / (a6.shape[2] * a6.shape[3])).expand_as(a6) * (a6 > 0))
    for l in range(len(C.STRIDES) - 1, -1, -1):
        xin = acts[l]
        w = W(f"conv{l}.w").permute(0, 3, 1, 2)
        env[f"conv{l}.w"] = torch.nn.grad.conv2d_weight(xin.abs(), w.shape, dz.abs(), stride=C.STRIDES[l],
                                                        padding=1).permute(0, 2, 3, 1)
        env[f"conv{l}.b"] = dz.abs().sum(dim=(0, 2, 3))
        if l > 0:
            dz = C.bf16(torch.nn.grad.conv2d_input(xin.shape, w, dz, stride=C.STRIDES[l], padding=1) * (xin > 0))
    return C.flatten(env)
