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


def exact_case():
    rng = np.random.default_rng(11)
    img = rng.integers(0, 5, size=(EXACT_BATCH, 64, 64)) * 0.25
    tgt = rng.integers(-4, 5, size=(EXACT_BATCH, C.NT)) * 0.25
    return sparse_int_params(12), img, tgt
