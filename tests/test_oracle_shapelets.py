"""Pins of the oracle's shapelet basis (Refregier 2003): Hermite polynomials
against numpy's, orthonormality of the 2-D basis by quadrature, the n = 0
function is the unit-norm Gaussian, the odd functions integrate to zero and
the even ones to their closed-form flux, and a source is the coefficient
sum."""
import math

import numpy as np
import torch
from numpy.polynomial import hermite as nph

from oracle import lens_oracle as O


def test_hermite_matches_numpy():
    x = torch.linspace(-3, 3, 41, dtype=torch.float64)
    for n in range(9):
        c = np.zeros(n + 1)
        c[n] = 1.0
        np.testing.assert_allclose(O.hermite_phys(n, x).numpy(), nph.hermval(x.numpy(), c), rtol=1e-12, atol=1e-9)


def test_basis_is_orthonormal():
    beta = 0.3
    g = torch.linspace(-3.0, 3.0, 601, dtype=torch.float64)
    h = float(g[1] - g[0])
    X, Y = torch.meshgrid(g, g, indexing="xy")
    B = O.shapelet_basis(X, Y, beta, 4).reshape(15, -1)
    G = (B @ B.T).numpy() * h * h
    np.testing.assert_allclose(G, np.eye(15), atol=1e-9)


def test_lowest_order_is_the_unit_norm_gaussian():
    x = torch.linspace(-1, 1, 21, dtype=torch.float64)
    beta = 0.25
    want = (math.pi ** -0.25) / math.sqrt(beta) * torch.exp(-0.5 * (x / beta) ** 2)
    np.testing.assert_allclose(O.shapelet_1d(0, x, beta).numpy(), want.numpy(), rtol=1e-14)


def test_one_dimensional_fluxes():
    beta = 0.4
    g = torch.linspace(-6.0, 6.0, 4001, dtype=torch.float64)
    h = float(g[1] - g[0])
    for n in range(8):
        f = float(O.shapelet_1d(n, g, beta).sum()) * h
        if n % 2:
            assert abs(f) < 1e-12
        else:
            # closed form: sqrt(2^(1-n) sqrt(pi) beta) sqrt(n!) / (n/2)!
            want = math.sqrt(2.0 ** (1 - n) * math.sqrt(math.pi) * beta) * math.sqrt(math.factorial(n)) \
                / math.factorial(n // 2)
            assert abs(f - want) < 1e-10, (n, f, want)


def test_source_is_the_coefficient_sum():
    rng = np.random.default_rng(2)
    c = rng.normal(size=10)                  # n_max = 3
    x = torch.tensor(rng.normal(size=50) * 0.3)
    y = torch.tensor(rng.normal(size=50) * 0.3)
    s = O.shapelet_source(x, y, 0.05, -0.02, 0.2, c)
    B = O.shapelet_basis(x - 0.05, y + 0.02, 0.2, 3)
    np.testing.assert_allclose(s.numpy(), (torch.tensor(c)[:, None] * B).sum(0).numpy(), rtol=1e-13)
