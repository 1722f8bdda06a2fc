"""Pins of the oracle's shapelet basis (Refregier 2003): Hermite polynomials
against numpy's, orthonormality of the 2-D basis by quadrature, the n = 0
function is the unit-norm Gaussian, the odd functions integrate to zero and
the even ones to their closed-form flux, and a source is the coefficient
sum.  A lensed shapelet source without deflection is the unlensed one; the
lensed image is linear in the coefficients, which a weighted least-squares
solve recovers from noiseless data (the backward use of shapelets)."""
import math

import numpy as np
import pytest
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


def _lens_case():
    from paper_2606_30633_amd import synth
    spec = synth.ModelSpec(20, 18, 0.12, 2, 5, synth.MASS_SIE, 1, 1)
    psf = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF)
    sysm = synth.make_system_box(spec, 0, psf=psf)
    return spec, psf, sysm


def test_lensed_shapelets_without_deflection_are_the_unlensed_source():
    spec, psf, sysm = _lens_case()
    th = np.array(sysm.truth, dtype=np.float64)
    th[0] = 1e-12                                  # theta_E -> 0: no mass deflection
    th[5], th[6] = 0.0, 0.0                        # no shear (SIE layout: theta_E, e1, e2, x, y, g1, g2)
    c = np.random.default_rng(3).normal(size=6)    # n_max = 2
    img = O.lensed_shapelet_image(th, spec, psf, 0.1, -0.05, 0.3, c)
    X, Y = O.subpixel_grid(spec.nx, spec.ny, spec.pix_scale, spec.supersample)
    want = O.convolve_psf(O.downsample(O.shapelet_source(X, Y, 0.1, -0.05, 0.3, c), spec.supersample), psf)
    # theta_E = 1e-12 leaves a deflection of that order: agreement to 1e-9 of the image's scale
    np.testing.assert_allclose(img.numpy(), want.numpy(), rtol=0, atol=1e-9 * float(want.abs().max()))


def test_lensed_shapelets_are_linear_and_recoverable_by_least_squares():
    spec, psf, sysm = _lens_case()
    rng = np.random.default_rng(4)
    th = np.array(sysm.truth, dtype=np.float64)
    c1, c2 = rng.normal(size=10), rng.normal(size=10)          # n_max = 3
    f = lambda c: O.lensed_shapelet_image(th, spec, psf, 0.02, 0.03, 0.15, c).numpy()
    np.testing.assert_allclose(f(c1 + 2 * c2), f(c1) + 2 * f(c2), rtol=1e-10, atol=1e-12)
    # backward use: the coefficients are the weighted least-squares solution on noiseless data
    B = np.stack([f(e) for e in np.eye(10)]).reshape(10, -1)
    w = sysm.invvar.reshape(-1).astype(np.float64)
    d = f(c1).reshape(-1)
    sol = np.linalg.solve((B * w) @ B.T, (B * w) @ d)
    np.testing.assert_allclose(sol, c1, rtol=1e-6, atol=1e-8)


def test_lensed_shapelet_gradient_matches_finite_differences():
    """Autograd through the lensed shapelet image (mass, shear, centre, scale)
    against central differences of a chi^2 on it: the derivative a shapelet
    adjoint would have to reproduce."""
    spec, psf, sysm = _lens_case()
    rng = np.random.default_rng(5)
    c = rng.normal(size=6)
    data = O.lensed_shapelet_image(sysm.truth, spec, psf, 0.02, 0.01, 0.2, c).numpy() + 0.01 * rng.normal(
        size=(spec.ny, spec.nx))

    def chi(v):
        t = torch.tensor(sysm.truth, dtype=torch.float64)
        t[:7] = v[:7]
        m = O.lensed_shapelet_image(t, spec, psf, v[7], v[8], v[9], c)
        return ((m - torch.tensor(data)) ** 2).sum()

    v0 = torch.cat([torch.tensor(sysm.truth[:7], dtype=torch.float64) * 1.01,
                    torch.tensor([0.025, 0.005, 0.21], dtype=torch.float64)]).requires_grad_(True)
    (g,) = torch.autograd.grad(chi(v0), v0)
    for j in range(10):
        h = 1e-6
        e = torch.zeros(10, dtype=torch.float64)
        e[j] = h
        fd = (float(chi(v0.detach() + e)) - float(chi(v0.detach() - e))) / (2 * h)
        assert abs(fd - float(g[j])) <= 1e-5 * float(g.abs().max()), (j, fd, float(g[j]))


# ---------------------------------------------------------------------------
# A shapelet source inside the parameter vector (spec.n_shapelet = 1): the
# layout, superposition with the Sersic model, the likelihood gradient by
# central differences, linear inversion of its coefficients, validity.
# ---------------------------------------------------------------------------
def _sh_case(nmax=3, mass="EPL", nl=1, ns=1):
    import dataclasses
    from paper_2606_30633_amd import synth
    base = synth.ModelSpec(22, 20, 0.1, 2, 5, mass, nl, ns)
    spec = dataclasses.replace(base, n_shapelet=1, shapelet_nmax=nmax)
    psf = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF)
    sysm = synth.make_system_box(base, 1, psf=psf)
    rng = np.random.default_rng(11 + nmax)
    nb = (nmax + 1) * (nmax + 2) // 2
    block = np.concatenate([[0.18, 0.03, -0.04], 0.5 * rng.normal(size=nb)])
    th = np.concatenate([np.asarray(sysm.truth, np.float64), block])
    return base, spec, psf, sysm, th


def test_shapelet_block_layout():
    base, spec, psf, sysm, th = _sh_case(4)
    assert O.n_params(spec) == O.n_params(base) + 3 + 15 == spec.n_params == len(spec.param_names())
    slots = O.intensity_slots(spec)
    assert slots[:2] == O.intensity_slots(base)
    assert slots[2:] == list(range(O.n_params(base) + 3, O.n_params(spec)))
    assert spec.param_names()[O.n_params(base)] == "sh_beta"


@pytest.mark.parametrize("nmax", [0, 3])
def test_model_is_the_sersic_model_plus_the_lensed_shapelet_source(nmax):
    base, spec, psf, sysm, th = _sh_case(nmax)
    d0 = O.n_params(base)
    m = O.model_image(th, spec, psf).numpy()
    m_base = O.model_image(th[:d0], base, psf).numpy()
    m_sh = O.lensed_shapelet_image(th[:d0], base, psf, th[d0 + 1], th[d0 + 2], th[d0], th[d0 + 3:]).numpy()
    np.testing.assert_allclose(m, m_base + m_sh, rtol=1e-12, atol=1e-14 * np.abs(m).max())
    # zero coefficients leave the Sersic model
    th0 = th.copy()
    th0[d0 + 3:] = 0.0
    np.testing.assert_allclose(O.model_image(th0, spec, psf).numpy(), m_base, rtol=1e-14, atol=0)


def test_loglike_gradient_with_shapelets_matches_finite_differences():
    base, spec, psf, sysm, th = _sh_case(3)
    data = (O.model_image(th * (1 + 1e-3), spec, psf).numpy() + sysm.noise).astype(np.float32)
    L, g = O.loglike_and_grad(th, spec, psf, data, sysm.invvar)
    d0 = O.n_params(base)
    for j in [0, 2, d0, d0 + 1, d0 + 2, d0 + 3, d0 + 7, d0 + 9]:
        h = 1e-6 * max(abs(th[j]), 1e-2)
        e = np.zeros_like(th)
        e[j] = h
        fd = (O.loglike(th + e, spec, psf, data, sysm.invvar) - O.loglike(th - e, spec, psf, data, sysm.invvar)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * (abs(g[j]) + np.abs(g).max()), (j, fd, g[j])


def test_backward_solves_the_shapelet_coefficients_and_intensities():
    base, spec, psf, sysm, th = _sh_case(3)
    data = O.model_image(th, spec, psf).numpy()            # noiseless
    L, g, A = O.loglike_backward(th, spec, psf, data, sysm.invvar)
    slots = O.intensity_slots(spec)
    assert A.shape == (len(slots),)
    np.testing.assert_allclose(A, th[slots], rtol=1e-6, atol=1e-8)
    assert -L < 1e-12 * float(np.sum(sysm.invvar * data ** 2))


def test_nonpositive_shapelet_scale_is_invalid():
    base, spec, psf, sysm, th = _sh_case(2)
    d0 = O.n_params(base)
    data = O.model_image(th, spec, psf).numpy()
    bad = th.copy()
    bad[d0] = 0.0
    assert O.loglike(bad, spec, psf, data, sysm.invvar) == -math.inf
    bad[d0] = -0.1
    assert O.loglike(bad, spec, psf, data, sysm.invvar) == -math.inf
