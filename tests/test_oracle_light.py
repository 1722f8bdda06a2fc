"""Pins of the oracle's Sersic light, grid, downsampling and PSF convolution.

Checks against properties the definitions must have: the effective-radius
contour, total flux by the incomplete-gamma closed form (integrated by
quadrature over the oracle's own 2-D profile), flux conservation of the
mean downsampling, a delta image convolved to the PSF itself with an
asymmetric kernel, and agreement with scipy's 2-D convolution.
"""
import math

import numpy as np
import pytest
import torch
from scipy import signal, special

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth

T = lambda v: torch.tensor(float(v), dtype=torch.float64)


def test_grid_centred_and_symmetric():
    for (nx, ny, s) in [(6, 4, 1), (5, 7, 2), (8, 8, 3), (3, 3, 4)]:
        X, Y = O.subpixel_grid(nx, ny, 0.05, s)
        assert X.shape == (ny * s, nx * s)
        assert abs(float(X.mean())) < 1e-15 and abs(float(Y.mean())) < 1e-15
        # sub-pixel block means are the pixel centres
        bx = X.reshape(ny, s, nx, s).mean(dim=(1, 3))
        xc = (np.arange(nx) - (nx - 1) / 2) * 0.05
        np.testing.assert_allclose(bx.numpy(), np.broadcast_to(xc, (ny, nx)), atol=1e-15)
        # uniform spacing pix/s
        np.testing.assert_allclose(np.diff(X[0].numpy()), 0.05 / s, rtol=1e-12)
        np.testing.assert_allclose(np.diff(Y[:, 0].numpy()), 0.05 / s, rtol=1e-12)


@pytest.mark.parametrize("n,e1,e2", [(0.7, 0.2, -0.1), (2.5, -0.3, 0.2), (4.0, 0.0, 0.3)])
def test_sersic_effective_radius_contour(n, e1, e2):
    """I = I_e on the R = R_e ellipse (axes R_e/sqrt(q), R_e sqrt(q))."""
    Re, Ie, xc, yc = 0.4, 0.77, 0.1, -0.2
    q, phi = O.ellipticity_to_q_phi(T(e1), T(e2))
    s = torch.linspace(0, 2 * math.pi, 50, dtype=torch.float64)
    xp, yp = Re / torch.sqrt(q) * torch.cos(s), Re * torch.sqrt(q) * torch.sin(s)
    cp, sp = torch.cos(phi), torch.sin(phi)
    x, y = xc + cp * xp - sp * yp, yc + sp * xp + cp * yp
    I = O.sersic(x, y, T(Re), T(n), T(e1), T(e2), T(xc), T(yc), T(Ie))
    np.testing.assert_allclose(I.numpy(), Ie, rtol=1e-13)


def test_sersic_special_indices():
    """n = 1/2 is a Gaussian in R, n = 1 an exponential in R (circular case)."""
    x = torch.linspace(0.01, 2.0, 40, dtype=torch.float64)
    y = torch.zeros_like(x)
    Re, Ie = 0.5, 1.3
    g = O.sersic(x, y, T(Re), T(0.5), T(0), T(0), T(0), T(0), T(Ie))
    lg = torch.log(g / Ie)
    # log I is linear in R^2 for a Gaussian
    A = np.vstack([np.ones(40), (x ** 2).numpy()]).T
    coef, res, *_ = np.linalg.lstsq(A, lg.numpy(), rcond=None)
    assert np.abs(A @ coef - lg.numpy()).max() < 1e-12
    e = O.sersic(x, y, T(Re), T(1.0), T(0), T(0), T(0), T(0), T(Ie))
    le = torch.log(e / Ie)
    A = np.vstack([np.ones(40), x.numpy()]).T
    coef, *_ = np.linalg.lstsq(A, le.numpy(), rcond=None)
    assert np.abs(A @ coef - le.numpy()).max() < 1e-12


def _sersic_total_flux_closed(Re, n, Ie):
    b = 1.9992 * n - 0.3271
    return 2 * math.pi * n * Re ** 2 * Ie * math.exp(b) * b ** (-2 * n) * math.gamma(2 * n)


def _polar_flux(Re, n, e1, e2, Ie, rmax, nr=600, nth=512):
    """Integral of the oracle's 2-D profile over the disk r < rmax by quadrature.

    Gauss-Legendre in log r (resolves the central cusp) x periodic trapezoid
    in angle; the disk r < rmin (rmin tiny) is added as I(0) pi rmin^2.
    """
    rmin = 1e-7
    xg, wg = np.polynomial.legendre.leggauss(nr)
    lo, hi = math.log(rmin), math.log(rmax)
    s = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
    ws = 0.5 * (hi - lo) * wg
    r = np.exp(s)
    th = np.linspace(0, 2 * math.pi, nth + 1)[:-1]
    R, TH = np.meshgrid(r, th, indexing="ij")
    x = torch.tensor(R * np.cos(TH)); y = torch.tensor(R * np.sin(TH))
    I = O.sersic(x, y, T(Re), T(n), T(e1), T(e2), T(0), T(0), T(Ie)).numpy()
    inner = (I * (R ** 2)).mean(axis=1) * 2 * math.pi  # d(log r): r dr = r^2 ds
    I0 = float(O.sersic(torch.zeros(1, dtype=torch.float64), torch.zeros(1, dtype=torch.float64),
                        T(Re), T(n), T(e1), T(e2), T(0), T(0), T(Ie))[0])
    return float((inner * ws).sum()) + I0 * math.pi * rmin ** 2


@pytest.mark.parametrize("n", [0.5, 1.0, 2.0, 4.0])
def test_sersic_aperture_flux_incomplete_gamma(n):
    """Circular case: flux inside r < Ra = closed form x P(2n, b (Ra/Re)^(1/n))."""
    Re, Ie = 0.3, 0.9
    b = 1.9992 * n - 0.3271
    for Ra in (0.1, 0.3, 1.0, 3.0):
        num = _polar_flux(Re, n, 0.0, 0.0, Ie, Ra)
        ref = _sersic_total_flux_closed(Re, n, Ie) * special.gammainc(2 * n, b * (Ra / Re) ** (1 / n))
        assert abs(num - ref) < 1e-7 * ref, (Ra, num, ref)


@pytest.mark.parametrize("n,e1,e2", [(0.6, 0.25, 0.1), (1.0, -0.2, 0.3), (1.5, 0.0, -0.4)])
def test_sersic_total_flux_is_independent_of_ellipticity(n, e1, e2):
    """Area-preserving radius: total flux equals the circular closed form."""
    Re, Ie = 0.2, 0.6
    q = (1 - math.hypot(e1, e2)) / (1 + math.hypot(e1, e2))
    rmax = 40 * Re / math.sqrt(q)     # flux outside is < 1e-12 for n <= 1.5
    num = _polar_flux(Re, n, e1, e2, Ie, rmax)
    ref = _sersic_total_flux_closed(Re, n, Ie)
    assert abs(num - ref) < 1e-7 * ref


def test_sersic_flux_on_fine_grid():
    """Riemann sum on a fine pixel grid also reproduces the closed form."""
    Re, n, Ie = 0.25, 1.0, 1.0
    X, Y = O.subpixel_grid(400, 400, 0.02, 2)
    I = O.sersic(X, Y, T(Re), T(n), T(0.15), T(-0.1), T(0.013), T(-0.021), T(Ie))
    num = float(I.sum()) * (0.01 ** 2)
    ref = _sersic_total_flux_closed(Re, n, Ie)
    assert abs(num - ref) < 2e-4 * ref


def test_downsample_conserves_flux_and_is_block_mean():
    rng = np.random.default_rng(9)
    for s in (1, 2, 3, 4):
        v = torch.tensor(rng.normal(size=(5 * s, 7 * s)))
        img = O.downsample(v, s)
        assert abs(float(img.sum()) - float(v.sum()) / s ** 2) < 1e-12
        brute = np.zeros((5, 7))
        vn = v.numpy()
        for i in range(5):
            for j in range(7):
                brute[i, j] = vn[i * s:(i + 1) * s, j * s:(j + 1) * s].mean()
        np.testing.assert_allclose(img.numpy(), brute, atol=1e-14)


@pytest.mark.parametrize("K", [3, 5, 11, 21])
def test_delta_image_convolves_to_the_psf(K):
    psf = synth.asymmetric_psf(K, synth.SEED_TEST_PSF)
    ny = nx = K + 9
    img = torch.zeros((ny, nx), dtype=torch.float64)
    i0, j0 = ny // 2 + 1, nx // 2 - 2
    img[i0, j0] = 1.0
    m = O.convolve_psf(img, psf).numpy()
    h = (K - 1) // 2
    np.testing.assert_allclose(m[i0 - h:i0 + h + 1, j0 - h:j0 + h + 1], psf.astype(np.float64), atol=0)
    mask = np.ones_like(m, dtype=bool)
    mask[i0 - h:i0 + h + 1, j0 - h:j0 + h + 1] = False
    assert np.all(m[mask] == 0.0)


@pytest.mark.parametrize("K,shape", [(3, (9, 12)), (11, (30, 25)), (21, (40, 40))])
def test_psf_matches_scipy_same_convolution(K, shape):
    rng = np.random.default_rng(10)
    psf = synth.asymmetric_psf(K, synth.SEED_TEST_PSF + K)
    img = rng.normal(size=shape)
    m = O.convolve_psf(torch.tensor(img), psf).numpy()
    ref = signal.convolve2d(img, psf.astype(np.float64), mode="same", boundary="fill")
    np.testing.assert_allclose(m, ref, atol=1e-13)


def test_constant_interior_is_scaled_by_psf_sum():
    K = 7
    psf = synth.asymmetric_psf(K, 3)
    img = torch.full((30, 30), 2.5, dtype=torch.float64)
    m = O.convolve_psf(img, psf).numpy()
    h = 3
    np.testing.assert_allclose(m[h:-h, h:-h], 2.5 * psf.astype(np.float64).sum(), rtol=1e-14)
