"""Pins of the oracle's lens-mass model against closed forms and invariants.

None of these re-types the oracle's formula: each checks a property that the
elliptical power law / SIE / shear must have (Sec. 3 names the mass model):
the SIS and spherical power-law deflections, the isothermal closed form at
gamma = 2, the Poisson equation div(alpha) = 2 kappa, zero curl, the mass
normalisation of theta_E, and the independent 1-D integral representation of
elliptical lenses (Schramm 1990; Keeton 2001).
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import lens_oracle as O

T = lambda v: torch.tensor(float(v), dtype=torch.float64)


def _pts(n=200, seed=1, lo=-2.5, hi=2.5):
    rng = np.random.default_rng(seed)
    x = torch.tensor(rng.uniform(lo, hi, n), dtype=torch.float64)
    y = torch.tensor(rng.uniform(lo, hi, n), dtype=torch.float64)
    return x, y


def test_sis_deflection_magnitude_is_theta_E():
    x, y = _pts()
    for tE in (0.8, 1.3, 1.8):
        ax, ay = O.epl_deflection(x, y, T(tE), T(2.0), T(0.0), T(0.0), T(0.0), T(0.0))
        mag = torch.sqrt(ax * ax + ay * ay)
        np.testing.assert_allclose(mag.numpy(), tE, rtol=1e-14)
        # radial, pointing away from the centre
        r = torch.sqrt(x * x + y * y)
        np.testing.assert_allclose((ax * x + ay * y).numpy(), (tE * r).numpy(), rtol=1e-13)


@pytest.mark.parametrize("gamma", [1.5, 1.8, 2.3, 2.5])
def test_spherical_power_law(gamma):
    x, y = _pts(seed=2)
    x0, y0, tE = 0.07, -0.04, 1.2
    ax, ay = O.epl_deflection(x, y, T(tE), T(gamma), T(0.0), T(0.0), T(x0), T(y0))
    dx, dy = x - x0, y - y0
    r = torch.sqrt(dx * dx + dy * dy)
    t = gamma - 1.0
    mag = tE * (tE / r) ** (t - 1.0)
    np.testing.assert_allclose(ax.numpy(), (mag * dx / r).numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ay.numpy(), (mag * dy / r).numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("e1,e2", [(0.2, 0.0), (-0.1, 0.25), (0.3, -0.3), (0.0, 0.05), (0.45, 0.2)])
def test_epl_at_gamma_2_equals_sie_closed_form(e1, e2):
    x, y = _pts(seed=3)
    args = (T(1.1), T(e1), T(e2), T(0.05), T(-0.08))
    ax_s, ay_s = O.sie_deflection(x, y, *args)
    ax_e, ay_e = O.epl_deflection(x, y, args[0], T(2.0), *args[1:])
    np.testing.assert_allclose(ax_e.numpy(), ax_s.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(ay_e.numpy(), ay_s.numpy(), rtol=1e-12, atol=1e-13)


def _kappa(x, y, tE, gamma, e1, e2, x0, y0):
    q, phi = O.ellipticity_to_q_phi(T(e1), T(e2))
    xp, yp = O.to_frame(x, y, T(x0), T(y0), phi)
    R = torch.sqrt(q * q * xp * xp + yp * yp)
    t = gamma - 1.0
    b = tE * torch.sqrt(q)
    return (2.0 - t) / 2.0 * (b / R) ** t


@pytest.mark.parametrize("gamma,e1,e2", [(1.6, 0.2, 0.1), (2.0, -0.3, 0.2), (2.4, 0.1, -0.35), (1.9, 0.4, 0.0)])
def test_poisson_equation_and_zero_curl(gamma, e1, e2):
    """div alpha = 2 kappa and d(alpha_x)/dy = d(alpha_y)/dx (central FD, FP64)."""
    x, y = _pts(n=60, seed=4, lo=-2.0, hi=2.0)
    keep = torch.sqrt(x * x + y * y) > 0.3
    x, y = x[keep], y[keep]
    p = (T(1.3), T(gamma), T(e1), T(e2), T(0.03), T(-0.02))
    h = 1e-5
    axp, _ = O.epl_deflection(x + h, y, *p)
    axm, _ = O.epl_deflection(x - h, y, *p)
    _, ayp = O.epl_deflection(x, y + h, *p)
    _, aym = O.epl_deflection(x, y - h, *p)
    div = (axp - axm + ayp - aym) / (2 * h)
    kap = _kappa(x, y, 1.3, gamma, e1, e2, 0.03, -0.02)
    np.testing.assert_allclose(div.numpy(), (2 * kap).numpy(), rtol=2e-7)
    ax_yp, _ = O.epl_deflection(x, y + h, *p)
    ax_ym, _ = O.epl_deflection(x, y - h, *p)
    _, ay_xp = O.epl_deflection(x + h, y, *p)
    _, ay_xm = O.epl_deflection(x - h, y, *p)
    curl = (ax_yp - ax_ym - ay_xp + ay_xm) / (2 * h)
    assert float(curl.abs().max()) < 1e-7 * float(kap.abs().max())


@pytest.mark.parametrize("gamma,e1,e2", [(1.5, 0.3, 0.0), (2.0, 0.1, 0.2), (2.5, -0.2, -0.25)])
def test_theta_E_normalisation_flux_through_ellipse(gamma, e1, e2):
    """Outward flux of alpha through the R = b ellipse equals 2 pi theta_E^2.

    By Gauss' theorem that is twice the mass inside, i.e. the mean
    convergence inside the ellipse of area pi theta_E^2 is exactly 1.
    """
    tE = 1.37
    q, phi = O.ellipticity_to_q_phi(T(e1), T(e2))
    b = tE * math.sqrt(float(q))
    s = torch.linspace(0, 2 * math.pi, 4097, dtype=torch.float64)[:-1]
    xp, yp = b / q * torch.cos(s), b * torch.sin(s)
    cp, sp = torch.cos(phi), torch.sin(phi)
    x, y = cp * xp - sp * yp, sp * xp + cp * yp
    ax, ay = O.epl_deflection(x, y, T(tE), T(gamma), T(e1), T(e2), T(0.0), T(0.0))
    # rotate deflection into the ellipse frame
    axr, ayr = cp * ax + sp * ay, -sp * ax + cp * ay
    dxp, dyp = -b / q * torch.sin(s), b * torch.cos(s)
    flux = float((axr * dyp - ayr * dxp).mean()) * 2 * math.pi
    assert abs(flux - 2 * math.pi * tE ** 2) < 1e-10 * 2 * math.pi * tE ** 2


def _keeton_deflection(xp, yp, tE, gamma, q):
    """Schramm/Keeton 1-D integrals for kappa constant on x^2 + y^2/q^2 ellipses."""
    t = gamma - 1.0
    b = tE * math.sqrt(q)
    pref = (2.0 - t) / 2.0 * (b / q) ** t

    def J(n):
        f = lambda u: pref * (xp * xp + yp * yp / (1.0 - (1.0 - q * q) * u)) ** (-t / 2.0) \
            / (1.0 - (1.0 - q * q) * u) ** (n + 0.5)
        val, err = integrate.quad(f, 0.0, 1.0, weight="alg", wvar=(-t / 2.0, 0.0),
                                  epsabs=0.0, epsrel=1e-13, limit=200)
        return val

    return q * xp * J(0), q * yp * J(1)


@pytest.mark.parametrize("gamma,e1", [(1.5, 0.3), (1.8, 0.1), (2.2, 0.4), (2.5, 0.25)])
def test_epl_matches_elliptical_integral_representation(gamma, e1):
    x, y = _pts(n=25, seed=5, lo=-2.0, hi=2.0)
    tE = 1.21
    ax, ay = O.epl_deflection(x, y, T(tE), T(gamma), T(e1), T(0.0), T(0.0), T(0.0))
    q = (1 - e1) / (1 + e1)
    for k in range(len(x)):
        kx, ky = _keeton_deflection(float(x[k]), float(y[k]), tE, gamma, q)
        assert abs(float(ax[k]) - kx) < 1e-9 * (abs(kx) + 1e-3)
        assert abs(float(ay[k]) - ky) < 1e-9 * (abs(ky) + 1e-3)


def test_series_truncation_converged():
    x, y = _pts(n=500, seed=6)
    p = (T(1.2), T(1.7), T(0.42), T(-0.2), T(0.0), T(0.1))
    ax, ay, used = O.epl_deflection(x, y, *p, return_terms=True)
    ax2, ay2 = O.epl_deflection(x, y, *p, n_terms=2 * used)
    scale = float(torch.sqrt(ax * ax + ay * ay).max())
    assert float((ax - ax2).abs().max()) < 1e-15 * scale
    assert float((ay - ay2).abs().max()) < 1e-15 * scale


def test_sie_round_limit_is_sis():
    x, y = _pts(seed=7)
    ax, ay = O.sie_deflection(x, y, T(1.4), T(1e-9), T(0.0), T(0.0), T(0.0))
    np.testing.assert_allclose(torch.sqrt(ax * ax + ay * ay).numpy(), 1.4, rtol=1e-8)


def test_shear_is_trace_free_and_linear():
    x, y = _pts(seed=8)
    g1, g2 = 0.07, -0.03
    ax, ay = O.shear_deflection(x, y, T(g1), T(g2))
    # Jacobian by finite differences: [[g1, g2], [g2, -g1]]
    h = 1e-3
    axh, ayh = O.shear_deflection(x + h, y, T(g1), T(g2))
    axv, ayv = O.shear_deflection(x, y + h, T(g1), T(g2))
    J = np.array([[float((axh - ax)[0]) / h, float((axv - ax)[0]) / h],
                  [float((ayh - ay)[0]) / h, float((ayv - ay)[0]) / h]])
    np.testing.assert_allclose(J, [[g1, g2], [g2, -g1]], atol=1e-12)
    assert abs(np.trace(J)) < 1e-12
    # zero at the origin
    z = torch.zeros(1, dtype=torch.float64)
    a0 = O.shear_deflection(z, z, T(g1), T(g2))
    assert float(a0[0]) == 0.0 and float(a0[1]) == 0.0
