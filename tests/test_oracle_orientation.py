"""Pin of the ellipticity orientation of every elliptical profile in the oracle.

Sec. 3 parametrises each elliptical component by two eccentricities (e1, e2).
The reading adopted (the usual convention of lens-modelling codes) puts the
major axis at the position angle phi = atan2(e2, e1) / 2, counted
counter-clockwise from +x: e = (c, 0) -> 0 deg, (0, c) -> 45 deg,
(-c, 0) -> 90 deg, (0, -c) -> 135 deg.

These tests never call the oracle's own angle code (ellipticity_to_q_phi,
to_frame, from_frame).  They look at what the profiles produce: on a circle
around the component centre, the convergence of the mass model (half the
divergence of its deflection, by central differences) and the Sersic surface
brightness are largest where the circle crosses the major axis.  A brute-force
search over angles locates that maximum.  A half-angle slip, swapped e1/e2 or
a reversed rotation moves it to another angle, which the second group of
tests plants in a copy of the oracle's frame code to show.
"""
import math

import numpy as np
import pytest
import torch

from oracle import lens_oracle as O

T = lambda v: torch.tensor(float(v), dtype=torch.float64)

C = 0.3
CASES = [((C, 0.0), 0.0), ((0.0, C), 45.0), ((-C, 0.0), 90.0), ((0.0, -C), 135.0)]
X0, Y0 = 0.13, -0.07
RADIUS = 0.6
STEP_DEG = 0.25


def _circle():
    ang = torch.arange(0.0, 360.0, STEP_DEG, dtype=torch.float64)
    a = ang * math.pi / 180.0
    return ang, X0 + RADIUS * torch.cos(a), Y0 + RADIUS * torch.sin(a)


def _axis_of_max(ang, val):
    """Angle in [0, 180) of the largest value (the two maxima are 180 deg apart)."""
    return float(ang[int(torch.argmax(val))]) % 180.0


def _angle_error(a, b):
    d = abs(a - b) % 180.0
    return min(d, 180.0 - d)


def _kappa_on_circle(deflect):
    ang, x, y = _circle()
    h = 1e-5
    axp, _ = deflect(x + h, y)
    axm, _ = deflect(x - h, y)
    _, ayp = deflect(x, y + h)
    _, aym = deflect(x, y - h)
    return ang, 0.5 * (axp - axm + ayp - aym) / (2 * h)


def _epl_axis(e1, e2, gamma):
    f = lambda x, y: O.epl_deflection(x, y, T(1.1), T(gamma), T(e1), T(e2), T(X0), T(Y0))
    return _axis_of_max(*_kappa_on_circle(f))


def _sie_axis(e1, e2):
    f = lambda x, y: O.sie_deflection(x, y, T(1.1), T(e1), T(e2), T(X0), T(Y0))
    return _axis_of_max(*_kappa_on_circle(f))


def _sersic_axis(e1, e2):
    ang, x, y = _circle()
    I = O.sersic(x, y, T(0.4), T(1.7), T(e1), T(e2), T(X0), T(Y0), T(1.0))
    return _axis_of_max(ang, I)


def _all_errors():
    errs = []
    for (e1, e2), want in CASES:
        for got in (_epl_axis(e1, e2, 1.7), _epl_axis(e1, e2, 2.3), _sie_axis(e1, e2), _sersic_axis(e1, e2)):
            errs.append(_angle_error(got, want))
    return errs


@pytest.mark.parametrize("e,want", CASES)
def test_epl_major_axis(e, want):
    for gamma in (1.6, 2.0, 2.4):
        assert _angle_error(_epl_axis(*e, gamma), want) <= STEP_DEG, gamma


@pytest.mark.parametrize("e,want", CASES)
def test_sie_major_axis(e, want):
    assert _angle_error(_sie_axis(*e), want) <= STEP_DEG


@pytest.mark.parametrize("e,want", CASES)
def test_sersic_major_axis(e, want):
    assert _angle_error(_sersic_axis(*e), want) <= STEP_DEG


def test_intermediate_angle():
    """A general ellipticity: the axis follows atan2(e2, e1) / 2 (here 60 deg)."""
    c, pa = 0.25, 60.0
    e1, e2 = c * math.cos(math.radians(2 * pa)), c * math.sin(math.radians(2 * pa))
    assert _angle_error(_epl_axis(e1, e2, 2.1), pa) <= STEP_DEG
    assert _angle_error(_sersic_axis(e1, e2), pa) <= STEP_DEG


def test_axis_ratio_from_isophote():
    """The Sersic isophote through the major-axis point at radius a reaches
    the minor axis at a q, with q = (1 - c)/(1 + c) (Sec. 3 eccentricity)."""
    e1, e2 = 0.0, C
    q = (1 - C) / (1 + C)
    d_major = torch.tensor([math.cos(math.pi / 4), math.sin(math.pi / 4)], dtype=torch.float64)
    d_minor = torch.tensor([-math.sin(math.pi / 4), math.cos(math.pi / 4)], dtype=torch.float64)
    a = 0.5
    Ia = O.sersic(T(X0 + a * d_major[0]), T(Y0 + a * d_major[1]), T(0.4), T(1.7), T(e1), T(e2), T(X0), T(Y0), T(1.0))
    lo, hi = 0.0, a
    for _ in range(80):   # bisection along the minor axis for the same brightness
        mid = 0.5 * (lo + hi)
        Im = O.sersic(T(X0 + mid * d_minor[0]), T(Y0 + mid * d_minor[1]), T(0.4), T(1.7), T(e1), T(e2),
                      T(X0), T(Y0), T(1.0))
        if float(Im) > float(Ia):
            lo = mid
        else:
            hi = mid
    assert abs(0.5 * (lo + hi) / a - q) < 1e-12


# --- the same checks fail on plausible mistakes planted in the frame code ---------

def _planted_errors(monkeypatch, q_phi=None, frame=None, back=None):
    with monkeypatch.context() as mp:
        if q_phi is not None:
            mp.setattr(O, "ellipticity_to_q_phi", q_phi)
        if frame is not None:
            mp.setattr(O, "to_frame", frame)
        if back is not None:
            mp.setattr(O, "from_frame", back)
        return _all_errors()


def test_correct_oracle_passes_all():
    assert max(_all_errors()) <= STEP_DEG


def test_planted_full_angle_fails(monkeypatch):
    def q_phi(e1, e2):
        c = torch.sqrt(e1 * e1 + e2 * e2)
        return (1 - c) / (1 + c), torch.atan2(e2, e1)
    assert max(_planted_errors(monkeypatch, q_phi=q_phi)) > 20.0


def test_planted_swapped_components_fails(monkeypatch):
    def q_phi(e1, e2):
        c = torch.sqrt(e1 * e1 + e2 * e2)
        return (1 - c) / (1 + c), 0.5 * torch.atan2(e1, e2)
    assert max(_planted_errors(monkeypatch, q_phi=q_phi)) > 20.0


def test_planted_reversed_rotation_fails(monkeypatch):
    def frame(x, y, x0, y0, phi):
        dx, dy = x - x0, y - y0
        cp, sp = torch.cos(phi), torch.sin(phi)
        return cp * dx - sp * dy, sp * dx + cp * dy

    def back(ax, ay, phi):
        cp, sp = torch.cos(phi), torch.sin(phi)
        return cp * ax + sp * ay, -sp * ax + cp * ay
    assert max(_planted_errors(monkeypatch, frame=frame, back=back)) > 20.0
    # the frame rotation reversed alone (deflection rotated back correctly)
    assert max(_planted_errors(monkeypatch, frame=frame)) > 20.0
