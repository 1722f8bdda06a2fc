"""GPU parity: liblens.so (through the C ABI) against the FP64 oracle.

Tolerances (1e-5 relative, FP32 GPU vs FP64 oracle), per particle:
  images   max|dm| <= 1e-5 max|m_ref|
  logL     |dL| <= 1e-5 |L_ref| + B, where B = 2 sum w |d - m| |m| 2^-23 bounds the
           effect of storing the model image in float32 (one ulp) on the
           residual sum; it matters only near the optimum (B << 1e-5 |L| for
           prior draws)
  gradient prior draws: ||dg||_2 <= 1e-5 ||g_ref||_2;
           all checked particles, per component:
           |dg_j| <= 1e-5 (|g_ref,j| + S_j), S_j = sum_pix |r dm/dtheta_j|
           (near the optimum g -> 0 and only this scale-aware form is meaningful)
Inputs are the seeded generators' float32 arrays; the oracle evaluates the
same float32 values promoted to float64.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth
from tests.cases import make_case

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_30633_amd import lens  # noqa: E402

DEV = "cuda"
RTOL = 1e-5


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _plan(spec, psf, data, invvar, maxp):
    return lens.LensPlan(spec, psf, data, invvar, maxp, DEV)


def _fp32_bound(th, spec, psf, data, invvar):
    m = O.model_image(th, spec, psf).numpy()
    return 2.0 * float(np.sum(invvar * np.abs(data - m) * np.abs(m))) * 2.0 ** -23


def check_images(spec, psf, th, img_gpu):
    for p in range(th.shape[0]):
        ref = O.model_image(th[p], spec, psf).numpy()
        err = np.abs(img_gpu[p].astype(np.float64) - ref).max()
        assert err <= RTOL * np.abs(ref).max(), (p, err, np.abs(ref).max())


def check_loglike(spec, psf, data, invvar, th, L_gpu, idx=None):
    idx = range(th.shape[0]) if idx is None else idx
    for p in idx:
        ref = O.loglike(th[p], spec, psf, data, invvar)
        tol = RTOL * abs(ref) + _fp32_bound(th[p], spec, psf, data, invvar)
        assert abs(float(L_gpu[p]) - ref) <= tol, (p, float(L_gpu[p]), ref, tol)


def check_grad(spec, psf, data, invvar, th, G_gpu, idx=None, near=()):
    """Every checked particle, every component: |dg_j| <= 1e-5 (|g_j| + S_j);
    prior draws (not in ``near``) also in L2: ||dg|| <= 1e-5 ||g||.

    Near the optimum (indices in ``near``) the gradient is a small sum of large
    terms and only the scale-aware per-component form is meaningful.
    """
    idx = list(range(th.shape[0]) if idx is None else idx)
    for p in sorted(set(idx) | set(near)):
        _, g = O.loglike_and_grad(th[p], spec, psf, data, invvar)
        dg = G_gpu[p].astype(np.float64) - g
        if p not in near:
            assert np.linalg.norm(dg) <= RTOL * np.linalg.norm(g), (p, np.linalg.norm(dg) / np.linalg.norm(g))
        S = O.gradient_scale(th[p], spec, psf, data, invvar)
        bad = np.abs(dg) > RTOL * (np.abs(g) + S)
        assert not bad.any(), (p, np.nonzero(bad), dg[bad], g[bad], S[bad])


# ---------------------------------------------------------------------------
# Parity workload: 60x60, s = 2, SIE + shear, Sersic lens + source, 11x11
# Gaussian PSF (FWHM 0.1"), 64 uniform prior draws (+ 4 near the truth)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1():
    spec = synth.config1_spec()
    sysm, psf, data, th = make_case(spec, 0, 64, psf="gauss", near_truth=4)
    plan = _plan(spec, psf, data, sysm.invvar, th.shape[0])
    return spec, sysm, psf, data, th, plan


def test_config1_forward_images(c1):
    spec, sysm, psf, data, th, plan = c1
    _log("config1 forward: P=%d" % th.shape[0])
    img = lens.lens_forward(plan, torch.tensor(th, device=DEV)).cpu().numpy()
    check_images(spec, psf, th, img)


def test_config1_loglike(c1):
    spec, sysm, psf, data, th, plan = c1
    L = lens.lens_loglike(plan, torch.tensor(th, device=DEV)).cpu().numpy()
    check_loglike(spec, psf, data, sysm.invvar, th, L)


@pytest.fixture(scope="module")
def c1_grad(c1):
    spec, sysm, psf, data, th, plan = c1
    L, G, L64 = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV), want_logl64=True)
    return L.cpu().numpy(), G.cpu().numpy(), L64.cpu().numpy()


def test_config1_loglike_grad(c1, c1_grad):
    spec, sysm, psf, data, th, plan = c1
    L, G, L64 = c1_grad
    check_loglike(spec, psf, data, sysm.invvar, th, L)
    check_loglike(spec, psf, data, sysm.invvar, th, L64)


@pytest.mark.parametrize("block", range(4))
def test_config1_gradient_every_component(c1, c1_grad, block):
    """All 64 prior draws and the 4 near-truth particles, per component (in
    four blocks of 17 particles to keep each test short)."""
    spec, sysm, psf, data, th, plan = c1
    _, G, _ = c1_grad
    idx = range(17 * block, 17 * block + 17)
    check_grad(spec, psf, data, sysm.invvar, th, G, idx=idx, near=[p for p in idx if p >= 64])


# ---------------------------------------------------------------------------
# Headline workload at full size, in the benchmark's launch configuration:
# 100x100, s = 3, EPL + shear, Sersic lens, 2 Sersic sources, 21x21 PSF,
# 4096 particles; sampled particles checked one by one against the oracle.
# ---------------------------------------------------------------------------
def test_config2_full_size_sampled():
    spec = synth.config2_spec()
    sysm, psf, data, _ = make_case(spec, 0, 1, psf="double")
    th = synth.particles_box(sysm, 4096, 0)
    rng = np.random.default_rng(5)
    near = sysm.truth[None, :] * (1 + 1e-3 * rng.standard_normal((2, spec.n_params)))
    th[-2:] = near.astype(np.float32)
    _log("config2 full size: P=4096")
    plan = _plan(spec, psf, data, sysm.invvar, 4096)
    tt = torch.tensor(th, device=DEV)
    L, G = lens.lens_loglike_grad(plan, tt)
    L2 = lens.lens_loglike(plan, tt)
    img = lens.lens_forward(plan, tt[:8])
    torch.cuda.synchronize()
    L, G, L2, img = L.cpu().numpy(), G.cpu().numpy(), L2.cpu().numpy(), img.cpu().numpy()
    assert np.array_equal(L, L2), "logL from the gradient path differs from the logL path"
    sample = [0, 1, 777, 2048, 4093, 4094, 4095]
    check_loglike(spec, psf, data, sysm.invvar, th, L, idx=sample)
    check_grad(spec, psf, data, sysm.invvar, th, G, idx=sample[:5], near=[4094, 4095])
    check_images(spec, psf, th[:3], img[:3])
    assert np.all(np.isfinite(L)) and np.all(np.isfinite(G))


# ---------------------------------------------------------------------------
# Shapes: ragged tiles, non-square images, s = 1..4, K = 1..31, component
# counts, both mass models
# ---------------------------------------------------------------------------
SHAPES = [
    synth.ModelSpec(37, 23, 0.09, 1, 5, "EPL", 1, 1),
    synth.ModelSpec(21, 30, 0.12, 4, 3, "SIE", 0, 1),
    synth.ModelSpec(45, 45, 0.07, 2, 1, "EPL", 2, 3),
    synth.ModelSpec(33, 29, 0.11, 3, 31, "EPL", 3, 2),
    synth.ModelSpec(50, 50, 0.08, 2, 13, "SIE", 1, 3),
    synth.ModelSpec(17, 61, 0.10, 2, 9, "EPL", 0, 2),
]


@pytest.mark.parametrize("spec", SHAPES, ids=lambda s: f"{s.nx}x{s.ny}s{s.supersample}K{s.psf_size}{s.mass_model}{s.n_lens_light}{s.n_source}")
def test_shapes(spec):
    _log(f"shape case {spec}")
    sysm, psf, data, th = make_case(spec, 3, 5, psf="asym", near_truth=1)
    plan = _plan(spec, psf, data, sysm.invvar, th.shape[0])
    tt = torch.tensor(th, device=DEV)
    img = lens.lens_forward(plan, tt).cpu().numpy()
    L, G = lens.lens_loglike_grad(plan, tt)
    check_images(spec, psf, th, img)
    check_loglike(spec, psf, data, sysm.invvar, th, L.cpu().numpy())
    check_grad(spec, psf, data, sysm.invvar, th, G.cpu().numpy(), idx=[0, 1], near=[5])


def test_largest_supported_size():
    spec = synth.ModelSpec(160, 160, 0.05, 4, 31, "EPL", 1, 1)
    _log(f"largest case {spec}")
    sysm, psf, data, th = make_case(spec, 4, 2, psf="double")
    plan = _plan(spec, psf, data, sysm.invvar, 2)
    L, G = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
    check_loglike(spec, psf, data, sysm.invvar, th, L.cpu().numpy())
    check_grad(spec, psf, data, sysm.invvar, th, G.cpu().numpy())


# ---------------------------------------------------------------------------
# Degenerate inputs and the launch contract
# ---------------------------------------------------------------------------
def test_single_particle_and_invalid_and_nonfinite():
    spec = synth.ModelSpec(24, 24, 0.1, 2, 5, "EPL", 1, 1)
    sysm, psf, data, th = make_case(spec, 5, 4)
    th = th.copy()
    th[1, 2], th[1, 3] = 0.9, 0.6           # |e_mass| > 1
    th[2, 8 + 2] = 1.2                      # |e_light| > 1
    th[3, 5] = np.nan
    plan = _plan(spec, psf, data, sysm.invvar, 4)
    L, G = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
    L, G = L.cpu().numpy(), G.cpu().numpy()
    assert L[1] == -math.inf and L[2] == -math.inf and np.all(G[1:3] == 0)
    assert math.isnan(L[3]) and np.all(np.isnan(G[3]))
    check_loglike(spec, psf, data, sysm.invvar, th, L, idx=[0])
    L1 = lens.lens_loglike(plan, torch.tensor(th[:1], device=DEV)).cpu().numpy()
    assert L1[0] == L[0]


def test_round_mass_and_near_round_light():
    """Tiny ellipticities: the gradient stays accurate as |e| -> 0."""
    spec = synth.ModelSpec(30, 30, 0.1, 2, 5, "EPL", 1, 1)
    sysm, psf, data, th = make_case(spec, 6, 3)
    th = th.copy()
    th[0, 2:4] = [1e-4, -2e-4]
    th[1, 2:4] = [3e-3, 1e-3]
    th[2, 8 + 2: 8 + 4] = [2e-4, 1e-4]
    plan = _plan(spec, psf, data, sysm.invvar, 3)
    L, G = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
    check_loglike(spec, psf, data, sysm.invvar, th, L.cpu().numpy())
    check_grad(spec, psf, data, sysm.invvar, th, G.cpu().numpy())


def test_bitwise_deterministic_and_tiling_independent():
    spec = synth.ModelSpec(64, 64, 0.06, 3, 11, "EPL", 1, 2)
    sysm, psf, data, th = make_case(spec, 7, 64)
    plan = _plan(spec, psf, data, sysm.invvar, 64)
    tt = torch.tensor(th, device=DEV)
    a = [t.clone() for t in lens.lens_loglike_grad(plan, tt)]
    b = lens.lens_loglike_grad(plan, tt)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for ppt in (1, 3, 16):
        plan.set_pixels_per_thread(ppt)
        c = lens.lens_loglike_grad(plan, tt)
        assert torch.equal(a[0], c[0])          # logL does not depend on the sub-pixel tiling
        torch.testing.assert_close(c[1], a[1], rtol=2e-6, atol=1e-6 * float(a[1].abs().max()))


def test_argument_errors():
    spec = synth.ModelSpec(16, 16, 0.1, 2, 3, "SIE", 1, 1)
    sysm, psf, data, th = make_case(spec, 8, 2)
    plan = _plan(spec, psf, data, sysm.invvar, 2)
    big = torch.zeros((3, spec.n_params), device=DEV)
    with pytest.raises(lens.LensError) as e:
        lens.lens_loglike(plan, big)
    assert e.value.status == lens.LENS_EINVAL
    # empty input: zero particles is an argument error on every entry point
    empty = torch.zeros((0, spec.n_params), device=DEV)
    for fn in (lens.lens_forward, lens.lens_loglike, lens.lens_loglike_grad):
        with pytest.raises(lens.LensError) as e:
            fn(plan, empty)
        assert e.value.status == lens.LENS_EINVAL
    # a plan stays usable after rejected calls
    L = lens.lens_loglike(plan, torch.tensor(th, device=DEV)).cpu().numpy()
    check_loglike(spec, psf, data, sysm.invvar, th, L)
    big_spec = synth.ModelSpec(2049, 16, 0.05, 1, 3, "EPL", 1, 1)    # side above LENS_MAX_SIDE
    with pytest.raises(lens.LensError) as e:
        lens.LensPlan(big_spec, np.ones((3, 3), np.float32), np.zeros((16, 2049), np.float32),
                      np.ones((16, 2049), np.float32), 1, DEV)
    assert e.value.status == lens.LENS_EINVAL


def test_autograd_function():
    spec = synth.ModelSpec(20, 20, 0.12, 2, 5, "EPL", 1, 1)
    sysm, psf, data, th = make_case(spec, 9, 3)
    plan = _plan(spec, psf, data, sysm.invvar, 3)
    x = torch.tensor(th, device=DEV, requires_grad=True)
    L = lens.LensLogLike.apply(x, plan)
    w = torch.tensor([1.0, -2.0, 0.5], device=DEV)
    (L * w).sum().backward()
    _, G = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
    torch.testing.assert_close(x.grad, w[:, None] * G)


@pytest.mark.parametrize("mass", ["EPL", "SIE"])
def test_high_ellipticity_series(mass):
    """Mass ellipticities |e| from 0.3 to 0.85, on and off the real axis of the
    series variable: covers both float32 series forms of the adjoint (switch
    at |e| = 0.55) and the long float64 series."""
    spec = synth.ModelSpec(40, 40, 0.06, 2, 7, mass, 1, 1)
    sysm, psf, data, th = make_case(spec, 8, 10)
    th = th.copy()
    o = 2 if mass == "EPL" else 1
    for p, (c, ang) in enumerate([(0.3, 0.0), (0.5, 0.4), (0.54, 0.0), (0.56, 0.0), (0.6, 1.2),
                                  (0.7, 0.0), (0.7, 2.5), (0.8, 0.7), (0.85, 0.0), (0.85, 3.0)]):
        th[p, o:o + 2] = [c * math.cos(ang), c * math.sin(ang)]
    _log(f"high ellipticity {mass}")
    plan = _plan(spec, psf, data, sysm.invvar, th.shape[0])
    tt = torch.tensor(th, device=DEV)
    check_images(spec, psf, th, lens.lens_forward(plan, tt).cpu().numpy())
    L, G = lens.lens_loglike_grad(plan, tt)
    check_loglike(spec, psf, data, sysm.invvar, th, L.cpu().numpy())
    check_grad(spec, psf, data, sysm.invvar, th, G.cpu().numpy())
