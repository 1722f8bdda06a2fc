"""Pins of the oracle's backward ("linear inversion") likelihood (Sec. 3:
intensities solved for instead of sampled).

- noiseless data: the solved intensities are the truth's and chi^2 = 0;
- the solved intensities maximise logL: the backward logL is at least the
  forward logL at any intensities and equals it at the solved ones;
- the intensities equal a weighted least-squares solve by numpy.linalg.lstsq;
- envelope theorem: the gradient through the solve equals the forward
  gradient at the solved intensities;
- central finite differences of the backward logL;
- a component with no flux in the image is left out (A = 0) and a duplicated
  component shares nothing (the later copy gets 0).
"""
import numpy as np
import torch

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth

SPEC = synth.ModelSpec(18, 16, 0.15, 2, 5, synth.MASS_EPL, 1, 2)


def _case(k=0, noise=True, spec=SPEC):
    psf = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF + k)
    sysm = synth.make_system_box(spec, k, psf=psf)
    model = O.model_image(sysm.truth, spec, psf).numpy()
    data = (model + (sysm.noise if noise else 0)).astype(np.float64)
    return sysm, psf, data


def _with_amps(theta, spec, A):
    t = np.array(theta, dtype=np.float64)
    t[O.intensity_slots(spec)] = A
    return t


def test_noiseless_recovers_truth_intensities():
    sysm, psf, data = _case(noise=False)
    L, _, A = O.loglike_backward(sysm.truth, SPEC, psf, data, sysm.invvar, with_grad=False)
    np.testing.assert_allclose(A, sysm.truth[O.intensity_slots(SPEC)], rtol=1e-9)
    assert abs(L) < 1e-12 * float(np.sum(sysm.invvar * data ** 2))


def test_solved_intensities_maximise_the_likelihood():
    sysm, psf, data = _case(1)
    rng = np.random.default_rng(3)
    th = synth.particles_box(sysm, 3, 1).astype(np.float64)
    for t in th:
        Lb, _, A = O.loglike_backward(t, SPEC, psf, data, sysm.invvar, with_grad=False)
        Lf = O.loglike(_with_amps(t, SPEC, A), SPEC, psf, data, sysm.invvar)
        assert abs(Lb - Lf) <= 1e-10 * abs(Lf)
        for _ in range(4):
            Ar = A * (1 + 0.1 * rng.standard_normal(A.shape))
            assert O.loglike(_with_amps(t, SPEC, Ar), SPEC, psf, data, sysm.invvar) <= Lb


def test_intensities_match_lstsq():
    sysm, psf, data = _case(2)
    t = synth.particles_box(sysm, 1, 2)[0].astype(np.float64)
    _, _, A = O.loglike_backward(t, SPEC, psf, data, sysm.invvar, with_grad=False)
    B = O.component_images(t, SPEC, psf).numpy().reshape(len(A), -1)
    sw = np.sqrt(sysm.invvar.reshape(-1).astype(np.float64))
    ref, *_ = np.linalg.lstsq((B * sw).T, data.reshape(-1) * sw, rcond=None)
    np.testing.assert_allclose(A, ref, rtol=1e-8)


def test_envelope_gradient_equals_forward_gradient_at_solution():
    sysm, psf, data = _case(3)
    for t in synth.particles_box(sysm, 2, 3).astype(np.float64):
        L, g, A = O.loglike_backward(t, SPEC, psf, data, sysm.invvar)
        Lf, gf = O.loglike_and_grad(_with_amps(t, SPEC, A), SPEC, psf, data, sysm.invvar)
        slots = O.intensity_slots(SPEC)
        assert np.all(g[slots] == 0)
        rest = np.setdiff1d(np.arange(len(t)), slots)
        np.testing.assert_allclose(g[rest], gf[rest], rtol=1e-7, atol=1e-9 * np.abs(gf[rest]).max())
        # and the forward gradient in the intensity entries vanishes there (optimality)
        assert np.abs(gf[slots]).max() <= 1e-7 * np.abs(gf).max()


def test_backward_gradient_matches_finite_differences():
    sysm, psf, data = _case(4)
    t = synth.particles_box(sysm, 1, 4)[0].astype(np.float64)
    L, g, _ = O.loglike_backward(t, SPEC, psf, data, sysm.invvar)
    for j in (0, 1, 3, 8, 9):
        h = 1e-6 * max(1.0, abs(t[j]))
        e = np.zeros_like(t)
        e[j] = h
        fp = O.loglike_backward(t + e, SPEC, psf, data, sysm.invvar, with_grad=False)[0]
        fm = O.loglike_backward(t - e, SPEC, psf, data, sysm.invvar, with_grad=False)[0]
        assert abs((fp - fm) / (2 * h) - g[j]) <= 1e-5 * np.abs(g).max(), j


def test_degenerate_components_are_left_out():
    spec = synth.ModelSpec(18, 16, 0.15, 2, 5, synth.MASS_EPL, 1, 2)
    sysm, psf, data = _case(5, spec=spec)
    t = np.array(sysm.truth, dtype=np.float64)
    # second source = copy of the first: its image is linearly dependent
    s1, s2 = O.intensity_slots(spec)[1] - 6, O.intensity_slots(spec)[2] - 6
    t[s2:s2 + 6] = t[s1:s1 + 6]
    L, g, A = O.loglike_backward(t, spec, psf, data, sysm.invvar)
    assert A[2] == 0 and np.isfinite(L) and np.all(np.isfinite(g))
    # a source far outside the cutout has no flux there
    t2 = np.array(sysm.truth, dtype=np.float64)
    t2[s2 + 4], t2[s2 + 5], t2[s2] = 80.0, 80.0, 0.05
    L2, g2, A2 = O.loglike_backward(t2, spec, psf, data, sysm.invvar)
    assert A2[2] == 0 and np.isfinite(L2) and np.all(np.isfinite(g2))


def test_backward_posterior_gradient_and_frozen_intensities():
    """The backward posterior in the unconstrained space: its gradient matches
    central differences and is zero in the intensity entries, whose values do
    not change it."""
    sysm, psf, data = _case(6)
    table = synth.prior_table(sysm.prior)
    t = synth.particles_box(sysm, 1, 6)[0].astype(np.float64)
    u = O.to_unconstrained(torch.tensor(t), table).numpy()
    for jac in (False, True):
        lp, g = O.log_posterior_backward(u, SPEC, psf, data, sysm.invvar, table, jac)
        slots = O.intensity_slots(SPEC)
        assert np.all(g[slots] == 0)
        u2 = u.copy()
        u2[slots] += 0.7
        assert abs(O.log_posterior_backward(u2, SPEC, psf, data, sysm.invvar, table, jac)[0] - lp) <= 1e-9 * abs(lp)
        for j in (0, 2, 9, 10):
            h = 1e-6
            e = np.zeros_like(u)
            e[j] = h
            fd = (O.log_posterior_backward(u + e, SPEC, psf, data, sysm.invvar, table, jac)[0]
                  - O.log_posterior_backward(u - e, SPEC, psf, data, sysm.invvar, table, jac)[0]) / (2 * h)
            assert abs(fd - g[j]) <= 1e-5 * np.abs(g).max(), (jac, j, fd, g[j])


def test_hmc_zero_inverse_mass_freezes_a_coordinate():
    cov = np.array([[1.0, 0.3], [0.3, 0.5]])
    P = np.linalg.inv(cov)
    f = lambda u: (-0.5 * u[:2] @ P @ u[:2], np.concatenate([-(P @ u[:2]), [0.0]]))
    u = np.array([0.1, -0.2, 3.0])
    for t in range(20):
        u, *_ = O.hmc_transition(u, f, np.array([1.0, 1.0, 0.0]), 0.3, 4, 5, 0, t)
        assert u[2] == 3.0 and np.all(np.isfinite(u))
