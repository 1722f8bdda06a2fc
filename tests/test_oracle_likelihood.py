"""Pins of the oracle's likelihood, gradient, prior/bijection, Adam, HMC, RNG.

- logL is the Gaussian log-density up to a parameter-independent constant
  (scipy.stats.norm), its noise-only chi-square follows chi2(N_pix), and the
  noiseless truth is a zero-gradient maximum.
- autograd gradients agree with central finite differences in FP64.
- prior densities match scipy.stats; the bijection round-trips and its
  log-Jacobian matches finite differences.
- Adam matches torch.optim.Adam; leapfrog is reversible with O(eps^2)
  energy error and HMC reproduces Gaussian moments.
- Philox matches numpy.random.Philox (4x64) and published 4x32 answers.
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, stats

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth

SMALL_EPL = synth.ModelSpec(16, 16, 0.15, 2, 5, synth.MASS_EPL, 1, 2)
SMALL_SIE = synth.ModelSpec(14, 12, 0.18, 3, 3, synth.MASS_SIE, 1, 1)


def _system(spec, k=0):
    psf = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF + k)
    sysm = synth.make_system_box(spec, k, psf=psf)
    model = O.model_image(sysm.truth, spec, psf).numpy()
    data = (model + sysm.noise).astype(np.float32)
    return sysm, psf, model, data


def test_loglike_is_gaussian_logpdf_up_to_constant():
    spec = SMALL_EPL
    sysm, psf, model, data = _system(spec)
    th = synth.particles_box(sysm, 3, 5)
    sigma = 1.0 / np.sqrt(sysm.invvar.astype(np.float64))
    const = float(np.sum(np.log(sigma * math.sqrt(2 * math.pi))))
    for t in th:
        L = O.loglike(t, spec, psf, data, sysm.invvar)
        m = O.model_image(t, spec, psf).numpy()
        ref = stats.norm.logpdf(data.astype(np.float64), loc=m, scale=sigma).sum()
        assert abs((L - ref) - const) < 1e-9 * abs(ref)


def test_noise_only_chi2_follows_chi2_distribution():
    spec = synth.ModelSpec(20, 20, 0.12, 2, 5, synth.MASS_SIE, 1, 1)
    sysm, psf, model, _ = _system(spec)
    m = torch.tensor(model)
    npix = spec.nx * spec.ny
    vals = []
    for k in range(400):
        nz = synth.noise((spec.ny, spec.nx), synth.SIGMA_NOISE, 777 + k)
        vals.append(float(O.chi2(m, model + nz.astype(np.float64), sysm.invvar)))
    vals = np.array(vals)
    # mean N (+- 4 sigma of the sample mean) and variance 2N
    assert abs(vals.mean() - npix) < 4 * math.sqrt(2 * npix / len(vals))
    assert 0.75 < vals.var(ddof=1) / (2 * npix) < 1.3
    assert stats.kstest(vals, stats.chi2(npix).cdf).pvalue > 1e-3


def test_noiseless_truth_is_zero_gradient_maximum():
    for spec in (SMALL_EPL, SMALL_SIE):
        sysm, psf, model, _ = _system(spec)
        L, g = O.loglike_and_grad(sysm.truth, spec, psf, model, sysm.invvar)
        assert abs(L) < 1e-10
        assert np.abs(g).max() < 1e-8
        # any other particle is strictly worse
        other = synth.particles_box(sysm, 2, 9)
        for t in other:
            assert O.loglike(t, spec, psf, model, sysm.invvar) < -1.0


@pytest.mark.parametrize("spec", [SMALL_EPL, SMALL_SIE], ids=["EPL", "SIE"])
def test_autograd_gradient_matches_central_differences(spec):
    sysm, psf, model, data = _system(spec, 1)
    th = synth.particles_box(sysm, 2, 11).astype(np.float64)
    # one near-truth particle as well (small residuals, small gradient)
    th = np.vstack([th, sysm.truth.astype(np.float64) + 0.01 * np.random.default_rng(3).normal(size=spec.n_params)])
    for t in th:
        L, g = O.loglike_and_grad(t, spec, psf, data, sysm.invvar)
        fd = np.zeros_like(g)

        def central(j, h):
            tp, tm = t.copy(), t.copy()
            tp[j] += h
            tm[j] -= h
            return (O.loglike(tp, spec, psf, data, sysm.invvar) - O.loglike(tm, spec, psf, data, sysm.invvar)) / (2 * h)

        for j in range(len(t)):
            # Richardson-extrapolated central difference: O(h^4) truncation,
            # needed because compact n ~ 5 sources make logL very curved.
            h = 1e-5 * max(1.0, abs(t[j]))
            fd[j] = (4.0 * central(j, h / 2) - central(j, h)) / 3.0
        scale = np.abs(g).max()
        np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * scale)


def test_invalid_ellipticity_gives_minus_infinity():
    spec = SMALL_SIE
    sysm, psf, model, data = _system(spec)
    t = sysm.truth.astype(np.float64).copy()
    t[1], t[2] = 0.8, 0.7       # |e| > 1 for the mass
    assert O.loglike(t, spec, psf, data, sysm.invvar) == -math.inf
    L, g = O.loglike_and_grad(t, spec, psf, data, sysm.invvar)
    assert L == -math.inf and np.all(g == 0)


# --------------------------------------------------------------------------
# prior and bijection
# --------------------------------------------------------------------------
def _scipy_logpdf(row, x):
    kind, a, b, c, d = row
    if kind == synth.PRIOR_UNIFORM:
        return stats.uniform(a, b - a).logpdf(x)
    if kind == synth.PRIOR_NORMAL:
        return stats.norm(a, b).logpdf(x)
    if kind == synth.PRIOR_LOGNORMAL:
        return stats.lognorm(s=b, scale=math.exp(a)).logpdf(x)
    return stats.truncnorm((c - a) / b, (d - a) / b, loc=a, scale=b).logpdf(x)


def test_log_prior_matches_scipy_densities():
    dists = synth.paper_prior_dists()
    table = synth.prior_table(dists).astype(np.float64)
    th = synth.draw_params(dists, 20, 4).astype(np.float64)
    for t in th:
        lp = float(O.log_prior(torch.tensor(t), table))
        ref = sum(_scipy_logpdf(table[k], t[k]) for k in range(len(t)))
        assert abs(lp - ref) < 1e-10 * max(1.0, abs(ref))


def test_prior_densities_normalised():
    table = synth.prior_table(synth.paper_prior_dists()).astype(np.float64)
    for row in table[:10]:
        kind, a, b, c, d = row
        one = torch.tensor(row[None, :])
        f = lambda x: math.exp(float(O.log_prior(torch.tensor([x], dtype=torch.float64), one)))
        if kind == synth.PRIOR_UNIFORM:
            lo, hi = a, b
        elif kind == synth.PRIOR_TRUNCNORMAL:
            lo, hi = c, d
        elif kind == synth.PRIOR_LOGNORMAL:
            lo, hi = math.exp(a - 12 * b), math.exp(a + 12 * b)
        else:
            lo, hi = a - 12 * b, a + 12 * b
        val, _ = integrate.quad(f, lo, hi, limit=200, epsrel=1e-11)
        assert abs(val - 1.0) < 1e-8


def test_bijection_round_trip_and_log_jacobian():
    table = synth.prior_table(synth.paper_prior_dists() + synth.uniform_box_dists(SMALL_EPL)[:5]).astype(np.float64)
    rng = np.random.default_rng(12)
    u = torch.tensor(rng.normal(scale=1.5, size=table.shape[0]))
    th, logj = O.to_constrained(u, table)
    back = O.to_unconstrained(th, table)
    np.testing.assert_allclose(back.numpy(), u.numpy(), rtol=1e-10, atol=1e-10)
    # elementwise transform: log|J| = sum log|d theta_k / d u_k| (central FD)
    h = 1e-6
    tot = 0.0
    for k in range(len(u)):
        up, um = u.clone(), u.clone()
        up[k] += h
        um[k] -= h
        d = (O.to_constrained(up, table)[0][k] - O.to_constrained(um, table)[0][k]) / (2 * h)
        tot += math.log(abs(float(d)))
    assert abs(float(logj) - tot) < 1e-7 * max(1, abs(tot))


# --------------------------------------------------------------------------
# Adam and HMC
# --------------------------------------------------------------------------
def test_adam_matches_torch_optim():
    rng = np.random.default_rng(13)
    A = rng.normal(size=(5, 5))
    H = A @ A.T + np.eye(5)
    x = rng.normal(size=5)
    xt = torch.tensor(x.copy(), requires_grad=True)
    opt = torch.optim.Adam([xt], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(5)
    v = np.zeros(5)
    for k in range(1, 31):
        g = H @ x
        x, m, v = O.adam_step(x, g, m, v, k, 0.05)
        opt.zero_grad()
        loss = 0.5 * xt @ torch.tensor(H) @ xt
        loss.backward()
        opt.step()
        np.testing.assert_allclose(x, xt.detach().numpy(), rtol=1e-12, atol=1e-14)


def _gauss_target(cov):
    P = np.linalg.inv(cov)
    return (lambda u: -0.5 * u @ P @ u), (lambda u: -(P @ u))


def test_leapfrog_reversible_and_second_order():
    cov = np.array([[1.0, 0.6], [0.6, 2.0]])
    logp, grad = _gauss_target(cov)
    u0 = np.array([0.3, -1.1])
    p0 = np.array([0.8, 0.2])
    inv_m = np.array([1.0, 0.7])
    u1, p1 = O.leapfrog(u0, p0, grad, 0.1, 10, inv_m)
    u2, p2 = O.leapfrog(u1, -p1, grad, 0.1, 10, inv_m)
    np.testing.assert_allclose(u2, u0, atol=1e-12)
    np.testing.assert_allclose(-p2, p0, atol=1e-12)
    errs = []
    for eps in (0.1, 0.05, 0.025):
        n = int(round(1.0 / eps))
        u1, p1 = O.leapfrog(u0, p0, grad, eps, n, inv_m)
        errs.append(abs(O.hamiltonian(logp(u1), p1, inv_m) - O.hamiltonian(logp(u0), p0, inv_m)))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_hmc_reproduces_gaussian_moments():
    cov = np.array([[1.0, 0.5], [0.5, 0.8]])
    logp, grad = _gauss_target(cov)
    rng = np.random.default_rng(14)
    inv_m = np.ones(2)
    u = np.zeros(2)
    samples = []
    for it in range(3000):
        p = rng.normal(size=2)
        u1, p1 = O.leapfrog(u, p, grad, 0.25, 6, inv_m)
        dH = O.hamiltonian(logp(u1), p1, inv_m) - O.hamiltonian(logp(u), p, inv_m)
        if math.log(rng.uniform()) < -dH:
            u = u1
        samples.append(u)
    s = np.array(samples[200:])
    assert np.abs(s.mean(0)).max() < 0.15
    np.testing.assert_allclose(np.cov(s.T), cov, atol=0.15)


# --------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------
def test_philox4x64_matches_numpy():
    for ctr, key in [([5, 0, 0, 0], [7, 9]), ([2 ** 62 + 5, 3, 0, 11], [2 ** 40 + 1, 12345])]:
        bg = np.random.Philox(counter=ctr, key=key)
        raw = [int(v) for v in bg.random_raw(8)]
        c1 = list(ctr)
        c1[0] = (c1[0] + 1) % 2 ** 64
        if c1[0] == 0:
            c1[1] += 1
        c2 = list(c1)
        c2[0] = (c2[0] + 1) % 2 ** 64
        if c2[0] == 0:
            c2[1] += 1
        assert O.philox4(c1, key, 64) + O.philox4(c2, key, 64) == raw


def test_philox4x32_known_answers():
    # Known-answer vectors published with the Philox reference implementation
    # (Salmon, Moraes, Dror & Shaw 2011).
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for c, k, out in kat:
        assert O.philox4x32(c, k) == out


def test_philox_box_muller_momenta_are_standard_normal():
    z = np.concatenate([O.hmc_momenta(29, 1234, c, t) for c in range(40) for t in range(20)])
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    assert abs(z.var() - 1) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-3
    u = np.array([O.hmc_accept_uniform(29, 1234, c, t) for c in range(50) for t in range(20)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_philox_hmc_transition_samples_gaussian():
    cov = np.array([[1.0, 0.4], [0.4, 0.5]])
    P = np.linalg.inv(cov)
    f = lambda u: (-0.5 * u @ P @ u, -(P @ u))
    u = np.zeros(2)
    acc, out = 0, []
    for t in range(3000):
        u, lp, a, *_ = O.hmc_transition(u, f, np.ones(2), 0.3, 5, 99, 0, t)
        acc += a
        out.append(u)
    s = np.array(out[200:])
    assert acc > 2000
    assert np.abs(s.mean(0)).max() < 0.15
    np.testing.assert_allclose(np.cov(s.T), cov, atol=0.12)


def test_float32_theta_posterior_close_to_float64():
    spec = SMALL_SIE
    sysm, psf, model, data = _system(spec)
    table = synth.prior_table(sysm.prior)
    th = synth.particles_box(sysm, 2, 3).astype(np.float64)
    for t in th:
        u = O.to_unconstrained(torch.tensor(t), table).numpy().astype(np.float32)
        for jac in (True, False):
            a, ga = O.log_posterior_unconstrained(u, spec, psf, data, sysm.invvar, table, jac)
            b, gb = O.log_posterior_unconstrained(u, spec, psf, data, sysm.invvar, table, jac,
                                                  theta_float32=True)
            assert abs(a - b) <= 1e-6 * abs(a)
            assert np.linalg.norm(ga - gb) <= 1e-5 * np.linalg.norm(ga)


def test_hmc_rejects_non_finite_energy():
    """A proposal whose log density is -inf (outside the support) is never
    accepted: the chain stays put and its log density stays finite."""
    def f(u):
        if u[0] > 0.5:                                   # hard wall: no density beyond it
            return -math.inf, np.zeros(2)
        return -0.5 * float(u @ u), -u
    u = np.array([0.45, 0.0])
    moved_out = 0
    for t in range(200):
        u1, lp, acc, H0, H1, lu = O.hmc_transition(u, f, np.ones(2), 0.4, 3, 11, 0, t)
        if not math.isfinite(H1):
            assert not acc and np.array_equal(u1, u)
            moved_out += 1
        assert u1[0] <= 0.5 and math.isfinite(lp)
        u = u1
    assert moved_out > 0
