"""Pins of the oracle's SVI stage (Sec. 3: eq. vi, eq. elbo, eq. elbo-grad;
Sec. 3.2: AdaBelief).

- For a Gaussian target N(m, S) and a sample set whose mean is 0 and whose
  second moment is the identity (eps = +-sqrt(d) e_k), the Monte-Carlo ELBO
  equals KL(q || p) and the pathwise gradient equals the gradient of that KL,
  both in closed form.
- SVI with AdaBelief recovers a Gaussian target's mean and covariance, and
  the ELBO goes to 0 (the KL of a normalised target).
- AdaBelief under a constant gradient matches its geometric-series closed form.
- Surrogate draws are standard normal and a stream of their own.
- The ELBO gradient through the lens posterior matches central differences.
"""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth


def _spd(rng, d, scale=1.0):
    A = rng.normal(size=(d, d))
    return scale * (A @ A.T / d + 0.5 * np.eye(d))


def _gauss_fn(m, S):
    P = np.linalg.inv(S)
    _, logdet = np.linalg.slogdet(S)
    d = m.shape[0]

    def f(U):
        r = U - m[None, :]
        lp = -0.5 * np.einsum("ni,ij,nj->n", r, P, r) - 0.5 * logdet - 0.5 * d * math.log(2 * math.pi)
        return lp, -(r @ P)
    return f


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def test_elbo_and_gradient_exact_for_gaussian_target():
    rng = np.random.default_rng(1)
    d = 5
    S = _spd(rng, d)
    m = rng.normal(size=d)
    mu = rng.normal(size=d)
    L = np.tril(0.3 * rng.normal(size=(d, d)))
    np.fill_diagonal(L, 0.4 + rng.uniform(size=d))
    phi = O.svi_pack(mu, L)
    E = math.sqrt(d) * np.vstack([np.eye(d), -np.eye(d)])
    elbo, g, u = O.svi_elbo_grad(phi, E, _gauss_fn(m, S), round_u=False)
    np.testing.assert_allclose(u, mu[None, :] + E @ L.T, atol=1e-14)
    Sig = L @ L.T
    P = np.linalg.inv(S)
    kl = 0.5 * (np.trace(P @ Sig) + (m - mu) @ P @ (m - mu) - d
                + np.linalg.slogdet(S)[1] - np.linalg.slogdet(Sig)[1])
    assert abs(elbo - kl) < 1e-12 * max(1.0, abs(kl))
    g_mu = P @ (mu - m)
    g_L = np.tril(P @ L) - np.diag(1.0 / np.diag(L))
    r, c = np.tril_indices(d)
    g_tri = g_L[r, c].copy()
    rho = phi[d:][r == c]
    g_tri[r == c] *= _sigmoid(rho)
    np.testing.assert_allclose(g, np.concatenate([g_mu, g_tri]), rtol=1e-11, atol=1e-12)


def test_svi_adabelief_recovers_gaussian_target():
    rng = np.random.default_rng(2)
    d = 3
    S = _spd(rng, d, 0.5)
    m = rng.normal(size=d)
    phi0 = O.svi_pack(np.zeros(d), np.eye(d))
    phi, elbos, _ = O.svi_run(phi0, 32, 3000, 77, _gauss_fn(m, S), O.SVI_ADABELIEF,
                              lr=5e-3, b1=0.95, b2=0.99, round_u=False)
    mu, Sig = O.svi_moments(phi, d)
    assert np.abs(mu - m).max() < 0.1
    assert np.abs(Sig - S).max() < 0.1 * np.abs(S).max()
    assert elbos[0] > 1.0
    assert abs(np.mean(elbos[-500:])) < 0.05


def test_svi_adam_also_converges_on_gaussian_target():
    rng = np.random.default_rng(3)
    d = 2
    S = _spd(rng, d, 0.7)
    m = rng.normal(size=d)
    phi, _, _ = O.svi_run(O.svi_pack(np.zeros(d), np.eye(d)), 32, 2000, 5, _gauss_fn(m, S),
                          O.SVI_ADAM, lr=5e-3, b1=0.9, b2=0.999, eps=1e-8, round_u=False)
    mu, Sig = O.svi_moments(phi, d)
    assert np.abs(mu - m).max() < 0.1
    assert np.abs(Sig - S).max() < 0.1 * np.abs(S).max()


@pytest.mark.parametrize("eps", [1e-16, 1e-3])
def test_adabelief_constant_gradient_closed_form(eps):
    b1, b2, lr = 0.95, 0.99, 0.01
    g = np.array([3.0, -0.2, 1e-3, -40.0])
    x = np.zeros(4)
    m = np.zeros(4)
    s = np.zeros(4)
    xc = np.zeros(4)
    for t in range(1, 60):
        x, m, s = O.adabelief_step(x, g, m, s, t, lr, b1, b2, eps)
        m_c = g * (1 - b1 ** t)
        s_c = ((1 - b2) * g * g * b1 ** 2 * (b2 ** t - b1 ** (2 * t)) / (b2 - b1 ** 2)
               + eps * (1 - b2 ** t) / (1 - b2))
        xc = xc - lr * g / (np.sqrt(s_c / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(m, m_c, rtol=1e-12)
        np.testing.assert_allclose(s, s_c, rtol=1e-10)
        np.testing.assert_allclose(x, xc, rtol=1e-12)
    # a predictable gradient gets steps of about lr / b1 at first, growing as (g - m) -> 0
    x1, *_ = O.adabelief_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr, b1, b2, 1e-16)
    np.testing.assert_allclose(x1, -lr / b1 * np.sign(g), rtol=1e-6)


def test_svi_normals_standard_and_own_stream():
    z = np.concatenate([O.svi_normals(29, 31, i, t) for i in range(40) for t in range(20)])
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    assert abs(z.var() - 1) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-3
    a = O.svi_normals(29, 31, 5, 7)
    b = O.hmc_momenta(29, 31, 5, 7)
    assert np.abs(a - b).min() > 0


def test_svi_pack_unpack_round_trip_positive_diagonal():
    rng = np.random.default_rng(4)
    d = 6
    phi = rng.normal(size=O.svi_n_params(d)) * 5
    mu, L = O.svi_unpack(torch.tensor(phi), d)
    assert (torch.diagonal(L) > O.SVI_DIAG_SHIFT * 0.999).all()
    assert torch.equal(L, torch.tril(L))
    np.testing.assert_allclose(O.svi_pack(mu.numpy(), L.numpy()), phi, rtol=1e-9, atol=1e-9)


def test_svi_gradient_matches_finite_differences_on_lens_posterior():
    spec = synth.ModelSpec(14, 12, 0.18, 2, 3, synth.MASS_SIE, 1, 1)
    psf = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF)
    sysm = synth.make_system_box(spec, 0, psf=psf)
    data = (O.model_image(sysm.truth, spec, psf).numpy() + sysm.noise).astype(np.float32)
    table = synth.prior_table(sysm.prior)
    d = spec.n_params

    def f(U):
        out = [O.log_posterior_unconstrained(u, spec, psf, data, sysm.invvar, table, True) for u in U]
        return np.array([o[0] for o in out]), np.stack([o[1] for o in out])

    rng = np.random.default_rng(5)
    mu = O.to_unconstrained(torch.tensor(sysm.truth, dtype=torch.float64), table).numpy()
    L = np.diag(np.full(d, 0.02)) + np.tril(0.004 * rng.normal(size=(d, d)), -1)
    phi = O.svi_pack(mu, L)
    E = rng.normal(size=(3, d))
    elbo, g, _ = O.svi_elbo_grad(phi, E, f, round_u=False)
    r, c = np.tril_indices(d)
    tri = d + np.arange(len(r))
    picks = [0, 3, d - 1, int(tri[r == c][2]), int(tri[r == c][-1]), int(tri[(r == 5) & (c == 2)][0])]
    h = 1e-5
    for k in picks:
        e = np.zeros_like(phi)
        e[k] = h
        fp = O.svi_elbo_grad(phi + e, E, f, round_u=False)[0]
        fm = O.svi_elbo_grad(phi - e, E, f, round_u=False)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 2e-5 * max(1.0, np.abs(g).max()), (k, fd, g[k])


def test_frozen_coordinates_stay_put_and_leave_the_rest_exact():
    """A coordinate that the target ignores (a backward-modelled intensity)
    is held fixed with every surrogate entry in its row and column; on a
    Gaussian target over the other coordinates the rest of the gradient is
    still the closed-form KL gradient, and the frozen entries never move."""
    rng = np.random.default_rng(9)
    d, fz = 4, [2]
    keep = [0, 1, 3]
    S = _spd(rng, 3)
    m = rng.normal(size=3)
    base = _gauss_fn(m, S)

    def f(U):
        lp, g = base(U[:, keep])
        G = np.zeros_like(U)
        G[:, keep] = g
        return lp, G

    mu = rng.normal(size=d)
    L = np.tril(0.2 * rng.normal(size=(d, d)))
    np.fill_diagonal(L, 0.5 + rng.uniform(size=d))
    L[2, :2] = 0.0
    L[3, 2] = 0.0
    phi = O.svi_pack(mu, L)
    E = 2.0 * np.vstack([np.eye(d), -np.eye(d)])          # mean 0, second moment I (sqrt(d) = 2)
    _, g, _ = O.svi_elbo_grad(phi, E, f, round_u=False, frozen=fz)
    mask = O.svi_frozen_mask(d, fz)
    assert np.all(g[mask] == 0)
    Lk = L[np.ix_(keep, keep)]
    P = np.linalg.inv(S)
    g_mu = P @ (mu[keep] - m)
    g_L = np.tril(P @ Lk) - np.diag(1.0 / np.diag(Lk))
    r, c = np.tril_indices(d)
    full = np.zeros((d, d))
    full[np.ix_(keep, keep)] = g_L
    want = full[r, c].copy()
    rho = phi[d:][r == c]
    want[r == c] *= 1.0 / (1.0 + np.exp(-rho))
    np.testing.assert_allclose(g[:d][keep], g_mu, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(g[d:][~mask[d:]], want[~mask[d:]], rtol=1e-11, atol=1e-12)
    phi2, _, _ = O.svi_run(phi, 16, 30, 3, f, O.SVI_ADABELIEF, lr=1e-2, round_u=False, frozen=fz)
    assert np.array_equal(phi2[mask], phi[mask])
