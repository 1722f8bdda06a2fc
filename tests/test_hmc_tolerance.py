"""Where the tolerance of the full-size HMC parity test comes from (CPU only).

The GPU keeps the chain state (positions, momenta, gradients) in float32;
the oracle's transition (Neal 2011 leapfrog, Sec. 3 HMC) runs in float64.
On the benchmarked system (100x100 EPL + shear, two Sersic sources, the
inverse Hessian diagonal as the inverse mass matrix, step size 0.15) the
posterior is strongly correlated, so a diagonal mass matrix leaves the
leapfrog map far from isometric: rounding-sized differences in the state grow
along the trajectory.  This test measures that growth with the oracle itself.
It reruns the oracle's leapfrog for the chains the GPU test checks, storing
every position, momentum and gradient in float32 with a randomised rounding
(each stored value within one float32 ulp of the exact one, the spread of two
different float32 implementations), and records how far the end point moves
from the float64 trajectory, in units of the posterior scale sqrt(M^-1)
after the same two-ulp allowance the GPU test grants.

Measured with 30 rounding patterns over the three chains: 0 after one
leapfrog step, 0.0008 to 0.0093 after ten (the GPU run's 0.0093 lies at the
top of that range).  HMC_L10_TOL is three times the largest of them; a wrong
kick, drift or sign moves the end point by O(1) in these units, which the
planted-mistake test below shows.
"""
import numpy as np
import pytest
import torch

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth
from tests.cases import make_case

HMC_L1_TOL = 1e-3
HMC_L10_TOL = 3e-2
HMC_CHAINS = (0, 4321, 8191)
HMC_EPS, HMC_SEED, HMC_C = 0.15, 0x5EED1234, 8192


def headline_hmc_setup():
    """The full-size HMC case: system, oracle target, inverse mass matrix and
    the chains' starting points (shared with the GPU parity test)."""
    spec = synth.config2_spec()
    sysm, psf, data, _ = make_case(spec, 0, 1, psf="double")
    table = synth.prior_table(sysm.prior)
    d = spec.n_params

    def f(uu):
        return O.log_posterior_unconstrained(np.asarray(uu, np.float32), spec, psf, data, sysm.invvar, table, True,
                                             theta_float32=True)
    ut = O.to_unconstrained(torch.tensor(sysm.truth, dtype=torch.float64), table).numpy()
    h = 1e-3
    hd = np.array([(f(ut + h * np.eye(d)[j])[1][j] - f(ut - h * np.eye(d)[j])[1][j]) / (2 * h) for j in range(d)])
    inv_mass = (1.0 / np.maximum(np.abs(hd), 1e-6)).astype(np.float32)
    rng = np.random.default_rng(31)
    u0 = (ut[None, :] + 0.5 * np.sqrt(inv_mass)[None, :] * rng.standard_normal((HMC_C, d))).astype(np.float32)
    return spec, sysm, psf, data, table, f, inv_mass, u0


def _trajectory(f, u0, inv_mass, chain, L, rounding=None, rng=None, kick_sign=1.0):
    """End point of L leapfrog steps from u0 with the chain's Philox momenta.
    rounding=None: float64; 'random': every stored value to float32 with a
    random offset below half an ulp before rounding (error below one ulp)."""
    im = inv_mass.astype(np.float64)
    d = u0.shape[0]
    p = O.hmc_momenta(d, HMC_SEED, chain, 0) / np.sqrt(im)
    u = u0.astype(np.float64)

    def r(x):
        if rounding is None:
            return x
        sp = np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)
        return (x + rng.uniform(-0.5, 0.5, x.shape) * sp).astype(np.float32).astype(np.float64)
    u, p = r(u), r(p)
    g = r(f(u)[1])
    for _ in range(L):
        p = r(p + 0.5 * HMC_EPS * kick_sign * g)
        u = r(u + HMC_EPS * im * p)
        g = r(f(u)[1])
        p = r(p + 0.5 * HMC_EPS * kick_sign * g)
    return u


def _excess(u, ref, scale):
    """max_j (|u_j - ref_j| - 2 ulp(ref_j))_+ / scale_j: the GPU test's measure."""
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    return float((np.maximum(np.abs(u - ref) - 2 * ulp, 0.0) / scale).max())


@pytest.fixture(scope="module")
def setup():
    return headline_hmc_setup()


def test_float32_state_rounding_spread_sets_the_tolerance(setup):
    spec, sysm, psf, data, table, f, inv_mass, u0 = setup
    scale = np.sqrt(inv_mass.astype(np.float64))
    worst = {1: 0.0, 10: 0.0}
    for c in HMC_CHAINS:
        for L in (1, 10):
            ref = _trajectory(f, u0[c], inv_mass, c, L)
            for k in range(4 if L == 10 else 2):
                rng = np.random.default_rng(7000 + 31 * c + k)
                u = _trajectory(f, u0[c], inv_mass, c, L, "random", rng)
                worst[L] = max(worst[L], _excess(u, ref, scale))
    assert worst[1] * 3 <= HMC_L1_TOL, worst
    # rounding alone moves ten-step end points by up to ~1e-2 of the posterior scale
    assert worst[10] > 1e-4, worst
    assert worst[10] * 3 <= HMC_L10_TOL, worst


def test_planted_leapfrog_mistakes_exceed_the_tolerance(setup):
    """A reversed kick (sign error) or a dropped inverse mass in the drift
    moves the ten-step end point far beyond HMC_L10_TOL."""
    spec, sysm, psf, data, table, f, inv_mass, u0 = setup
    scale = np.sqrt(inv_mass.astype(np.float64))
    c = HMC_CHAINS[0]
    ref = _trajectory(f, u0[c], inv_mass, c, 10)
    wrong = _trajectory(f, u0[c], inv_mass, c, 10, kick_sign=-1.0)
    assert _excess(wrong, ref, scale) > 30 * HMC_L10_TOL
    ones = np.ones_like(inv_mass)
    wrong2 = _trajectory(f, u0[c], ones, c, 1)
    ref1 = _trajectory(f, u0[c], inv_mass, c, 1)
    assert _excess(wrong2, ref1, scale) > 30 * HMC_L10_TOL
