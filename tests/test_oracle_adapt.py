"""Pins of the oracle's HMC adaptation (dual-averaged step size, Hoffman &
Gelman 2014; mass matrix from burn-in variances, Sec. 3.3).

- on a deterministic acceptance curve alpha(eps) = exp(-eps^2 / 2) the
  averaged step size converges to the root of alpha = delta;
- the first update follows the closed form of the recursion at m = 1;
- a burn-in on a Gaussian target ends with a step size whose acceptance is
  near the target and variances near the target's.
"""
import math

import numpy as np

from oracle import lens_oracle as O


def test_dual_averaging_finds_target_acceptance():
    for delta in (0.65, 0.8, 0.9):
        st = O.dual_averaging_init(1.0)
        for _ in range(4000):
            eps = math.exp(st["log_eps"])
            st = O.dual_averaging_update(st, math.exp(-eps * eps / 2), delta)
        want = math.sqrt(-2 * math.log(delta))
        assert abs(math.exp(st["log_eps_bar"]) / want - 1) < 0.02, (delta, math.exp(st["log_eps_bar"]), want)


def test_dual_averaging_first_update_closed_form():
    st = O.dual_averaging_update(O.dual_averaging_init(0.3), 0.2, 0.8)
    H1 = (0.8 - 0.2) / 11.0                         # eta = 1 / (1 + t0), H_bar_0 = 0
    le = math.log(3.0) - 1.0 / 0.05 * H1            # mu - sqrt(1) / gamma * H_bar
    assert abs(st["H_bar"] - H1) < 1e-15 and abs(st["log_eps"] - le) < 1e-12
    assert abs(st["log_eps_bar"] - le) < 1e-12      # weight 1^-kappa = 1


def test_hmc_adapt_on_gaussian_target():
    cov = np.array([[0.5, 0.2], [0.2, 0.3]])
    P = np.linalg.inv(cov)
    f = lambda u: (-0.5 * u @ P @ u, -(P @ u))
    rng = np.random.default_rng(1)
    U0 = rng.standard_normal((16, 2)) * 0.3
    U, eps_t, eps_bar, var, alphas, _ = O.hmc_adapt(U0, f, np.ones(2), 0.05, 0.8, 4, 300, 100, 7, eps_float32=False)
    assert abs(eps_t[0] - 0.05) < 1e-15 and np.all(np.isfinite(eps_t))
    assert 0.6 < np.mean(alphas[-100:]) < 0.95
    np.testing.assert_allclose(var, np.diag(cov), rtol=0.2)
    # with the adapted step size fixed, acceptance is near the target
    al = []
    for t in range(100):
        for c in range(16):
            U[c], _, _, H0, H1, _ = O.hmc_transition(U[c], f, np.ones(2), eps_bar, 4, 7, c, 1000 + t)
            al.append(O.accept_prob(H0, H1))
    assert 0.65 < np.mean(al) < 0.95
