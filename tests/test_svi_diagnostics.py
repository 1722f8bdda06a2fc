"""Host-side MCMC diagnostics of the SVI/HMC study (split-R-hat and the
cross-chain effective sample size of Bayesian Data Analysis, 3rd ed.,
Sec. 11.4-11.5), pinned on chains whose answer is known in closed form."""
import numpy as np

from paper_2606_30633_amd.svi_study import ess, split_rhat


def _ar1(rng, T, C, d, phi):
    x = np.empty((T, C, d))
    x[0] = rng.standard_normal((C, d)) / np.sqrt(1 - phi * phi)
    for t in range(1, T):
        x[t] = phi * x[t - 1] + rng.standard_normal((C, d))
    return x


def test_iid_chains():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2000, 4, 3))
    assert np.all(np.abs(split_rhat(x) - 1) < 0.01)
    e = ess(x)
    assert np.all(np.abs(e / 8000 - 1) < 0.2), e


def test_ar1_chains_match_closed_form_ess():
    # AR(1) with coefficient phi: integrated autocorrelation time (1 + phi) / (1 - phi)
    rng = np.random.default_rng(1)
    for phi in (0.5, 0.9):
        x = _ar1(rng, 4000, 8, 2, phi)
        want = 32000 * (1 - phi) / (1 + phi)
        e = ess(x)
        assert np.all(np.abs(e / want - 1) < 0.25), (phi, e, want)
        assert np.all(split_rhat(x) < 1.02)


def test_chains_stuck_apart_have_large_rhat():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((500, 4, 2))
    x[:, 0, :] += 3.0
    assert np.all(split_rhat(x) > 1.3)
    drift = rng.standard_normal((500, 4, 1)) + np.linspace(0, 4, 500)[:, None, None]
    assert split_rhat(drift)[0] > 1.3


def test_elbo_summary_and_hmc_comparison_helpers():
    from paper_2606_30633_amd.svi_study import compare_to_hmc, elbo_summary
    el = np.concatenate([np.linspace(100.0, 10.0, 150), [30.0], np.full(149, 10.0)])
    s = elbo_summary(el)
    assert s["elbo_first"] == 100.0 and s["elbo_last100"] == 10.0 and s["elbo_min"] == 10.0
    assert s["steps_above_start_after_100"] == 0
    assert abs(s["max_rise_above_running_min"] - 20.0) < 1e-12
    el2 = el.copy()
    el2[200:205] = 150.0                       # five steps above the start after step 100
    assert elbo_summary(el2)["steps_above_start_after_100"] == 5
    rng = np.random.default_rng(0)
    smp = rng.standard_normal((400, 8, 3)) * np.array([1.0, 2.0, 0.5]) + np.array([0.0, 1.0, -1.0])
    c = compare_to_hmc(np.array([0.0, 1.0, -1.0]), np.array([1.0, 4.0, 0.25]), smp)
    assert c["mean_offset_sd_max"] < 0.1 and abs(c["std_ratio_median"] - 1) < 0.05
    c2 = compare_to_hmc(np.array([1.0, 1.0, -1.0]), np.array([0.25, 1.0, 0.0625]), smp)
    assert abs(c2["std_ratio_median"] - 0.5) < 0.05 and c2["mean_offset_sd_max"] > 0.9
