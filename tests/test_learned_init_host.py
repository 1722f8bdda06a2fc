"""Host-side bookkeeping of the time-to-MAP comparison (learned_init): the
time at which an arm first reaches a target, arms run on groups of systems
taken as one batch, the saved arm state, and the target standardisation."""
import math
import os
import tempfile

import numpy as np
import torch

from paper_2606_30633_amd.learned_init import (ArmRun, _concat_arms, _load_arm, _save_arm, target_standardization,
                                               time_to_reach)


def _arm(best, t_init=1.0, t_step=0.5):
    best = np.asarray(best, dtype=np.float64)
    return ArmRun(t_init, t_step, best.shape[0] - 1, best, torch.zeros((best.shape[1], 3)))


def test_time_to_reach_first_hit_and_never():
    run = _arm([[-10.0, -5.0], [-3.0, -4.0], [-1.0, -2.0]])
    t = time_to_reach(run, np.array([-3.0, -1.0]))
    assert t[0] == 1.0 + 2 * 0.5            # reached after the second update (index 1)
    assert math.isinf(t[1])
    assert time_to_reach(run, np.array([-20.0, -20.0]))[0] == 1.0 + 0.5


def test_concat_arms_sums_times_and_joins_systems():
    a = _arm([[-3.0], [-2.0]], 1.0, 0.25)
    b = _arm([[-5.0, -6.0], [-4.0, -1.0]], 2.0, 0.5)
    c = _concat_arms([a, b])
    assert c.t_init == 3.0 and c.t_step == 0.75 and c.steps == 1
    np.testing.assert_array_equal(c.best, [[-3.0, -5.0, -6.0], [-2.0, -4.0, -1.0]])
    assert c.best_u.shape == (3, 3)


def test_saved_arm_round_trips():
    run = _arm([[-3.0, -2.0], [-1.0, 0.5]], 1.25, 0.125)
    run.best_u[:] = torch.arange(6.0).reshape(2, 3)
    with tempfile.TemporaryDirectory() as td:
        p = os.path.join(td, "arm.npz")
        _save_arm(p, run, flags=np.array([1, 0]))
        back, extra = _load_arm(p, "cpu")
    assert back.t_init == run.t_init and back.t_step == run.t_step and back.steps == run.steps
    np.testing.assert_array_equal(back.best, run.best)
    assert torch.equal(back.best_u, run.best_u)
    np.testing.assert_array_equal(extra["flags"], [1, 0])


def test_target_standardization_uses_the_regressed_columns():
    rng = np.random.default_rng(1)
    th = rng.normal(size=(5000, 22)) * np.arange(1, 23) + np.arange(22)
    mean, std = target_standardization(th.astype(np.float32))
    cols = np.array([0, 1, 2, 3, 6, 7, 8, 9, 15, 16, 17, 18, 19, 20])
    assert mean.shape == (14,) and std.shape == (14,)
    assert np.all(np.abs(mean - cols) <= 0.1 * (cols + 1))
    np.testing.assert_allclose(std, cols + 1, rtol=0.05)


def test_regressed_columns_are_the_named_parameters():
    from paper_2606_30633_amd import synth
    from paper_2606_30633_amd.learned_init import TARGET_IDX
    names = synth.paper_spec(64, 2, 21).param_names()
    assert [names[j] for j in TARGET_IDX] == [
        "theta_E", "gamma", "m_e1", "m_e2", "g1", "g2", "l0_R_e", "l0_n",
        "s0_R_e", "s0_n", "s0_e1", "s0_e2", "s0_x", "s0_y"]
