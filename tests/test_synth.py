"""The seeded input generators against the paper's printed distributions."""
import math
import os

import numpy as np
import pytest

from paper_2606_30633_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_sim_dist.txt")
KIND = {"LN": synth.PRIOR_LOGNORMAL, "TN": synth.PRIOR_TRUNCNORMAL,
        "N": synth.PRIOR_NORMAL, "U": synth.PRIOR_UNIFORM}


def _rows():
    out = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        out.append(line.split())
    return out


@pytest.mark.parametrize("which", ["sim", "prior"])
def test_paper_distributions_match_eq_sim_dist(which):
    rows = _rows()
    dists = synth.paper_sim_dists() if which == "sim" else synth.paper_prior_dists()
    assert len(rows) == len(dists) == 22
    for r, d in zip(rows, dists):
        name, kind = r[0], r[1]
        p1, p2 = (float(r[2]), float(r[3])) if which == "sim" else (float(r[4]), float(r[5]))
        assert d.kind == KIND[kind], name
        if kind == "LN":
            scale = 1e-3 if name.endswith("_I") else 1.0   # intensities / 1000
            assert math.isclose(d.a, math.log(p1 * scale), rel_tol=1e-12), name
            assert d.b == p2, name
        elif kind == "U":
            assert (d.a, d.b) == (p1, p2), name
        else:
            assert (d.a, d.b) == (p1, p2), name
            if kind == "TN":
                assert (d.c, d.d) == (float(r[6]), float(r[7])), name


def test_draws_are_seeded_and_in_support():
    a = synth.draw_params(synth.paper_sim_dists(), 5000, 3)
    b = synth.draw_params(synth.paper_sim_dists(), 5000, 3)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    assert np.all((a[:, 1] >= 1) & (a[:, 1] <= 3))
    assert np.all(np.abs(a[:, 10:12]) <= 0.15) and np.all(np.abs(a[:, 17:19]) <= 0.5)
    assert abs(np.median(a[:, 0]) - 1.25) < 0.03
    assert abs(np.std(np.log(a[:, 0])) - 0.25) < 0.02


def test_psf_kernels_normalised():
    for k in (11, 21, 31):
        for p in (synth.double_gaussian_psf(k, 0.05), synth.asymmetric_psf(k, 1)):
            assert p.shape == (k, k) and abs(float(p.astype(np.float64).sum()) - 1) < 1e-6
    g = synth.gaussian_psf(11, 0.1, 0.05).astype(np.float64)
    # second moment of a FWHM 0.1" Gaussian at 0.05"/px: sigma = 0.8493 px
    u = np.arange(11) - 5
    var = (g.sum(0) * u ** 2).sum()
    assert abs(math.sqrt(var) - 0.1 / 2.35482 / 0.05) < 1e-3


def test_uneven_batch_shapes():
    specs = synth.uneven_batch_specs(100)
    sides = np.array([s.nx for s in specs])
    assert sides.min() >= 48 and sides.max() <= 160
    assert set(s.supersample for s in specs) <= {2, 3, 4}
    assert all(s.psf_size % 2 == 1 and 11 <= s.psf_size <= 31 for s in specs)
    assert all(s.n_params == 22 for s in specs)
