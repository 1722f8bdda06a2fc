"""GPU parity of shapelet sources (Sec. 3: Sersic profiles and/or shapelets
for the source light; Cartesian basis of Refregier 2003) against the oracle.

Forward modelling (the coefficients are parameters): images, logL and the
gradient (incl. scale, centre and every coefficient) at n_max = 0, 4 and 8,
with the tolerances of test_gpu_parity.py.  A shapelet-only source is
compared with the oracle's lensed_shapelet_image (pinned on the CPU by
tests/test_oracle_shapelets.py).  Backward modelling (the coefficients and
Sersic intensities solved by linear inversion) with the tolerances of
test_gpu_backward.py, through the register-sized normal equations (6
components) and the LDS-tiled ones (17 and 47 components).
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_30633_amd import lens  # noqa: E402
from tests.test_gpu_backward import _check as check_backward  # noqa: E402
from tests.test_gpu_parity import check_grad, check_images, check_loglike  # noqa: E402

DEV = "cuda"
RTOL = 1e-5


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def shapelet_case(mass, nl, ns, nmax, n_prior=4, n_near=1, side=(40, 36), s=2, K=7, seed=0):
    """Base system from the uniform box plus a shapelet block: truth beta
    0.22", centre (0.04, -0.03)", coefficients N(0, 0.4^2); prior draws with
    beta U(0.1, 0.4), centre U(-0.2, 0.2), coefficients N(0, 0.4^2)."""
    base = synth.ModelSpec(side[0], side[1], 0.08, s, K, mass, nl, ns)
    spec = dataclasses.replace(base, n_shapelet=1, shapelet_nmax=nmax)
    psf = synth.asymmetric_psf(K, synth.SEED_TEST_PSF + K)
    sysm = synth.make_system_box(base, seed, psf=psf)
    nb = spec.n_shapelet_coeffs
    rng = np.random.default_rng(100 + 10 * nmax + seed)
    truth = np.concatenate([sysm.truth, [0.22, 0.04, -0.03], 0.4 * rng.normal(size=nb)]).astype(np.float32)
    data = (O.model_image(truth, spec, psf).numpy() + sysm.noise).astype(np.float32)
    thb = synth.particles_box(sysm, n_prior, seed) if base.n_params else np.zeros((n_prior, 0))
    blk = np.column_stack([rng.uniform(0.1, 0.4, n_prior), rng.uniform(-0.2, 0.2, (n_prior, 2)),
                           0.4 * rng.normal(size=(n_prior, nb))])
    th = np.hstack([thb, blk])
    near = truth[None, :] * (1 + 1e-3 * rng.standard_normal((n_near, spec.n_params)))
    th = np.vstack([th, near]).astype(np.float32)
    return spec, psf, sysm, data, th


@pytest.mark.parametrize("nmax", [0, 4, 8])
def test_forward_modelling_with_shapelets(nmax):
    spec, psf, sysm, data, th = shapelet_case("EPL", 1, 1, nmax)
    _log(f"shapelets forward: n_max {nmax}, d {spec.n_params}")
    assert lens.lens_num_params(spec) == spec.n_params
    plan = lens.LensPlan(spec, psf, data, sysm.invvar, th.shape[0], DEV)
    tt = torch.tensor(th, device=DEV)
    img = lens.lens_forward(plan, tt).cpu().numpy()
    L, G = (x.cpu().numpy() for x in lens.lens_loglike_grad(plan, tt))
    L1 = lens.lens_loglike(plan, tt).cpu().numpy()
    assert np.array_equal(L, L1)
    check_images(spec, psf, th, img)
    check_loglike(spec, psf, data, sysm.invvar, th, L)
    n = th.shape[0]
    check_grad(spec, psf, data, sysm.invvar, th, G, idx=[0, 1], near=[n - 1])


@pytest.mark.parametrize("mass,nmax", [("SIE", 4), ("EPL", 2)])
def test_shapelet_only_source_equals_the_lensed_shapelet_image(mass, nmax):
    """No Sersic components: the model image is the oracle's lensed shapelet
    image of the mass and shear parameters; the gradient is its autograd."""
    spec, psf, sysm, data, th = shapelet_case(mass, 0, 0, nmax)
    _log(f"shapelet-only source: {mass}, n_max {nmax}")
    plan = lens.LensPlan(spec, psf, data, sysm.invvar, th.shape[0], DEV)
    tt = torch.tensor(th, device=DEV)
    img = lens.lens_forward(plan, tt).cpu().numpy()
    nm = 8 if mass == "EPL" else 7
    for p in range(th.shape[0]):
        t = th[p].astype(np.float64)
        ref = O.lensed_shapelet_image(t[:nm], dataclasses.replace(spec, n_shapelet=0, n_source=0), psf,
                                      t[nm + 1], t[nm + 2], t[nm], t[nm + 3:]).numpy()
        assert np.abs(img[p] - ref).max() <= RTOL * np.abs(ref).max(), p
    L, G = (x.cpu().numpy() for x in lens.lens_loglike_grad(plan, tt))
    check_loglike(spec, psf, data, sysm.invvar, th, L)
    check_grad(spec, psf, data, sysm.invvar, th, G, idx=[0, 1, 2], near=[th.shape[0] - 1])


@pytest.mark.parametrize("nl,ns,nmax", [(0, 0, 2), (1, 1, 4), (1, 1, 8)], ids=["K6", "K17", "K47"])
def test_backward_modelling_with_shapelets(nl, ns, nmax):
    spec, psf, sysm, data, th = shapelet_case("EPL", nl, ns, nmax, n_prior=3, n_near=1)
    K = len(O.intensity_slots(spec))
    _log(f"shapelets backward: K = {K}")
    plan = lens.LensPlan(spec, psf, data, sysm.invvar, th.shape[0] * K, DEV)
    L, G, A = (t.cpu().numpy() for t in lens.lens_loglike_grad_backward(plan, torch.tensor(th, device=DEV)))
    assert A.shape == (th.shape[0], K)
    check_backward(spec, psf, data, sysm.invvar, th, L, G, A, near=(th.shape[0] - 1,))


def test_nonpositive_scale_is_invalid_and_batch_plans_refuse_shapelets():
    spec, psf, sysm, data, th = shapelet_case("EPL", 1, 1, 2, n_prior=3, n_near=0)
    th = th.copy()
    o = spec.n_params - spec.n_shapelet_coeffs - 3
    th[1, o] = 0.0
    th[2, o] = -0.2
    plan = lens.LensPlan(spec, psf, data, sysm.invvar, 3, DEV)
    L, G = (x.cpu().numpy() for x in lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV)))
    assert L[1] == -math.inf and L[2] == -math.inf and np.all(G[1:] == 0)
    check_loglike(spec, psf, data, sysm.invvar, th, L, idx=[0])
    with pytest.raises(lens.LensError) as e:
        lens.BatchPlan([spec], [psf], [data], [sysm.invvar], [4], DEV)
    assert e.value.status == lens.LENS_EUNSUPPORTED


@pytest.mark.parametrize("jac", [False, True])
def test_backward_posterior_with_more_than_64_parameters(jac):
    """EPL + one lens light + one Sersic source + an n_max = 8 shapelet source
    has d = 70, so backward-modelled intensity slots lie beyond the 64th
    parameter: the posterior must skip exactly those (no prior or Jacobian
    term, zero gradient) and agree with the oracle's backward posterior."""
    spec, psf, sysm, data, th = shapelet_case("EPL", 1, 1, 8, n_prior=3, n_near=1)
    assert spec.n_params == 70
    slots = O.intensity_slots(spec)
    assert max(slots) >= 64
    dists = synth.uniform_box_dists(spec) + [synth.U(0.05, 0.6), synth.U(-0.2, 0.2), synth.U(-0.2, 0.2)] + \
        [synth.N(0.0, 1.0)] * spec.n_shapelet_coeffs
    table = synth.prior_table(dists)
    assert table.shape[0] == spec.n_params
    # starting points inside the box (the shapelet block of the case is inside these ranges)
    thp = th.astype(np.float64).copy()
    lo = np.array([d.row()[1] for d in dists[:22]]); hi = np.array([d.row()[2] for d in dists[:22]])
    thp[:, :22] = np.clip(thp[:, :22], lo + 1e-3 * (hi - lo), hi - 1e-3 * (hi - lo))
    u = np.stack([O.to_unconstrained(torch.tensor(t, dtype=torch.float64), table).numpy() for t in thp])
    u = u.astype(np.float32)
    K = len(slots)
    plan = lens.LensPlan(spec, psf, data, sysm.invvar, u.shape[0] * K, DEV)
    plan.set_prior(table)
    plan.set_backward(True)
    _log(f"backward posterior d = {spec.n_params}, K = {K}, jac {jac}")
    lp, g = (t.cpu().numpy() for t in lens.lens_logpost_grad(plan, torch.tensor(u, device=DEV), jac))
    for p in range(u.shape[0]):
        lo_, go = O.log_posterior_backward(u[p], spec, psf, data, sysm.invvar, table, jac, theta_float32=True)
        assert np.all(g[p][slots] == 0), p
        assert abs(lp[p] - lo_) <= 1e-5 * abs(lo_), (p, lp[p], lo_)
        assert np.linalg.norm(g[p] - go) <= 1e-5 * np.linalg.norm(go), p
