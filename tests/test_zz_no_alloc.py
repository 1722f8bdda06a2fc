"""The allocation-free entry point (lens_loglike_grad_noalloc) against the
plan entry point (lens_loglike_grad) through the C ABI.

Both run the same kernels with the same launch shape (4 pixels per thread),
so every output must be bit-identical.  Three calls in a row share the one
static scratch array: the 100x100 px headline system at 1024 particles,
then 300 particles (a smaller input over the previous call's contents),
then the 60x60 px parity system.  Two particles of the first call are also
checked against the oracle (logL to 1e-5 relative; gradient to 1e-5 of its
norm), which ties the new entry point to the paper's definition directly.
"""
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

DEV = torch.device("cuda", 0)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _system(spec, n):
    sysm, psf, data, th = make_case(spec, 0, n_particles=n)
    arrs = [torch.tensor(a, device=DEV).contiguous() for a in (psf, data, sysm.invvar)]
    return sysm, psf, data, th, arrs


def _plan_result(spec, arrs, th_dev):
    plan = lens.LensPlan(spec, arrs[0], arrs[1], arrs[2], th_dev.shape[0], DEV)
    try:
        L, G, L64 = lens.lens_loglike_grad(plan, th_dev, want_logl64=True)
        torch.cuda.synchronize()
        return L.clone(), G.clone(), L64.clone()
    finally:
        plan.close()


def _noalloc_result(spec, arrs, th_dev):
    P, d = th_dev.shape
    L = torch.full((P,), float("nan"), device=DEV)
    G = torch.full((P, d), float("nan"), device=DEV)
    L64 = torch.full((P,), float("nan"), dtype=torch.float64, device=DEV)
    lens.lens_loglike_grad_noalloc(spec, arrs[0], arrs[1], arrs[2], th_dev, L, G, L64)
    torch.cuda.synchronize()
    return L, G, L64


def _same(a, b, what):
    assert torch.equal(a, b), (what, float((a.double() - b.double()).abs().max()))


def test_noalloc_equals_plan_entry_on_consecutive_calls():
    spec2 = synth.config2_spec()
    sysm, psf, data, th, arrs = _system(spec2, 1024)
    calls = [(spec2, arrs, th), (spec2, arrs, th[:300] * np.float32(1.0001))]
    spec1 = synth.config1_spec()
    _, _, _, th1, arrs1 = _system(spec1, 64)
    calls.append((spec1, arrs1, th1))
    first = None
    for k, (spec, a, t) in enumerate(calls):
        _log(f"noalloc call {k}: {spec.nx}x{spec.ny} px, P={t.shape[0]}")
        th_dev = torch.tensor(t, device=DEV).contiguous()
        got = _noalloc_result(spec, a, th_dev)
        ref = _plan_result(spec, a, th_dev)
        for x, y, what in zip(got, ref, ("logL", "grad", "logL64")):
            _same(x, y, f"call {k} {what}")
        assert torch.isfinite(got[0]).all() and torch.isfinite(got[1]).all()
        if k == 0:
            first = got
    L, G, _ = (x.cpu().numpy() for x in first)
    for p in (0, 517):
        lr, gr = O.loglike_and_grad(th[p], spec2, psf, data, sysm.invvar)
        assert abs(L[p] - lr) <= 1e-5 * abs(lr), (p, L[p], lr)
        assert np.linalg.norm(G[p] - gr) <= 1e-5 * np.linalg.norm(gr), p


def test_noalloc_rejects_a_request_beyond_its_scratch():
    spec = synth.config2_spec()
    _, _, _, th, arrs = _system(spec, 8)
    P = lens.LENS_NOALLOC_SCRATCH_BYTES // (4 * spec.nx * spec.ny) + 1
    big = torch.zeros((P, spec.n_params), device=DEV)
    out_l = torch.zeros(P, device=DEV)
    out_g = torch.zeros((P, spec.n_params), device=DEV)
    with pytest.raises(lens.LensError) as e:
        lens.lens_loglike_grad_noalloc(spec, arrs[0], arrs[1], arrs[2], big, out_l, out_g)
    assert e.value.status == lens.LENS_ESCRATCH
    torch.cuda.synchronize()
    assert float(out_l.abs().sum()) == 0.0   # nothing was launched
