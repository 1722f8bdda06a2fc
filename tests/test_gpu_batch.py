"""GPU: the uneven-batch path (persistent launches over many systems)
against per-system plans and the oracle; graph replay; autotuner cache."""
import json
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

DEV = "cuda"


def _batch(n_sys=6, seed=0, particles=(3, 5, 2, 4, 6, 3)):
    rng = np.random.default_rng(seed)
    specs, cases = [], []
    for k in range(n_sys):
        side = int(rng.integers(20, 56))
        spec = synth.ModelSpec(side, int(rng.integers(20, 56)), 0.1, int(rng.integers(1, 5)),
                               int(2 * rng.integers(0, 8) + 1), "EPL", 1, 1)
        specs.append(spec)
        cases.append(make_case(spec, 30 + k, particles[k % len(particles)], psf="asym"))
    return specs, cases


def test_batch_equals_single_plans_and_oracle():
    specs, cases = _batch()
    print("batch specs", specs, flush=True)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    theta = np.concatenate([c[3] for c in cases])
    tt = torch.tensor(theta, device=DEV)
    L, G = bp.loglike_grad(tt)
    L, G = L.cpu().numpy(), G.cpu().numpy()
    off = 0
    for spec, (sysm, psf, data, th) in zip(specs, cases):
        plan = lens.LensPlan(spec, psf, data, sysm.invvar, th.shape[0], DEV)
        Ls, Gs = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
        n = th.shape[0]
        assert np.array_equal(L[off:off + n], Ls.cpu().numpy())
        assert np.array_equal(G[off:off + n], Gs.cpu().numpy())
        lr, gr = O.loglike_and_grad(th[0], spec, psf, data, sysm.invvar)
        assert abs(L[off] - lr) <= 1e-5 * abs(lr)
        assert np.linalg.norm(G[off] - gr) <= 1e-5 * np.linalg.norm(gr)
        off += n


def test_batch_graph_replays_and_tiles():
    specs, cases = _batch(seed=1)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    tt = torch.tensor(np.concatenate([c[3] for c in cases]), device=DEV)
    Le, Ge = [t.clone() for t in bp.loglike_grad(tt)]
    Lg, Gg = torch.empty_like(Le), torch.empty_like(Ge)
    for _ in range(3):
        Lg.zero_()
        Gg.zero_()
        bp.loglike_grad(tt, Lg, Gg, use_graph=True)
        torch.cuda.synchronize()
        bp.loglike_grad(tt[:], None, None)        # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(Lg, Le) and torch.equal(Gg, Ge)
    bp.set_tiles([1, 2, 8, 3, 16, 1])
    L2, G2 = bp.loglike_grad(tt)
    assert torch.equal(L2, Le)
    torch.testing.assert_close(G2, Ge, rtol=2e-6, atol=1e-6 * float(Ge.abs().max()))


def test_autotune_and_cache(tmp_path):
    specs, cases = _batch(seed=2)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    tt = torch.tensor(np.concatenate([c[3] for c in cases]), device=DEV)
    path = tmp_path / "tiles.json"
    tiles = bp.autotune(tt, path)
    assert all(t in (1, 2, 4, 8) for t in tiles)
    cached = json.loads(path.read_text())
    assert list(cached.values())[0] == tiles
    bp.set_tiles([4] * len(tiles))
    assert bp.autotune(tt, path) == tiles        # read back from the cache
    L, G = bp.loglike_grad(tt)
    assert np.all(np.isfinite(L.cpu().numpy()))


def test_mixed_models_rejected():
    a = synth.ModelSpec(20, 20, 0.1, 2, 3, "EPL", 1, 1)
    b = synth.ModelSpec(20, 20, 0.1, 2, 3, "SIE", 1, 1)
    z = np.zeros((20, 20), np.float32)
    with pytest.raises(lens.LensError) as e:
        lens.BatchPlan([a, b], [np.ones((3, 3), np.float32)] * 2, [z, z], [z + 1, z + 1], [1, 1], DEV)
    assert e.value.status == lens.LENS_EUNSUPPORTED
