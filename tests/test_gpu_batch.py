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


def test_batch_per_call_particle_counts():
    """lens_batch_set_particles: fewer particles per system than the plan was
    created with, then back up; each call equals a plan created with those
    counts bit for bit (eager and graph), and segment operations follow."""
    specs, cases = _batch(seed=7, particles=(9, 4, 12, 6, 7, 5))
    args = ([c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases])
    full = [c[3] for c in cases]
    bp = lens.BatchPlan(specs, *args, [t.shape[0] for t in full], DEV)
    Lg, Gg = None, None
    for counts in ([3, 1, 12, 2, 7, 5], [1, 1, 1, 1, 1, 1], [9, 4, 12, 6, 7, 5], [5, 4, 2, 6, 1, 3]):
        print("counts", counts, flush=True)
        bp.set_particles(counts)
        assert bp.get_particles() == counts and bp.N == sum(counts)
        th = np.concatenate([t[:n] for t, n in zip(full, counts)])
        tt = torch.tensor(th, device=DEV)
        Le, Ge = bp.loglike_grad(tt)
        Lg, Gg = torch.full_like(Le, np.nan), torch.full_like(Ge, np.nan)
        bp.loglike_grad(tt, Lg, Gg, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(Lg, Le) and torch.equal(Gg, Ge)
        ref = lens.BatchPlan(specs, *args, counts, DEV)
        Lr, Gr = ref.loglike_grad(tt)
        assert torch.equal(Lr, Le) and torch.equal(Gr, Ge)
        Lc, Gc = bp.loglike_grad_counts(counts, tt)            # the one-call form
        assert torch.equal(Lc, Le) and torch.equal(Gc, Ge)
        best, arg = bp.argmin(-Le)
        off = 0
        Ln = Le.cpu().numpy()
        for k, n in enumerate(counts):
            i = int(np.argmax(Ln[off:off + n]))
            assert int(arg[k]) == off + i
            off += n
    with pytest.raises(ValueError):
        bp.set_particles([10, 4, 12, 6, 7, 5])       # above the capacity of system 0


def test_autotune_and_cache(tmp_path):
    specs, cases = _batch(seed=2)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    tt = torch.tensor(np.concatenate([c[3] for c in cases]), device=DEV)
    path = tmp_path / "tiles.json"
    tiles = bp.autotune(tt, path)
    assert all(t in (1, 2, 4, 8) for t in tiles)
    cached = list(json.loads(path.read_text()).values())[0]
    assert cached[:len(tiles)] == tiles
    assert len(cached) > len(tiles) and all(nt in (256, 512, 1024) for nt in cached[len(tiles):])
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


def _batch_with_prior(seed):
    specs, cases = _batch(seed=seed)
    table = synth.prior_table(synth.paper_prior_dists())
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    bp.set_prior(table)
    th = synth.draw_params(synth.paper_prior_dists(), bp.N, 5150 + seed)
    u = np.stack([O.to_unconstrained(torch.tensor(t, dtype=torch.float64), table).numpy() for t in th])
    return specs, cases, table, bp, u.astype(np.float32)


@pytest.mark.parametrize("jac", [False, True])
def test_batch_logpost_equals_single_plans_and_oracle(jac):
    specs, cases, table, bp, u = _batch_with_prior(3)
    print("batch logpost", specs, jac, flush=True)
    lp, g, th = bp.logpost_grad(torch.tensor(u, device=DEV), jac, want_theta=True)
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    off = 0
    for k, (spec, (sysm, psf, data, _)) in enumerate(zip(specs, cases)):
        n = bp.particles[k]
        plan = lens.LensPlan(spec, psf, data, sysm.invvar, n, DEV)
        plan.set_prior(table)
        lps, gs = lens.lens_logpost_grad(plan, torch.tensor(u[off:off + n], device=DEV), jac)
        assert np.array_equal(lp[off:off + n], lps.cpu().numpy())
        assert np.array_equal(g[off:off + n], gs.cpu().numpy())
        lr, gr = O.log_posterior_unconstrained(u[off], spec, psf, data, sysm.invvar, table, jac,
                                               theta_float32=True)
        assert abs(lp[off] - lr) <= 1e-5 * abs(lr)
        assert np.linalg.norm(g[off] - gr) <= 1e-5 * np.linalg.norm(gr)
        off += n


def test_batch_map_adam_graph_eager_and_single_plans():
    specs, cases, table, bp, u = _batch_with_prior(4)
    ue = torch.tensor(u, device=DEV)
    me, ve = torch.zeros_like(ue), torch.zeros_like(ue)
    le = torch.empty(bp.N, device=DEV)
    bp.map_reset()
    bp.map_adam(ue, me, ve, 3, 5e-3, decay=0.99, loss=le)
    ug = torch.tensor(u, device=DEV)
    mg, vg = torch.zeros_like(ug), torch.zeros_like(ug)
    lg = torch.empty(bp.N, device=DEV)
    bp.map_reset()
    for _ in range(3):
        bp.map_adam(ug, mg, vg, 1, 5e-3, decay=0.99, loss=lg, use_graph=True)
        torch.cuda.synchronize()
        bp.logpost_grad(ue, False)          # eager work between replays
        torch.cuda.synchronize()
    for a, b in ((ue, ug), (me, mg), (ve, vg), (le, lg)):
        assert torch.equal(a, b)
    off = 0
    for k, (spec, (sysm, psf, data, _)) in enumerate(zip(specs, cases)):
        n = bp.particles[k]
        plan = lens.LensPlan(spec, psf, data, sysm.invvar, n, DEV)
        plan.set_prior(table)
        us = torch.tensor(u[off:off + n], device=DEV)
        ms, vs = torch.zeros_like(us), torch.zeros_like(us)
        ls = torch.empty(n, device=DEV)
        lens.lens_map_reset(plan)
        lens.lens_map_adam(plan, us, ms, vs, 3, 5e-3, decay=0.99, loss=ls)
        assert torch.equal(us, ue[off:off + n]) and torch.equal(ls, le[off:off + n])
        off += n


def test_batch_argmin_exact():
    specs, cases = _batch(seed=5, particles=(300, 1, 7, 256, 257, 3))
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    rng = np.random.default_rng(9)
    val = rng.integers(-5, 5, bp.N).astype(np.float32)      # many ties
    val[rng.random(bp.N) < 0.1] = np.nan
    val[bp.particles[0]] = np.nan                            # a one-particle system holding NaN
    best, arg = bp.argmin(torch.tensor(val, device=DEV))
    best, arg = best.cpu().numpy(), arg.cpu().numpy()
    off = 0
    for k, n in enumerate(bp.particles):
        seg = np.where(np.isnan(val[off:off + n]), np.inf, val[off:off + n])
        i = int(np.argmin(seg))                              # first occurrence
        assert best[k] == seg[i] and arg[k] == off + i, k
        off += n


def test_batch_center_views_exact():
    specs, cases = _batch(seed=6)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [c[3].shape[0] for c in cases], DEV)
    for side in (64, 31, 20):
        views = bp.center_views(side).cpu().numpy()
        for k, (spec, c) in enumerate(zip(specs, cases)):
            img = c[2].astype(np.float64)
            ref = np.zeros((side, side))
            for i in range(side):
                for j in range(side):
                    r2, c2 = 2 * i + spec.ny - side, 2 * j + spec.nx - side
                    rs = {(r2 - (r2 & 1)) // 2, (r2 + (r2 & 1)) // 2}
                    cs = {(c2 - (c2 & 1)) // 2, (c2 + (c2 & 1)) // 2}
                    acc = 0.0
                    for r in sorted(rs) * (2 // len(rs)):
                        for cc in sorted(cs) * (2 // len(cs)):
                            if 0 <= r < spec.ny and 0 <= cc < spec.nx:
                                acc += img[r, cc]
                    ref[i, j] = 0.25 * acc
            np.testing.assert_allclose(views[k], ref.astype(np.float32), rtol=1e-6, atol=1e-7)


def test_full_size_uneven_batch_sampled_parity(tmp_path):
    """The uneven-batch workload at full size in the benchmark's launch
    configuration (100 systems of side 48-160 px, s 2-4, PSF 11-31 px, 512
    particles each, one persistent launch, autotuned tiles): sampled
    particles of the largest and smallest systems against the oracle.  Data
    are seeded noise images (the likelihood parity does not depend on them)."""
    specs = synth.uneven_batch_specs(100)
    psfs = [synth.double_gaussian_psf(sp.psf_size, sp.pix_scale) for sp in specs]
    datas = [synth.noise((sp.ny, sp.nx), synth.SIGMA_NOISE, synth.SEED_NOISE + k) for k, sp in enumerate(specs)]
    invvars = [synth.invvar_map(sp.ny, sp.nx, synth.SIGMA_NOISE) for sp in specs]
    P = 512
    bp = lens.BatchPlan(specs, psfs, datas, invvars, [P] * 100, DEV)
    theta = np.concatenate([synth.particles_paper(P, k) for k in range(100)]).astype(np.float32)
    tt = torch.tensor(theta, device=DEV)
    bp.autotune(tt, tmp_path / "tiles.json")
    L, G = bp.loglike_grad(tt, use_graph=True)
    L, G = L.cpu().numpy(), G.cpu().numpy()
    work = [sp.nx * sp.ny * sp.supersample ** 2 for sp in specs]
    order = np.argsort(work)
    picks = [(int(order[-1]), 0), (int(order[-2]), 511), (int(order[0]), 7), (int(order[50]), 300)]
    for k, p in picks:
        row = k * P + p
        sp = specs[k]
        print("batch parity", sp, "particle", p, flush=True)
        lr, gr = O.loglike_and_grad(theta[row], sp, psfs[k], datas[k], invvars[k])
        if not np.isfinite(lr):
            assert not np.isfinite(L[row])
            continue
        assert abs(L[row] - lr) <= 1e-5 * abs(lr), (k, p, L[row], lr)
        assert np.linalg.norm(G[row] - gr) <= 1e-5 * np.linalg.norm(gr), (k, p)


@pytest.mark.parametrize("mass,nl,ns", [("SIE", 0, 2), ("EPL", 2, 3), ("SIE", 1, 1)])
def test_batch_other_models_equal_single_plans_and_oracle(mass, nl, ns):
    """Other compositions (other instances of the batch kernels): batch ==
    per-system plans bitwise, sampled particles against the oracle."""
    rng = np.random.default_rng(40 + nl + 3 * ns)
    specs, cases = [], []
    for k in range(4):
        spec = synth.ModelSpec(int(rng.integers(16, 40)), int(rng.integers(16, 40)), 0.1, int(rng.integers(1, 4)),
                               int(2 * rng.integers(0, 6) + 1), mass, nl, ns)
        specs.append(spec)
        cases.append(make_case(spec, 60 + k, 3, psf="asym"))
    print("batch models", mass, nl, ns, specs, flush=True)
    bp = lens.BatchPlan(specs, [c[1] for c in cases], [c[2] for c in cases], [c[0].invvar for c in cases],
                        [3] * 4, DEV)
    theta = np.concatenate([c[3] for c in cases])
    L, G = bp.loglike_grad(torch.tensor(theta, device=DEV))
    L, G = L.cpu().numpy(), G.cpu().numpy()
    for k, (spec, (sysm, psf, data, th)) in enumerate(zip(specs, cases)):
        plan = lens.LensPlan(spec, psf, data, sysm.invvar, 3, DEV)
        Ls, Gs = lens.lens_loglike_grad(plan, torch.tensor(th, device=DEV))
        assert np.array_equal(L[3 * k:3 * k + 3], Ls.cpu().numpy())
        assert np.array_equal(G[3 * k:3 * k + 3], Gs.cpu().numpy())
        lr, gr = O.loglike_and_grad(th[1], spec, psf, data, sysm.invvar)
        assert abs(L[3 * k + 1] - lr) <= 1e-5 * abs(lr)
        assert np.linalg.norm(G[3 * k + 1] - gr) <= 1e-5 * np.linalg.norm(gr)
