"""Benchmark: batched logL + gradient evaluations per second at 100x100 px.

Workload (one GPU): 100x100 pixels at 0.05"/px, 3x3 supersampling, EPL +
external shear, one Sersic lens light, two Sersic sources, 21x21 PSF,
4096 particles drawn from the uniform prior box (synthetic, seeded).
One step = one multi-start MAP step over all particles: bijection + log
prior, forward model, likelihood and adjoint gradient, Adam update
(1 logL+grad evaluation per particle per step).

Prints ONE JSON line.  Timing: W untimed warm-up steps, then K steps between
two device synchronisations; the dominant kernel's average duration is read
from HIP events recorded around each of its launches on the launch stream.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "batched logL+grad evals/s at 100x100 px; time-to-MAP learned vs plain init"
PEAK_ALU_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, non-packed FP32 / FP64
PEAK_FP32_PACKED = 157.3
# HBM bytes per k_adjoint launch of this workload from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, scaled by a plain 256 MiB copy (profiles/
# map_step_100px_4096p_counters.txt).  Valid only for the kernel source it was
# measured on; reported as null otherwise.
TRAFFIC_MEASURED = {"kernel_src_sha256_16": "00b570ea922b3bcd", "bytes": 189554316}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=320)
    ap.add_argument("--workload", choices=["map", "hmc", "svi", "backward", "batch", "cnn", "parity", "large"],
                    default="map",
                    help="map: the headline MAP step (default); hmc: 8192 chains x 10 leapfrog on the same "
                         "system; svi: AdaBelief SVI steps with 4096 surrogate draws on the same system; "
                         "backward: logL + gradient with the intensities solved by linear inversion; "
                         "batch: 100 uneven systems x 512 particles; cnn: network training; parity: the small "
                         "60x60 parity system (64 particles), GPU and oracle rates for information; large: "
                         "one MAP step on a 1000x1000 px cutout (s=2, 21x21 PSF, tiled PSF stage), 128 particles")
    ap.add_argument("--cnn-batch", type=int, default=1024, help="batch of the cnn workload")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB (plain copy kernel, "
                         "for scaling HBM byte counters)")
    return ap.parse_args()


def adjoint_flops_per_subpixel(K_s, K_a, NL, NS, epl=True):
    """Algorithmic flops of the adjoint pass per sub-pixel (FMA = 2, other = 1).

    Counted from the operations the pass must perform: recompute of the
    sub-pixel forward model (float64 deflection with a K-term series, shear,
    lens equation, float32 Sersic values) and the reverse sweep (series
    derivatives, chain through the deflection, Sersic adjoints and the
    accumulated sums).
    """
    # a real-coefficient series at a complex point: 2 FMA per term (the
    # quadratic-division recurrence; the minimum for this evaluation)
    series_fwd = 4 * K_s                        # S in float64
    series_adj = 4 * K_a * (2 if epl else 1)    # S'(z) and dS/dt (float32)
    mass_fwd = 40 + (60 if epl else 0)          # offsets, U, 1/R, V0, z, pow, alpha
    shear_lens = 12
    sersic_fwd = 18                             # offset, R^2, log2, 2 exp2, mults
    sersic_adj = 30                             # + 8 accumulations, 1/R^2, beta adjoint
    mass_adj = 70
    return (series_fwd + series_adj + mass_fwd + shear_lens + mass_adj
            + (NL + NS) * (sersic_fwd + sersic_adj))


def render_flops_per_subpixel(K_s, NL, NS, epl=True):
    """Algorithmic flops of the render pass per sub-pixel (FMA = 2, other = 1):
    the forward part of the adjoint count (float64 series and deflection,
    shear and lens equation, Sersic values) plus the downsampling sum."""
    return 4 * K_s + 40 + (60 if epl else 0) + 12 + (NL + NS) * 18 + 1


def system_plan(spec, sysm, max_particles, dev, with_prior=True):
    """A plan on the system's observed image: the forward model at the truth
    (GPU) plus the system's seeded noise.  Returns (plan, data)."""
    import torch
    from paper_2606_30633_amd import lens, synth
    plan0 = lens.LensPlan(spec, sysm.psf, np.zeros((spec.ny, spec.nx), np.float32), sysm.invvar, 1, dev)
    data = (lens.lens_forward(plan0, torch.tensor(sysm.truth[None, :], device=dev))[0]
            + torch.tensor(sysm.noise, device=dev)).contiguous()
    plan0.close()
    plan = lens.LensPlan(spec, torch.tensor(sysm.psf, device=dev), data, torch.tensor(sysm.invvar, device=dev),
                         max_particles, dev)
    if with_prior:
        plan.set_prior(synth.prior_table(sysm.prior))
    return plan, data


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload != "map":
        return {"hmc": run_hmc, "svi": run_svi, "backward": run_backward, "batch": run_batch,
                "cnn": run_cnn, "parity": run_parity, "large": run_large}[args.workload](args)
    import torch
    from paper_2606_30633_amd import lens, synth

    dev = torch.device("cuda", 0)
    spec = synth.config2_spec()
    sysm = synth.config2_system()
    P = args.particles
    th = synth.particles_box(sysm, P, 0)
    # observed image: forward model at the truth (GPU) + seeded noise
    plan, data = system_plan(spec, sysm, P, dev)
    table = synth.prior_table(sysm.prior)
    u0 = torch.tensor(_to_unconstrained_box(th, table), device=dev)
    u, m, v = u0.clone(), torch.zeros_like(u0), torch.zeros_like(u0)
    loss = torch.empty(P, device=dev)

    def restart():
        u.copy_(u0)
        m.zero_()
        v.zero_()
        lens.lens_map_reset(plan)

    def step(graph=True):
        # one multi-start MAP step: T(u), log prior, logL + adjoint gradient, Adam
        lens.lens_map_adam(plan, u, m, v, 1, 1e-2, 0.99, loss=loss, use_graph=graph)

    restart()
    for _ in range(args.warmup):
        step()
    # the timed region: one gradient-descent run of K graph-replayed steps from the starts
    restart()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    evals_per_s = P / (ms_step * 1e-3)

    # per-call times: 100 graph-replayed steps, each between two events on the launch stream
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    call_ms = sorted(a.elapsed_time(b) for a, b in evs)
    median_ms = 0.5 * (call_ms[49] + call_ms[50])

    # per-kernel durations (HIP events around every launch on the launch stream), eager steps
    plan.enable_timing(True)
    for _ in range(20):
        step(graph=False)
    torch.cuda.synchronize()
    plan.enable_timing(False)
    tim = plan.read_timing()
    per = {k: t[0] / max(t[1], 1) for k, t in tim.items() if t[1]}

    # dominant kernel: adjoint sub-pixel pass
    adj_avg_ms = per["adjoint"]
    steps = _series_terms(th, spec).mean(axis=0)
    nsub = (spec.nx * spec.supersample) * (spec.ny * spec.supersample)
    fl_adj = adjoint_flops_per_subpixel(steps[0], steps[1], spec.n_lens_light, spec.n_source, True) * nsub * P
    fl_ren = render_flops_per_subpixel(steps[0], spec.n_lens_light, spec.n_source, True) * nsub * P
    fl_psf = 4.0 * spec.psf_size ** 2 * spec.nx * spec.ny * P
    achieved = fl_adj / (adj_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU_TFLOPS, 4),
                "traffic": _measured_traffic() if P == 4096 else None,
                "kernel": "k_adjoint", "avg_ms": round(adj_avg_ms, 4),
                "frac_of_fp32_packed_peak": round(achieved / PEAK_FP32_PACKED, 4),
                "kernel_ms_per_step": {k: round(x, 4) for k, x in per.items()},
                "kernel_frac": {"adjoint": round(achieved / PEAK_ALU_TFLOPS, 4),
                                "render": round(fl_ren / (per["render"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4),
                                "psf": round(fl_psf / (per["psf"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4)},
                "step_frac": round((fl_adj + fl_ren + fl_psf) / (ms_step * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4)}

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb * (1 << 20)
        src = torch.ones(nb // 4, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, sysm, th[:args.cpu_sample])

    out = {
        "metric": METRIC, "value": round(evals_per_s, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "100x100 px, s=3, EPL+shear, 1 Sersic lens, 2 Sersic sources, "
                               "21x21 PSF; one multi-start gradient-descent run of K graph-replayed MAP steps "
                               "(bijection, prior, logL + adjoint gradient, Adam) over all particles",
                   "particles": P, "sub_pixels_per_particle": nsub, "params": spec.n_params,
                   "gd_run_evals": P * args.steps, "gd_run_s": round(t1 - t0, 4),
                   "median_call_ms": round(median_ms, 4),
                   "median_call_evals_per_s": round(P / (median_ms * 1e-3), 1)},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2606_30633_amd", "csrc", "lens_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return TRAFFIC_MEASURED["bytes"] if h == TRAFFIC_MEASURED["kernel_src_sha256_16"] else None


def _to_unconstrained_box(th, table):
    """Inverse of the scaled-sigmoid map for uniform-box starting points."""
    lo, hi = table[:, 1].astype(np.float64), table[:, 2].astype(np.float64)
    p = (th.astype(np.float64) - lo) / (hi - lo)
    p = np.clip(p, 1e-6, 1 - 1e-6)
    return np.log(p / (1 - p)).astype(np.float32)


def _series_terms(th, spec):
    """Mean Horner steps per particle (host mirror of the kernel's tail bounds)."""
    o = 2
    c = np.hypot(th[:, o], th[:, o + 1]).astype(np.float64)
    t = th[:, 1].astype(np.float64) - 1.0
    out = []
    for ci, ti in zip(c, t):
        cn, Dn, cp, K, KA = 1.0, 0.0, 1.0, -1, -1
        for n in range(127):
            a, b = 2 * n + ti, 2 * n + 4 - ti
            cn1 = cn * a / b
            Dn1 = Dn + 1 / a + 1 / b
            ts = cn1 * cp * ci / (1 - ci)
            ta = max((n + 1) * cn1 * cp, cn1 * (Dn1 + 1) * cp * ci) / (1 - ci) ** 2
            if KA < 0 and ta < 2.0 ** -25:
                KA = n
            if K < 0 and ts < 2.0 ** -31:
                K = n
            if K >= 0 and KA >= 0:
                break
            cn, Dn, cp = cn1, Dn1, cp * ci
        KA = max(KA, 1)
        out.append((((K + 4) // 4) * 4, ((KA + 4) // 4) * 4))
    return np.array(out, dtype=np.float64)


def _oracle_chunk(job):
    """Worker: the oracle's logL + gradient (or logL only) of a chunk of
    particles on one torch thread; returns the wall time of the chunk."""
    spec, psf, data, invvar, th, with_grad = job
    import torch
    torch.set_num_threads(1)
    from oracle import lens_oracle as O
    fn = O.loglike_and_grad if with_grad else O.loglike
    fn(th[0], spec, psf, data, invvar)      # warm-up
    t0 = time.perf_counter()
    for t in th:
        fn(t, spec, psf, data, invvar)
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, sysm, th_sample, workers=None):
    """The FP64 oracle timed on the host cores on a bounded sample: the
    particles split over worker processes with one torch thread each (the
    particles are independent), logL + gradient (the reported value) and
    logL alone; plus the same on one process and thread (8 particles)."""
    import multiprocessing as mp
    import torch
    from oracle import lens_oracle as O
    model = O.model_image(sysm.truth, spec, sysm.psf).numpy()
    data = (model + sysm.noise).astype(np.float32)
    # at most 12 workers: with this process, at most 13 processes hold the GPU
    # runtime open (importing torch opens it), well inside a 16-process limit
    n = workers or max(1, min(12, os.cpu_count() or 1))
    chunks = [c for c in np.array_split(th_sample, n) if len(c)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(chunks)) as pool:
        pool.map(_oracle_chunk, [(spec, sysm.psf, data, sysm.invvar, c[:1], False) for c in chunks])  # start-up
        t0 = time.perf_counter()
        pool.map(_oracle_chunk, [(spec, sysm.psf, data, sysm.invvar, c, True) for c in chunks])
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        pool.map(_oracle_chunk, [(spec, sysm.psf, data, sysm.invvar, c, False) for c in chunks])
        dt_l = time.perf_counter() - t0
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        dt_1 = _oracle_chunk((spec, sysm.psf, data, sysm.invvar, th_sample[:8], True))
    finally:
        torch.set_num_threads(threads)
    return {"value": round(len(th_sample) / dt, 3), "unit": "evals/s", "cores": len(chunks),
            "kind": "oracle",
            "sample": f"{len(th_sample)} particles of the same workload, logL+grad (FP64 autograd), split over "
                      f"{len(chunks)} processes with one thread each",
            "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
            "logl_only_evals_per_s": round(len(th_sample) / dt_l, 3),
            "one_thread_evals_per_s": round(min(8, len(th_sample)) / dt_1, 3)}


def _line(args, value, unit, ms_step, workload, extra, roofline=None, dtype="f32+f64"):
    out = {"metric": METRIC, "value": round(value, 1), "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": {"workload": workload, **extra},
           "roofline": roofline, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def run_hmc(args):
    """HMC on the headline system: 8192 chains, 10 leapfrog steps per transition,
    graph-replayed transitions; value = logL+grad evals/s (chains x leapfrog x transitions/s)."""
    import torch
    from paper_2606_30633_amd import lens, synth
    dev = torch.device("cuda", 0)
    spec, sysm = synth.config2_spec(), synth.config2_system()
    C, L = 8192, 10
    plan, _ = system_plan(spec, sysm, C, dev)
    d = spec.n_params
    ut = lens.lens_to_unconstrained(plan, torch.tensor(sysm.truth[None, :], device=dev))
    # diagonal of the Hessian at the truth by central differences of the gradient -> mass matrix
    h = 1e-3
    probe = ut.repeat(2 * d, 1)
    for j in range(d):
        probe[2 * j, j] += h
        probe[2 * j + 1, j] -= h
    _, g = lens.lens_logpost_grad(plan, probe.contiguous(), True)
    hd = torch.stack([(g[2 * j, j] - g[2 * j + 1, j]) / (2 * h) for j in range(d)]).abs().clamp_min(1e-6)
    inv_mass = (1.0 / hd).float().contiguous()
    gen = torch.Generator(device="cpu").manual_seed(synth.SEED_HMC)
    u = (ut + torch.randn((C, d), generator=gen).to(dev) * inv_mass.sqrt() * 0.5).contiguous()
    logp, grad = lens.lens_logpost_grad(plan, u, True)
    acc = torch.zeros(C, dtype=torch.int32, device=dev)
    eps = 0.15
    for t in range(args.warmup):
        lens.lens_hmc_run(plan, u, grad, logp, inv_mass, eps, L, 1, synth.SEED_HMC, t, accepts=acc, use_graph=True)
    torch.cuda.synchronize()
    acc.zero_()
    t0 = time.perf_counter()
    for t in range(args.steps):
        lens.lens_hmc_run(plan, u, grad, logp, inv_mass, eps, L, 1, synth.SEED_HMC, args.warmup + t, accepts=acc,
                          use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    rate = float(acc.sum().item()) / (C * args.steps)
    # one eager transition with per-kernel events for the adjoint's roofline
    plan.enable_timing(True)
    lens.lens_hmc_run(plan, u, grad, logp, inv_mass, eps, L, 1, synth.SEED_HMC, 10 ** 6, use_graph=False)
    torch.cuda.synchronize()
    plan.enable_timing(False)
    tim = plan.read_timing()
    adj_ms = tim["adjoint"][0] / max(tim["adjoint"][1], 1)
    th = synth.particles_box(sysm, 64, 0)
    steps_k = _series_terms(th, spec).mean(axis=0)
    fl = adjoint_flops_per_subpixel(steps_k[0], steps_k[1], spec.n_lens_light, spec.n_source, True)
    achieved = fl * (spec.nx * spec.supersample) ** 2 * C / (adj_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_ALU_TFLOPS, 4), "traffic": None, "kernel": "k_adjoint",
            "avg_ms": round(adj_ms, 4), "note": "series lengths estimated from prior-box draws"}
    _line(args, C * L / dt, "evals/s", dt * 1e3,
          "HMC: 100x100 px EPL system, 8192 chains x 10 leapfrog per transition, hipGraph transitions",
          {"chains": C, "leapfrog": L, "transitions_per_s": round(1.0 / dt, 3), "acceptance": round(rate, 4),
           "eps": eps}, roof)


def run_svi(args):
    """SVI on the headline system: 4096 surrogate draws per step, AdaBelief (lr 1e-4,
    betas 0.95 / 0.99), graph-replayed steps; value = logL+grad evals/s (draws x steps/s)."""
    import torch
    from paper_2606_30633_amd import lens, synth
    dev = torch.device("cuda", 0)
    spec, sysm = synth.config2_spec(), synth.config2_system()
    n = 4096
    plan, _ = system_plan(spec, sysm, n, dev)
    d = spec.n_params
    ut = lens.lens_to_unconstrained(plan, torch.tensor(sysm.truth[None, :], device=dev))
    # surrogate start: mean at the truth, diagonal scale half the inverse-Hessian-diagonal width
    h = 1e-3
    probe = ut.repeat(2 * d, 1)
    for j in range(d):
        probe[2 * j, j] += h
        probe[2 * j + 1, j] -= h
    _, g = lens.lens_logpost_grad(plan, probe.contiguous(), True)
    hd = torch.stack([(g[2 * j, j] - g[2 * j + 1, j]) / (2 * h) for j in range(d)]).abs().clamp_min(1e-6)
    sig = (0.5 / hd.sqrt()).double().cpu().numpy()
    rho = np.log(np.expm1(sig - 1e-10))
    phi = np.concatenate([ut[0].double().cpu().numpy(), np.zeros(d * (d + 1) // 2)])
    phi[d + np.arange(d) * (np.arange(d) + 3) // 2] = rho
    x = torch.tensor(phi, dtype=torch.float32, device=dev)
    m = torch.zeros_like(x)
    s = torch.zeros_like(x)
    seed, lr = synth.SEED_HMC + 1, 1e-4
    lens.lens_svi_reset(plan)
    # warm-up and timed calls pass prefixes of one buffer: same pointer, so the captured graph is reused
    ebuf = torch.empty(max(args.warmup, args.steps), dtype=torch.float64, device=dev)
    lens.lens_svi_run(plan, x, m, s, n, args.warmup, "adabelief", lr, 0.95, 0.99, 1e-16, seed,
                      elbo=ebuf[:args.warmup], use_graph=True)
    torch.cuda.synchronize()
    el = ebuf[:args.steps]
    t0 = time.perf_counter()
    lens.lens_svi_run(plan, x, m, s, n, args.steps, "adabelief", lr, 0.95, 0.99, 1e-16, seed, elbo=el,
                      use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    elbos = el.cpu().numpy()
    # one eager step with per-kernel events for the adjoint's roofline; series lengths of these draws
    plan.enable_timing(True)
    lens.lens_svi_run(plan, x, m, s, n, 1, "adabelief", lr, 0.95, 0.99, 1e-16, seed, use_graph=False)
    torch.cuda.synchronize()
    plan.enable_timing(False)
    tim = plan.read_timing()
    adj_ms = tim["adjoint"][0] / max(tim["adjoint"][1], 1)
    _, _, u = lens.lens_svi_elbo_grad(plan, x, n, seed, 0, want_u=True)
    _, _, th = lens.lens_logpost_grad(plan, u[:256].contiguous(), True, want_theta=True)
    steps_k = _series_terms(th.cpu().numpy(), spec).mean(axis=0)
    fl = adjoint_flops_per_subpixel(steps_k[0], steps_k[1], spec.n_lens_light, spec.n_source, True)
    achieved = fl * (spec.nx * spec.supersample) ** 2 * n / (adj_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_ALU_TFLOPS, 4), "traffic": None, "kernel": "k_adjoint",
            "avg_ms": round(adj_ms, 4), "note": "series lengths from 256 of the step's draws"}
    _line(args, n / dt, "evals/s", dt * 1e3,
          "SVI: 100x100 px EPL system, full-covariance Gaussian surrogate (d = 29), 4096 draws per step, "
          "AdaBelief lr 1e-4, hipGraph steps",
          {"draws": n, "svi_steps_per_s": round(1.0 / dt, 3), "elbo_first": round(float(elbos[0]), 3),
           "elbo_last": round(float(elbos[-1]), 3)}, roof)


def run_large(args):
    """One multi-start MAP step (as in the headline workload) on a large cutout:
    1000 x 1000 px (10^6 pixels, Sec. 2's cluster-scale cutout size), s = 2
    (4 x 10^6 sub-pixels per particle), 21 x 21 PSF convolved by pixel tiles
    with halos, headline model composition with the field-scaled ranges,
    128 particles; value = logL+grad evals/s."""
    import torch
    from paper_2606_30633_amd import lens, synth
    dev = torch.device("cuda", 0)
    spec = synth.large_spec(1000, 2, 21)
    sysm = synth.make_system_large(spec, 0)
    P = 128
    th = synth.draw_params(sysm.prior, P, synth.SEED_PARTICLES)
    plan, _ = system_plan(spec, sysm, P, dev)
    table = synth.prior_table(sysm.prior)
    u = torch.tensor(_to_unconstrained_box(th, table), device=dev)
    m, v = torch.zeros_like(u), torch.zeros_like(u)
    loss = torch.empty(P, device=dev)
    lens.lens_map_reset(plan)
    for _ in range(args.warmup):
        lens.lens_map_adam(plan, u, m, v, 1, 1e-2, 0.99, loss=loss)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lens.lens_map_adam(plan, u, m, v, 1, 1e-2, 0.99, loss=loss)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    plan.enable_timing(False)
    tim = plan.read_timing()
    per = {k: t[0] / max(t[1], 1) for k, t in tim.items() if t[1]}
    steps_k = _series_terms(th, spec).mean(axis=0)
    nsub = (spec.nx * spec.supersample) * (spec.ny * spec.supersample)
    fl_adj = adjoint_flops_per_subpixel(steps_k[0], steps_k[1], spec.n_lens_light, spec.n_source, True) * nsub * P
    fl_ren = render_flops_per_subpixel(steps_k[0], spec.n_lens_light, spec.n_source, True) * nsub * P
    fl_psf = 4.0 * spec.psf_size ** 2 * spec.nx * spec.ny * P     # model (float64) + adjoint (float32) correlation
    ach = fl_adj / (per["adjoint"] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_ALU_TFLOPS, 4), "traffic": None, "kernel": "k_adjoint",
            "avg_ms": round(per["adjoint"], 4),
            "kernel_ms_per_step": {k: round(x, 4) for k, x in per.items()},
            "render_tflops": round(fl_ren / (per["render"] * 1e-3) / 1e12, 3),
            "psf_tiled_tflops": round(fl_psf / (per["psf"] * 1e-3) / 1e12, 3),
            "step_frac": round((fl_adj + fl_ren + fl_psf) / dt / 1e12 / PEAK_ALU_TFLOPS, 4)}
    _line(args, P / dt, "evals/s", dt * 1e3,
          "large cutout: 1000x1000 px, s=2, EPL+shear, 1 Sersic lens, 2 Sersic sources, 21x21 PSF by "
          "32x128-pixel tiles; one multi-start MAP step over all particles",
          {"particles": P, "sub_pixels_per_particle": nsub, "pixels": spec.nx * spec.ny,
           "sub_pixel_evals_per_s": round(P * nsub / dt, 1)}, roof)


def run_backward(args):
    """Backward modelling on the headline system: logL + gradient with the three
    Sersic intensities solved by linear inversion, 4096 particles per call
    (one render pass writing the 3 unit-intensity component images of each
    particle, their PSF, the normal equations, the model image assembled at
    the solved intensities, then the PSF/logL/adjoint pass)."""
    import torch
    from paper_2606_30633_amd import lens, synth
    dev = torch.device("cuda", 0)
    spec, sysm = synth.config2_spec(), synth.config2_system()
    P = 4096
    K = spec.n_lens_light + spec.n_source
    plan, _ = system_plan(spec, sysm, P * K, dev, with_prior=False)
    th_np = synth.particles_box(sysm, P, 0)
    th = torch.tensor(th_np, device=dev)
    for _ in range(args.warmup):
        lens.lens_loglike_grad_backward(plan, th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lens.lens_loglike_grad_backward(plan, th)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    plan.enable_timing(True)
    L, _, _ = lens.lens_loglike_grad_backward(plan, th)
    torch.cuda.synchronize()
    plan.enable_timing(False)
    tim = plan.read_timing()
    steps_k = _series_terms(th_np[:256], spec).mean(axis=0)
    nsub = (spec.nx * spec.supersample) ** 2
    adj_ms = tim["adjoint"][0] / max(tim["adjoint"][1], 1)
    fl = adjoint_flops_per_subpixel(steps_k[0], steps_k[1], spec.n_lens_light, spec.n_source, True)
    achieved = fl * nsub * P / (adj_ms * 1e-3) / 1e12
    ren_fl = render_flops_per_subpixel(steps_k[0], spec.n_lens_light, spec.n_source, True)
    ren_tf = ren_fl * nsub * P / (tim["render"][0] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_ALU_TFLOPS, 4), "traffic": None, "kernel": "k_adjoint",
            "avg_ms": round(adj_ms, 4),
            "kernel_ms_per_step": {k: round(v[0], 4) for k, v in tim.items() if v[1]},
            "render_split_tflops": round(ren_tf, 3),
            "note": "one split render pass (K component images); the model at the solved intensities is "
                    "assembled from them"}
    _line(args, P / dt, "evals/s", dt * 1e3,
          "backward modelling: 100x100 px EPL system, 3 Sersic intensities solved by linear inversion per particle, "
          "4096 particles",
          {"particles": P, "components": K, "finite_fraction": round(float(torch.isfinite(L).float().mean()), 4)},
          roof)


def run_parity(args):
    """The 60x60 parity system (SIE + shear, Sersic lens + source, s = 2, 11x11
    PSF), 64 particles: GPU logL and logL + gradient rates (a small, launch-bound
    call) and the oracle on all 64 particles, all host threads and one thread."""
    import torch
    from paper_2606_30633_amd import lens, synth
    dev = torch.device("cuda", 0)
    spec, sysm = synth.config1_spec(), synth.config1_system()
    psf = sysm.psf
    plan, _ = system_plan(spec, sysm, 64, dev, with_prior=False)
    th = synth.particles_box(sysm, 64, 0)
    t = torch.tensor(th, device=dev)
    for _ in range(args.warmup):
        lens.lens_loglike_grad(plan, t)
    torch.cuda.synchronize()
    reps = max(args.steps, 1) * 20
    t0 = time.perf_counter()
    for _ in range(reps):
        lens.lens_loglike_grad(plan, t)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        lens.lens_loglike(plan, t)
    torch.cuda.synchronize()
    dt_l = (time.perf_counter() - t0) / reps
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the host cores, with the data rendered by the oracle itself
        from oracle import lens_oracle as O
        data = (O.model_image(sysm.truth, spec, psf).numpy() + sysm.noise).astype(np.float32)
        cores = torch.get_num_threads()
        t0 = time.perf_counter()
        for x in th:
            O.loglike(x, spec, psf, data, sysm.invvar)
        c_l = len(th) / (time.perf_counter() - t0)
        t0 = time.perf_counter()
        for x in th:
            O.loglike_and_grad(x, spec, psf, data, sysm.invvar)
        c_g = len(th) / (time.perf_counter() - t0)
        torch.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            for x in th[:16]:
                O.loglike_and_grad(x, spec, psf, data, sysm.invvar)
            c_1 = 16 / (time.perf_counter() - t0)
        finally:
            torch.set_num_threads(cores)
        cpu = {"value": round(c_g, 3), "unit": "evals/s", "cores": cores, "kind": "oracle",
               "sample": "the 64 particles, logL+grad (FP64 autograd)", "logl_only_evals_per_s": round(c_l, 3),
               "one_thread_evals_per_s": round(c_1, 3)}
    out = {"metric": METRIC, "value": round(64 / dt, 1), "unit": "evals/s", "n_gpus": 1, "steps": reps,
           "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "parity system: 60x60 px, s=2, SIE+shear, Sersic lens + source, 11x11 Gaussian "
                                  "PSF, 64 particles (information only: a launch-bound call)",
                      "particles": 64, "logl_only_evals_per_s": round(64 / dt_l, 1)},
           "roofline": None, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_batch(args):
    """100 uneven systems x 512 particles: one batched logL + gradient call per step (graph replay)."""
    import tempfile
    import torch
    from paper_2606_30633_amd import lens, synth
    from paper_2606_30633_amd.learned_init import make_systems
    dev = torch.device("cuda", 0)
    sy = make_systems(100, dev)
    P = 512
    bp = lens.BatchPlan(sy.specs, sy.psfs, sy.datas, sy.invvars, [P] * 100, dev)
    table = synth.prior_table(synth.paper_prior_dists())
    theta = lens.lens_prior_sample(table, 100, P, synth.SEED_PARTICLES, dev).reshape(bp.N, bp.d).contiguous()
    t0 = time.perf_counter()
    with tempfile.TemporaryDirectory() as td:
        tiles = bp.autotune(theta, os.path.join(td, "tiles.json"))
    t_tune = time.perf_counter() - t0
    logl = torch.empty(bp.N, device=dev)
    grad = torch.empty((bp.N, bp.d), device=dev)
    for _ in range(args.warmup):
        bp.loglike_grad(theta, logl, grad, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bp.loglike_grad(theta, logl, grad, use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same work as 100 single-system plans (each with the tile the autotuner chose for its
    # system), launched one after another on the stream
    plans = []
    for k, sp in enumerate(sy.specs):
        pl = lens.LensPlan(sp, sy.psfs[k], sy.datas[k], sy.invvars[k], P, dev)
        pl.set_pixels_per_thread(int(tiles[k]))
        plans.append(pl)
    l2 = torch.empty_like(logl)
    g2 = torch.empty_like(grad)

    def per_system():
        for k, pl in enumerate(plans):
            r = slice(k * P, (k + 1) * P)
            lens.lens_loglike_grad(pl, theta[r], l2[r], g2[r])

    per_system()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        per_system()
    torch.cuda.synchronize()
    dt_sep = (time.perf_counter() - t0) / args.steps
    same = bool(torch.equal(l2, logl)) and bool(torch.equal(g2, grad))
    for pl in plans:
        pl.close()
    sub = sum(sp.nx * sp.ny * sp.supersample ** 2 for sp in sy.specs) * P
    # per-kernel durations of eager calls (HIP events on the launch stream)
    bp.enable_timing(True)
    for _ in range(5):
        bp.loglike_grad(theta, logl, grad)
    torch.cuda.synchronize()
    bp.enable_timing(False)
    per = {k: t[0] / max(t[1], 1) for k, t in bp.read_timing().items() if t[1]}
    # algorithmic flops of the persistent adjoint: every system's sub-pixels x its particles'
    # mean series lengths (one launch covers all 100 systems)
    th_np = theta.cpu().numpy()
    fl_adj = fl_ren = fl_psf = 0.0
    for k, sp in enumerate(sy.specs):
        ks = _series_terms(th_np[k * P:(k + 1) * P], sp).mean(axis=0)
        nsub_k = sp.nx * sp.ny * sp.supersample ** 2
        fl_adj += adjoint_flops_per_subpixel(ks[0], ks[1], sp.n_lens_light, sp.n_source, True) * nsub_k * P
        fl_ren += render_flops_per_subpixel(ks[0], sp.n_lens_light, sp.n_source, True) * nsub_k * P
        fl_psf += 4.0 * sp.psf_size ** 2 * sp.nx * sp.ny * P
    ach = fl_adj / (per["adjoint"] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_ALU_TFLOPS, 4), "traffic": None, "kernel": "k_batch_adjoint (persistent)",
            "avg_ms": round(per["adjoint"], 4), "kernel_ms_per_step": {k: round(x, 4) for k, x in per.items()},
            "kernel_frac": {"render": round(fl_ren / (per["render"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4),
                            "psf": round(fl_psf / (per["psf"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS, 4)},
            "step_frac": round((fl_adj + fl_ren + fl_psf) / dt / 1e12 / PEAK_ALU_TFLOPS, 4)}
    _line(args, bp.N / dt, "evals/s", dt * 1e3,
          "uneven batch: 100 systems (side 48-160 px, s 2-4, PSF 11-31), 512 particles each, "
          "one persistent render + adjoint launch per step, autotuned tiles",
          {"particles": bp.N, "sub_pixel_evals_per_s": round(sub / dt, 1), "autotune_s": round(t_tune, 2),
           "tiles": {str(t): tiles.count(t) for t in sorted(set(tiles))},
           "per_system_plans_evals_per_s": round(bp.N / dt_sep, 1),
           "persistent_gain": round(dt_sep / dt, 3), "per_system_results_identical": same}, roof)


def run_cnn(args):
    """Training throughput of the learned initializer's network (BF16 MFMA)."""
    import torch
    from paper_2606_30633_amd import lens, synth
    from paper_2606_30633_amd.learned_init import simulate, target_standardization, SIGMA, TARGET_IDX
    dev = torch.device("cuda", 0)
    B = args.cnn_batch
    theta, images = simulate(B * 16, synth.SEED_CNN_TRAIN, dev)
    mean, std = target_standardization(theta)
    tgt = torch.tensor((theta[:, TARGET_IDX] - mean) / std, dtype=torch.float32, device=dev)
    net = lens.Cnn(B, 1, dev)
    xb = net.prepare(images, SIGMA, add_noise=True, seed=1)
    loss = torch.empty(1, device=dev)
    for i in range(args.warmup):
        net.train_step(xb[(i % 16) * B:(i % 16 + 1) * B], tgt[(i % 16) * B:(i % 16 + 1) * B], 1e-3, loss)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        k = i % 16
        net.train_step(xb[k * B:(k + 1) * B], tgt[k * B:(k + 1) * B], 1e-3, loss)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # flops per image: forward convolutions + MLP, backward ~2x forward (no data gradient of the input)
    fwd = 0.0
    cin, H = 1, 64
    for c, s in zip([32, 32, 64, 64, 128, 128], [1, 2, 1, 2, 1, 2]):
        H //= s
        fwd += 2.0 * H * H * c * 9 * cin
        cin = c
    fwd += 2.0 * (128 * 256 + 256 * 28)
    train = 3.0 * fwd - 2.0 * 64 * 64 * 32 * 9
    achieved = train * B / dt / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": 2500.0, "unit": "TFLOP/s",
            "frac": round(achieved / 2500.0, 5), "traffic": None, "kernel": "training step (all kernels)"}
    _line(args, B / dt, "images/s", dt * 1e3, f"learned-initializer network training, batch {B}, 64x64 bf16",
          {"batch": B, "gflop_per_image_train": round(train / 1e9, 4)}, roof, dtype="bf16")


if __name__ == "__main__":
    main()
