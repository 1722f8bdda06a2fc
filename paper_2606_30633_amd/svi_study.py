"""SVI with Adam and with AdaBelief on synthetic systems, and the surrogates
against an HMC posterior (Sec. 3: the MAP -> SVI -> HMC pipeline; Sec. 3.2:
choice of the SVI optimizer, AdaBelief with lr 1e-4, betas 0.95 / 0.99, no
schedule; Sec. 3.3: the SVI covariance sets the HMC mass matrix).

Per system (the first S systems of the uneven batch, parameters drawn from
the paper's prior, eq. sim-dist):

1. MAP: multi-start Adam from n_map prior draws per system, all systems in
   one batch (the time-to-MAP study's plain arm: hold-then-decay learning
   rate, lens_batch_map_adam, lens_batch_argmin), the best particle by log
   posterior.
2. Surrogate start: mu = the MAP; L diagonal with L_jj = 0.5 / sqrt|H_jj|,
   H_jj the curvature of the HMC target at the MAP along u_j (central
   differences of lens_logpost_grad).
3. SVI from that start with Adam and with AdaBelief: n_vi draws per step,
   steps_vi steps, the same learning rate (lens_svi_run, graph replay);
   the ELBO of every step.
4. HMC: chains started at draws of the AdaBelief surrogate
   (lens_svi_elbo_grad), inverse mass matrix = the surrogate's variances
   (lens_svi_moments), the step size dual-averaged during burn-in towards an
   acceptance of 0.8 (lens_hmc_adapt), then n_hmc transitions of L leapfrog
   steps (lens_hmc_run); split-R-hat and effective sample size of the samples.
   As in Sec. 4.2, a system with split-R-hat >= 1.1 is run again with a
   longer burn-in and more samples (burn_rerun, n_rerun: 2000 and 7000),
   and one still above 1.1 gets the mass-matrix adaptation of Sec. 3.3
   (plus a short step-size retune) and is sampled again (n_rerun samples).  Defaults follow the paper's settings for
   its 100 simulated systems (MAP 1000 steps; SVI 5000 steps of 1000 draws;
   HMC 500 burn-in and 1500 samples) with 128 chains instead of 64.

Reported per optimizer: the ELBO at the start and over the last 100 steps,
the number of steps after the first 100 whose ELBO is above the starting
value, and the largest rise above the running minimum; for each surrogate
against the HMC sample: the offset of the means in units of the HMC
standard deviation and the ratio of the standard deviations (summarised
over the systems whose chains converged).

Stages run in one process: python -m paper_2606_30633_amd.svi_study --out r.json
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import lens, synth
from .learned_init import Schedule, make_systems, plain_arm


# ---------------------------------------------------------------------------
# Diagnostics of MCMC samples (host, on the drawn samples)
# ---------------------------------------------------------------------------
def split_rhat(x: np.ndarray) -> np.ndarray:
    """Split-R-hat of samples x [T, C, d] (Gelman et al., Bayesian Data
    Analysis, 3rd ed., Sec. 11.4): each chain is cut in two halves; R-hat =
    sqrt(var+ / W) with W the mean within-half variance and var+ =
    (n-1)/n W + B/n, B/n the variance of the half means."""
    T = x.shape[0] - x.shape[0] % 2
    n = T // 2
    h = np.concatenate([x[:n], x[n:T]], axis=1)          # [n, 2C, d]
    means = h.mean(axis=0)
    W = h.var(axis=0, ddof=1).mean(axis=0)
    B_over_n = means.var(axis=0, ddof=1)
    var_plus = (n - 1) / n * W + B_over_n
    return np.sqrt(var_plus / W)


def ess(x: np.ndarray) -> np.ndarray:
    """Effective sample size of x [T, C, d] over all chains (Bayesian Data
    Analysis, 3rd ed., Sec. 11.5): rho_t = 1 - (W - mean over chains of the
    lag-t autocovariance) / var+; the sum runs over rho_1 .. rho_T' with T'
    the first odd lag for which rho_{T'+1} + rho_{T'+2} < 0;
    ESS = C T / (1 + 2 sum rho_t)."""
    T, C, d = x.shape
    xc = x - x.mean(axis=0, keepdims=True)
    W = x.var(axis=0, ddof=1).mean(axis=0)
    var_plus = (T - 1) / T * W + x.mean(axis=0).var(axis=0, ddof=1) if C > 1 else W
    f = np.fft.rfft(xc, n=2 * T, axis=0)
    acov = np.fft.irfft(f * np.conj(f), axis=0)[:T] / T          # [T, C, d], biased autocovariance
    acov_mean = acov.mean(axis=1)                                 # [T, d]
    rho = 1.0 - (W[None, :] - acov_mean) / var_plus[None, :]
    out = np.empty(d)
    for j in range(d):
        s = rho[1, j] if T > 1 else 0.0
        t = 2
        while t + 1 < T:
            pair = rho[t, j] + rho[t + 1, j]
            if pair < 0:
                break
            s += pair
            t += 2
        out[j] = C * T / (1.0 + 2.0 * s)
    return out


# ---------------------------------------------------------------------------
def elbo_summary(el: np.ndarray) -> dict:
    run_min = np.minimum.accumulate(el)
    late = el[100:] if len(el) > 100 else el
    return {"elbo_first": float(el[0]), "elbo_last100": float(np.median(el[-100:])),
            "elbo_min": float(el.min()),
            "steps_above_start_after_100": int(np.sum(late > el[0])),
            "max_rise_above_running_min": float(np.max(el - run_min))}


def compare_to_hmc(mean, var, samples: np.ndarray) -> dict:
    flat = samples.reshape(-1, samples.shape[-1]).astype(np.float64)
    mh, sh = flat.mean(axis=0), flat.std(axis=0)
    off = np.abs(np.asarray(mean, np.float64) - mh) / sh
    ratio = np.sqrt(np.asarray(var, np.float64)) / sh
    return {"mean_offset_sd_median": float(np.median(off)), "mean_offset_sd_max": float(off.max()),
            "std_ratio_median": float(np.median(ratio)), "std_ratio_min": float(ratio.min()),
            "std_ratio_max": float(ratio.max())}


@dataclass
class StudyConfig:
    systems: int = 8
    n_map: int = 4096
    steps_map: int = 1000
    n_vi: int = 1000
    steps_vi: int = 5000
    lr_vi: float = 1e-4
    chains: int = 128
    leapfrog: int = 10
    burn: int = 500
    n_hmc: int = 1500
    burn_rerun: int = 2000
    n_rerun: int = 7000
    mass_burn_factor: int = 10
    seed: int = 20267000


def _start_phi(plan, u0, d, dev):
    h = 1e-4
    probe = u0[None, :].repeat(2 * d, 1)
    idx = torch.arange(d, device=dev)
    probe[2 * idx, idx] += h
    probe[2 * idx + 1, idx] -= h
    _, g = lens.lens_logpost_grad(plan, probe.contiguous(), True)
    hd = ((g[2 * idx, idx] - g[2 * idx + 1, idx]) / (2 * h)).abs().double().cpu().numpy()
    sig = 0.5 / np.sqrt(np.maximum(hd, 1e-12))
    phi = np.zeros(lens.lens_svi_num_params(d))
    phi[:d] = u0.double().cpu().numpy()
    phi[d + np.arange(d) * (np.arange(d) + 3) // 2] = np.log(np.expm1(sig))     # softplus^-1 (shift 1e-10 ignored)
    return torch.tensor(phi, dtype=torch.float32, device=dev)


def study_system(sy, k, table, cfg: StudyConfig, dev, u_map, lp_map, log=print) -> dict:
    spec = sy.specs[k]
    d = spec.n_params
    t0 = time.perf_counter()
    plan = lens.LensPlan(spec, sy.psfs[k], sy.datas[k], sy.invvars[k], max(cfg.n_vi, cfg.chains, 2 * d), dev)
    plan.set_prior(table)
    phi0 = _start_phi(plan, u_map, d, dev)
    ut = lens.lens_to_unconstrained(plan, torch.tensor(sy.truths[k][None, :], dtype=torch.float32, device=dev))
    lp_truth, _ = lens.lens_logpost_grad(plan, ut, False)
    res = {"system": k, "side": spec.nx, "supersample": spec.supersample, "psf": spec.psf_size,
           "map_logp": lp_map, "truth_logp": float(lp_truth[0].item())}
    phis = {}
    for opt in ("adam", "adabelief"):
        x = phi0.clone()
        m = torch.zeros_like(x)
        s = torch.zeros_like(x)
        el = torch.empty(cfg.steps_vi, dtype=torch.float64, device=dev)
        lens.lens_svi_reset(plan)
        b1, b2, eps = (0.95, 0.99, 1e-16) if opt == "adabelief" else (0.9, 0.999, 1e-8)
        lens.lens_svi_run(plan, x, m, s, cfg.n_vi, cfg.steps_vi, opt, cfg.lr_vi, b1, b2, eps, cfg.seed + k,
                          elbo=el, use_graph=True)
        e = el.cpu().numpy()
        res[opt] = elbo_summary(e)
        res[opt]["finite"] = bool(np.all(np.isfinite(e)))
        phis[opt] = x
    # HMC from the AdaBelief surrogate
    C = cfg.chains
    _, _, var = lens.lens_svi_moments(plan, phis["adabelief"])
    _, _, u = lens.lens_svi_elbo_grad(plan, phis["adabelief"], C, cfg.seed + 500 + k, 0, want_u=True)
    u = u.contiguous()
    logp, grad = lens.lens_logpost_grad(plan, u, True)
    inv_mass = var.contiguous()
    acc = torch.zeros(C, dtype=torch.int32, device=dev)
    hseed = cfg.seed + 900 + k
    st = {"t": 0}

    def adapt(n, mass, eps0, window_start):
        """n burn-in transitions with the library's dual-averaged step size
        (target acceptance 0.8) and window variances."""
        _, fin, wv = lens.lens_hmc_adapt(plan, u, grad, logp, mass, eps0, 0.8, cfg.leapfrog, n, window_start, hseed,
                                         st["t"], use_graph=True)
        st["t"] += n
        return float(fin.item()), wv

    def sample(mass, eps, n):
        acc.zero_()
        samples = torch.empty((n, C, d), device=dev)
        lens.lens_hmc_run(plan, u, grad, logp, mass, eps, cfg.leapfrog, n, hseed, st["t"],
                          samples=samples, accepts=acc, use_graph=True)
        st["t"] += n
        smp = samples.cpu().numpy()
        del samples
        return smp, split_rhat(smp), ess(smp), float(acc.sum().item()) / (n * C)

    eps_h, _ = adapt(cfg.burn, inv_mass, 0.1, cfg.burn)
    smp, rh, es, a = sample(inv_mass, eps_h, cfg.n_hmc)
    res["hmc"] = {"eps": eps_h, "acceptance": a, "rhat_max": float(rh.max()), "ess_min": float(es.min()),
                  "mass_adapted": False, "rerun": False, "rhat_max_first": float(rh.max())}
    if rh.max() >= 1.1 and cfg.n_rerun > 0:
        # Sec. 4.2: non-converged systems are rerun with a longer burn-in and
        # more samples; the chains continue from where they are
        log(f"system {k}: split-R-hat {rh.max():.3f} after {cfg.n_hmc} samples; rerun with "
            f"{cfg.burn_rerun} burn-in and {cfg.n_rerun} samples")
        eps_h, _ = adapt(cfg.burn_rerun, inv_mass, eps_h, cfg.burn_rerun)
        smp, rh, es, a = sample(inv_mass, eps_h, cfg.n_rerun)
        res["hmc"].update({"eps": eps_h, "acceptance": a, "rhat_max": float(rh.max()), "ess_min": float(es.min()),
                           "rerun": True, "rhat_max_rerun": float(rh.max())})
    if rh.max() >= 1.1 and cfg.mass_burn_factor > 0:
        # mass-matrix adaptation (Sec. 3.3): a burn-in mass_burn_factor times
        # longer whose last 90 % give the variances of the new inverse mass;
        # the chains continue from where they are.  The step size is then
        # retuned over burn/5 transitions (the second burn-in phase the paper
        # names as a possible improvement), and the chains are sampled.
        nb = cfg.mass_burn_factor * cfg.burn
        eps_h, wv = adapt(nb, inv_mass, eps_h, nb // 10)
        inv_mass = wv.clamp_min(1e-30).contiguous()
        eps_h, _ = adapt(max(cfg.burn // 5, 10), inv_mass, eps_h, cfg.burn)
        smp, rh, es, a = sample(inv_mass, eps_h, cfg.n_rerun if cfg.n_rerun > 0 else cfg.n_hmc)
        res["hmc"].update({"eps": eps_h, "acceptance": a, "rhat_max": float(rh.max()), "ess_min": float(es.min()),
                           "mass_adapted": True})
    res["hmc"]["converged"] = bool(rh.max() < 1.1)
    for opt in ("adam", "adabelief"):
        mo, _, vo = lens.lens_svi_moments(plan, phis[opt])
        res[opt]["vs_hmc"] = compare_to_hmc(mo.cpu().numpy(), vo.cpu().numpy(), smp)
    torch.cuda.synchronize()
    plan.close()
    res["seconds"] = time.perf_counter() - t0
    log(f"system {k}: side {spec.nx} s {spec.supersample}: map {lp_map:.1f} (truth {res['truth_logp']:.1f}); "
        f"adam {res['adam']['elbo_last100']:.1f} (above start {res['adam']['steps_above_start_after_100']}), "
        f"adabelief {res['adabelief']['elbo_last100']:.1f} "
        f"(above start {res['adabelief']['steps_above_start_after_100']}); hmc acc {res['hmc']['acceptance']:.2f} "
        f"rhat {res['hmc']['rhat_max']:.3f} ess {res['hmc']['ess_min']:.0f} mass adapted "
        f"{res['hmc']['mass_adapted']}; {res['seconds']:.1f} s")
    return res


def run_study(cfg: StudyConfig, dev=None, log=print) -> dict:
    dev = dev or torch.device("cuda", 0)
    lens.load_library()
    sy = make_systems(cfg.systems, dev)
    table = synth.prior_table(synth.paper_prior_dists())
    mp = plain_arm(sy, table, cfg.n_map, Schedule(cfg.steps_map, 3e-2, 1e-4, 0.7), cfg.seed + 100,
                   log=log, tag="map")
    log(f"MAP: {cfg.systems} systems x {cfg.n_map} starts x {cfg.steps_map} steps, {mp.t_step * 1e3:.1f} ms/step")
    per = [study_system(sy, k, table, cfg, dev, mp.best_u[k].contiguous(), float(mp.best[-1, k]), log)
           for k in range(cfg.systems)]
    a = np.array([r["adam"]["elbo_last100"] for r in per])
    b = np.array([r["adabelief"]["elbo_last100"] for r in per])
    conv = [r for r in per if r["hmc"]["converged"]]
    summ = {
        "hmc_converged": len(conv),
        "hmc_converged_first_run": int(sum(r["hmc"]["rhat_max_first"] < 1.1 for r in per)),
        "hmc_converged_after_rerun": int(sum(r["hmc"].get("rhat_max_rerun", r["hmc"]["rhat_max_first"]) < 1.1
                                             for r in per)),
        "adabelief_lower_final_elbo": int(np.sum(b < a)),
        "final_elbo_adam_minus_adabelief_median": float(np.median(a - b)),
        "steps_above_start_after_100_adam": [r["adam"]["steps_above_start_after_100"] for r in per],
        "steps_above_start_after_100_adabelief": [r["adabelief"]["steps_above_start_after_100"] for r in per],
    }
    for opt in ("adam", "adabelief"):
        for key in ("std_ratio_median", "mean_offset_sd_median"):
            vals = [r[opt]["vs_hmc"][key] for r in conv]
            summ[f"{key}_{opt}_converged_systems"] = float(np.median(vals)) if vals else None
    return {"config": cfg.__dict__, "summary": summ, "per_system": per}


def main():
    ap = argparse.ArgumentParser()
    for f, v in StudyConfig().__dict__.items():
        ap.add_argument("--" + f.replace("_", "-"), type=type(v), default=v)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    cfg = StudyConfig(**{f: getattr(args, f) for f in StudyConfig().__dict__})
    res = run_study(cfg, log=lambda s: print(s, flush=True))
    print(json.dumps(res["summary"]), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
