"""Learned initializer: training data, training loop, and the time-to-MAP
comparison of learned against plain multi-start MAP.

The network is not part of the paper: it proposes starting particles for
the multi-start gradient-descent (MAP) stage of Sec. 3, which otherwise
starts from prior draws.  Everything numerical runs in the library's HIP
kernels (forward model, network training and inference, proposals, prior
draws, bijection, posterior, Adam, per-system best); this module sequences
the calls, shuffles indices and keeps the bookkeeping.

Regressed parameters (14 of the 22 of the EPL + shear + one Sersic lens
light + one Sersic source model, TARGET_IDX): theta_E, gamma, the mass
ellipticity (e1, e2), the external shear (g1, g2), the lens light's R_e and
n, and the source's R_e, n, e1, e2, x, y.  The source position is what
makes the MAP objective multi-modal, so the network's proposals matter most
there; the parameters left to the prior (mass centre, lens-light
ellipticity and centre, both intensities) have tight priors or, for the
intensities, an objective that gradient descent handles from any start.

Time-to-MAP of a system (per arm): wall-clock from the start of the arm
(network inference and proposals included, plan creation excluded) until
the best particle's log-posterior reaches L_ref - 1, with L_ref the best
log-posterior found for that system by either arm or by a final polishing
run from both arms' best particles.  Fallback: when the learned arm's best
particle leaves a reduced chi^2 above 1 + 5 sqrt(2 / N_pix), the system is
rerun from plain prior starts and that time is added to the learned arm.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import lens, synth

N_TARGETS = 14
# columns of the 22-parameter vector regressed by the network (network output k -> parameter TARGET_IDX[k])
TARGET_IDX = np.array([0, 1, 2, 3, 6, 7, 8, 9, 15, 16, 17, 18, 19, 20])
SIDE = 64
SIGMA = synth.SIGMA_NOISE


def train_spec() -> synth.ModelSpec:
    """Training images: 64x64 px at 0.05"/px, 2x2 supersampling, 21x21 PSF."""
    return synth.paper_spec(SIDE, 2, 21)


def _sync():
    torch.cuda.synchronize()
    return time.perf_counter()


def simulate(n: int, seed: int, device, chunk: int = 8192):
    """Parameters [n, 22] (numpy, from the simulation distribution) and the
    noiseless model images [n, 64, 64] rendered by lens_forward."""
    spec = train_spec()
    theta = synth.draw_params(synth.paper_sim_dists(), n, seed).astype(np.float32)
    psf = synth.double_gaussian_psf(spec.psf_size, spec.pix_scale)
    zero = np.zeros((spec.ny, spec.nx), np.float32)
    plan = lens.LensPlan(spec, psf, zero, zero + 1.0, min(chunk, n), device)
    images = torch.empty((n, SIDE, SIDE), dtype=torch.float32, device=device)
    th = torch.tensor(theta, device=device)
    for i in range(0, n, chunk):
        j = min(n, i + chunk)
        lens.lens_forward(plan, th[i:j].contiguous(), out=images[i:j])
    torch.cuda.synchronize()
    plan.close()
    return theta, images


def target_standardization(theta: np.ndarray):
    t = theta[:, TARGET_IDX].astype(np.float64)
    return t.mean(axis=0).astype(np.float32), t.std(axis=0).astype(np.float32)


@dataclass
class TrainReport:
    images: int
    epochs: int
    batch: int
    seconds: float
    images_per_s: float
    loss_first: float
    loss_last: float
    val_nll: float
    val_rmse_std: List[float] = field(default_factory=list)


def train(net: lens.Cnn, images: torch.Tensor, theta: np.ndarray, mean, std, epochs: int, batch: int = 256,
          lr: float = 1e-3, lr_final: float = 1e-4, seed: int = synth.SEED_CNN_TRAIN, log=print,
          val=None) -> TrainReport:
    """Adam on the Gaussian NLL of the standardised targets; fresh noise on
    every pass (Philox, counter = image draw index)."""
    dev = images.device
    n = images.shape[0]
    tgt = torch.tensor((theta[:, TARGET_IDX] - mean) / std, dtype=torch.float32, device=dev)
    xb = torch.empty((batch, SIDE, SIDE), dtype=torch.bfloat16, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    steps = max(1, n // batch)
    total = steps * epochs
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    first = None
    t0 = _sync()
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            x = images.index_select(0, idx)
            draw = (ep * steps + s) * batch
            net.prepare(x, SIGMA, add_noise=True, seed=seed, counter0=draw * SIDE * SIDE, out=xb)
            rate = lr * (lr_final / lr) ** (k / max(1, total - 1))
            net.train_step(xb, tgt.index_select(0, idx), rate, loss)
            k += 1
            if first is None:
                first = float(loss.item())
        log(f"epoch {ep + 1}/{epochs} loss {float(loss.item()):.4f}")
    t1 = _sync()
    last = float(loss.item())
    rep = TrainReport(n, epochs, batch, t1 - t0, steps * epochs * batch / (t1 - t0), first, last, float("nan"))
    if val is not None:
        vtheta, vimages = val
        nll, rmse = evaluate(net, vimages, vtheta, mean, std)
        rep.val_nll, rep.val_rmse_std = nll, rmse
        log(f"validation nll {nll:.4f} rmse/std {np.round(rmse, 3).tolist()}")
    return rep


def evaluate(net: lens.Cnn, images: torch.Tensor, theta: np.ndarray, mean, std, seed: int = synth.SEED_CNN_VAL):
    """Mean NLL and per-target RMSE of the predicted means (standardised units)."""
    dev = images.device
    n = images.shape[0]
    B = net.max_batch
    outs = []
    for i in range(0, n, B):
        j = min(n, i + B)
        xb = net.prepare(images[i:j], SIGMA, add_noise=True, seed=seed, counter0=i * SIDE * SIDE)
        outs.append(net.forward(xb))
    out = torch.cat(outs).double().cpu().numpy()
    z = (theta[:, TARGET_IDX].astype(np.float64) - mean) / std
    mu, s = out[:, :N_TARGETS], out[:, N_TARGETS:]
    nll = float(np.mean(np.sum(0.5 * (z - mu) ** 2 * np.exp(-s) + 0.5 * s, axis=1)))
    rmse = np.sqrt(np.mean((z - mu) ** 2, axis=0))
    return nll, rmse.tolist()


def configure(net: lens.Cnn, mean, std):
    table = synth.prior_table(synth.paper_prior_dists())
    slot = np.full(table.shape[0], -1, np.int32)
    slot[TARGET_IDX] = np.arange(N_TARGETS)
    net.set_target_map(table, slot, mean, std, SIGMA)
    return table


# ---------------------------------------------------------------------------
# Time-to-MAP
# ---------------------------------------------------------------------------
@dataclass
class Systems:
    specs: list
    psfs: list
    datas: list
    invvars: list
    truths: np.ndarray


def make_systems(n: int, device) -> Systems:
    """The uneven batch (sides 48-160 px, supersampling 2-4, PSF 11-31 px),
    observed images = lens_forward at the seeded truth + seeded noise."""
    specs = synth.uneven_batch_specs(n)
    psfs, datas, invvars, truths = [], [], [], []
    for k, spec in enumerate(specs):
        s = synth.make_system_paper(spec, k)
        zero = np.zeros((spec.ny, spec.nx), np.float32)
        plan = lens.LensPlan(spec, s.psf, zero, s.invvar, 1, device)
        model = lens.lens_forward(plan, torch.tensor(s.truth[None, :], device=device))[0]
        datas.append((model + torch.tensor(s.noise, device=device)).contiguous())
        psfs.append(torch.tensor(s.psf, device=device))
        invvars.append(torch.tensor(s.invvar, device=device))
        truths.append(s.truth)
        torch.cuda.synchronize()
        plan.close()
    torch.cuda.synchronize()
    return Systems(specs, psfs, datas, invvars, np.asarray(truths))


def _plan(sy: Systems, per_system, table, idx=None):
    idx = list(range(len(sy.specs))) if idx is None else list(idx)
    per = per_system if isinstance(per_system, (list, tuple)) else [per_system] * len(idx)
    bp = lens.BatchPlan([sy.specs[k] for k in idx], [sy.psfs[k] for k in idx], [sy.datas[k] for k in idx],
                        [sy.invvars[k] for k in idx], per, sy.datas[0].device)
    bp.set_prior(table)
    return bp


@dataclass
class ArmRun:
    t_init: float              # s, proposals + bijection
    t_step: float              # s per Adam step (with per-system best tracking)
    steps: int
    best: np.ndarray           # [steps + 1, S] best log-posterior after t updates
    best_u: torch.Tensor       # [S, d] best particle at the end


def run_arm(bp: lens.BatchPlan, theta0_fn, steps: int, lr: float, lr_final: float, log=print,
            tag: str = "", start_is_u: bool = False, hold: float = 0.0) -> ArmRun:
    """theta0_fn() -> packed starting points [N, d] (timed; unconstrained if
    start_is_u).  Then `steps` Adam updates (graph replay) with the
    per-system best after each.  Learning rate: lr for the first
    round(hold * steps) updates, then geometric decay to lr_final."""
    dev = bp.device
    n1 = int(round(hold * steps))
    n2 = steps - n1
    decay = (lr_final / lr) ** (1.0 / max(1, n2 - 1))
    # the kernel's rate at update k (1-based) is lr_arg * decay_arg^(k - 1)
    phases = [(n1, lr, 1.0), (n2, lr / decay ** n1, decay)]
    m = torch.zeros((bp.N, bp.d), dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    loss = torch.empty(bp.N, dtype=torch.float32, device=dev)
    hist = torch.empty((steps + 1, bp.S), dtype=torch.float32, device=dev)
    bp.map_reset()
    t0 = _sync()
    start = theta0_fn()
    u = start.clone() if start_is_u else bp.to_unconstrained(start)
    t1 = _sync()
    t = 0
    for n, lr_arg, dec in phases:
        for _ in range(n):
            bp.map_adam(u, m, v, 1, lr_arg, dec, loss=loss, use_graph=True)
            hist[t].copy_(bp.argmin(loss)[0])
            t += 1
            if t % 50 == 0:
                torch.cuda.synchronize()
                log(f"{tag} step {t}/{steps}")
    t2 = _sync()
    logp, _ = bp.logpost_grad(u, False)
    final = (-logp).float().contiguous()
    bv, arg = bp.argmin(final)
    hist[steps].copy_(bv)
    best_u = u.index_select(0, arg.long())
    torch.cuda.synchronize()
    return ArmRun(t1 - t0, (t2 - t1) / max(1, steps), steps, -hist.double().cpu().numpy(), best_u)


def polish(sy: Systems, table, us: List[torch.Tensor], steps: int = 400, lr: float = 2e-3, lr_final: float = 1e-5):
    """Adam from each arm's best particle; returns the best log-posterior seen per system."""
    S = len(sy.specs)
    k = len(us)
    bp = _plan(sy, k, table)
    u = torch.stack(us, dim=1).reshape(S * k, -1).contiguous()
    run = run_arm(bp, lambda: u, steps, lr, lr_final, log=lambda *_: None, start_is_u=True)
    bp.close()
    return run.best.max(axis=0)


def best_chi2_nu(sy: Systems, table, best_u: torch.Tensor, idx=None) -> np.ndarray:
    idx = list(range(len(sy.specs))) if idx is None else list(idx)
    bp = _plan(sy, 1, table, idx)
    _, _, theta = bp.logpost_grad(best_u.contiguous(), False, want_theta=True)
    logl, _ = bp.loglike_grad(theta)
    npix = np.array([sy.specs[k].nx * sy.specs[k].ny for k in idx], np.float64)
    bp.close()
    return -2.0 * logl.double().cpu().numpy() / npix


def time_to_reach(run: ArmRun, target: np.ndarray) -> np.ndarray:
    """Seconds until the best log-posterior of each system reaches target (inf if never)."""
    out = np.full(run.best.shape[1], np.inf)
    for s in range(run.best.shape[1]):
        hit = np.nonzero(run.best[:, s] >= target[s])[0]
        if hit.size:
            out[s] = run.t_init + (hit[0] + 1) * run.t_step
    return out


def _save_arm(path: str, run: ArmRun, **extra):
    np.savez(path, t_init=run.t_init, t_step=run.t_step, steps=run.steps, best=run.best,
             best_u=run.best_u.cpu().numpy(), **extra)


def _load_arm(path: str, device):
    z = np.load(path)
    run = ArmRun(float(z["t_init"]), float(z["t_step"]), int(z["steps"]), z["best"],
                 torch.tensor(z["best_u"], device=device))
    return run, {k: z[k] for k in z.files if k not in ("t_init", "t_step", "steps", "best", "best_u")}


def _concat_arms(parts: List[ArmRun]) -> ArmRun:
    """Arms run on disjoint groups of systems, taken as one batch: the per-step
    time of the whole batch is the sum of the groups' (the same work)."""
    return ArmRun(sum(r.t_init for r in parts), sum(r.t_step for r in parts), parts[0].steps,
                  np.concatenate([r.best for r in parts], axis=1), torch.cat([r.best_u for r in parts]))


@dataclass
class Schedule:
    steps: int = 1000
    lr: float = 3e-2
    lr_final: float = 1e-4
    hold: float = 0.7


def learned_arm(net: lens.Cnn, sy: Systems, table, n: int, sch: Schedule, seed: int, log=print):
    S = len(sy.specs)
    bp = _plan(sy, n, table)
    flags = {}

    def start():
        views = bp.center_views(SIDE)
        th, fl = lens.init_propose(net, views, n, seed)
        flags["f"] = fl
        return th.reshape(bp.N, bp.d)

    run = run_arm(bp, start, sch.steps, sch.lr, sch.lr_final, log, "learned", hold=sch.hold)
    bp.close()
    chi = best_chi2_nu(sy, table, run.best_u)
    return run, chi, flags["f"].cpu().numpy()


def plain_arm(sy: Systems, table, n: int, sch: Schedule, seed: int, idx=None, log=print, tag="plain"):
    idx = list(range(len(sy.specs))) if idx is None else list(idx)
    bp = _plan(sy, n, table, idx)
    dev = sy.datas[0].device
    # one draw for the whole batch, so that a group of systems sees the same
    # starting points as in a single run (Philox counters use the system index)

    sel = torch.as_tensor(np.asarray(idx, dtype=np.int64), device=dev)

    def start():
        th = lens.lens_prior_sample(table, max(idx) + 1, n, seed, dev)
        return th.index_select(0, sel).reshape(bp.N, bp.d).contiguous()

    run = run_arm(bp, start, sch.steps, sch.lr, sch.lr_final, log, tag, hold=sch.hold)
    bp.close()
    return run


def summarize(sy: Systems, table, learned: ArmRun, chi, flags, plain: ArmRun, sch: Schedule, n_learned: int,
              n_plain: int, seed: int, log=print, save_dir: Optional[str] = None) -> Dict:
    """Fallback reruns, L_ref and the time-to-MAP statistics.

    Primary L_ref: the best log-posterior seen for the system in any run
    (learned arm, plain arm, fallback rerun).  Also reported: the stricter
    reference that adds a polishing run from the runs' best particles."""
    import os
    S = len(sy.specs)
    npix = np.array([sp.nx * sp.ny for sp in sy.specs], np.float64)
    thr = 1.0 + 5.0 * np.sqrt(2.0 / npix)
    fb = np.nonzero(chi > thr)[0]
    chi_plain = best_chi2_nu(sy, table, plain.best_u)
    log(f"fallback systems ({fb.size}): {fb.tolist()}")
    rerun = plain_arm(sy, table, n_plain, sch, seed + 2, fb, log, "fallback") if fb.size else None
    ref = np.maximum(learned.best.max(axis=0), plain.best.max(axis=0))
    starts = [learned.best_u, plain.best_u]
    if rerun is not None:
        ref[fb] = np.maximum(ref[fb], rerun.best.max(axis=0))
        fb_u = learned.best_u.clone()
        fb_u[torch.as_tensor(fb, device=fb_u.device)] = rerun.best_u
        starts.append(fb_u)
    pol = polish(sy, table, starts)
    if save_dir:
        if rerun is not None:
            _save_arm(os.path.join(save_dir, "fallback.npz"), rerun, idx=fb)
        np.save(os.path.join(save_dir, "polish.npy"), pol)
    learned_total = learned.t_init + sch.steps * learned.t_step
    final_learned = learned.best[-1].copy()
    if rerun is not None:
        final_learned[fb] = np.maximum(final_learned[fb], rerun.best[-1])
    d_final = final_learned - plain.best[-1]

    def times(target):
        # the learned arm's best particle first reaching the target: during its
        # own run, else (fallback systems) during the rerun that follows it
        t_plain = time_to_reach(plain, target)
        t_learn = time_to_reach(learned, target)
        if rerun is not None:
            late = learned_total + time_to_reach(rerun, target[fb])
            t_learn[fb] = np.where(np.isfinite(t_learn[fb]), t_learn[fb], late)
        return t_learn, t_plain

    def summ(t):
        ok = np.isfinite(t)
        return {"success_frac": float(ok.mean()),
                "median_s": float(np.median(t[ok])) if ok.any() else None,
                "mean_s": float(np.mean(t[ok])) if ok.any() else None,
                "max_s": float(np.max(t[ok])) if ok.any() else None}

    def block(target):
        t_learn, t_plain = times(target)
        both = np.isfinite(t_plain) & np.isfinite(t_learn)
        # a system never reached counts as the arm's whole run time (a lower bound)
        tl = np.where(np.isfinite(t_learn), t_learn, learned_total + (sch.steps * rerun.t_step
                                                                     if rerun is not None else 0.0))
        tp = np.where(np.isfinite(t_plain), t_plain, plain.t_init + sch.steps * plain.t_step)
        return {"learned": summ(t_learn), "plain": summ(t_plain),
                "speedup_median_both_reached": float(np.median(t_plain[both] / t_learn[both])) if both.any()
                else None,
                "systems_both_reached": int(both.sum()),
                "median_time_all_systems_s": {"learned": float(np.median(tl)), "plain": float(np.median(tp))},
                "per_system": {"time_learned_s": t_learn.tolist(), "time_plain_s": t_plain.tolist()}}

    return {
        "systems": S, "schedule": {"steps": sch.steps, "lr": sch.lr, "lr_final": sch.lr_final, "hold": sch.hold},
        "learned": {"particles_per_system": n_learned, "t_init_s": learned.t_init,
                    "ms_per_step": learned.t_step * 1e3, "total_s": learned_total,
                    "clipped_proposal_systems": int(np.sum(flags)),
                    "chi2_nu_pass_frac": float(np.mean(chi <= thr)),
                    "fallback_systems": fb.tolist(),
                    "fallback_ms_per_step": rerun.t_step * 1e3 if rerun is not None else None},
        "plain": {"particles_per_system": n_plain, "t_init_s": plain.t_init,
                  "ms_per_step": plain.t_step * 1e3, "total_s": plain.t_init + sch.steps * plain.t_step,
                  "chi2_nu_pass_frac": float(np.mean(chi_plain <= thr))},
        "time_to_map": block(ref - 1.0),
        "time_to_map_polished_ref": block(np.maximum(ref, pol) - 1.0),
        "final_logp_learned_minus_plain": {"median": float(np.median(d_final)), "min": float(np.min(d_final)),
                                           "max": float(np.max(d_final)),
                                           "frac_learned_not_worse_by_1": float(np.mean(d_final >= -1.0))},
        "per_system": {"L_ref": ref.tolist(), "polished": pol.tolist(), "final_learned": final_learned.tolist(),
                       "final_plain": plain.best[-1].tolist(), "chi2_nu_learned": chi.tolist(),
                       "chi2_nu_plain": chi_plain.tolist(), "npix": npix.tolist()},
    }


def time_to_map_experiment(net: lens.Cnn, n_systems: int = 100, n_learned: int = 512, n_plain: int = 4096,
                           sch: Schedule = Schedule(), seed: int = 7, device="cuda", log=print) -> Dict:
    """Both arms in one call (small runs; the full comparison runs in stages, see main)."""
    table = synth.prior_table(synth.paper_prior_dists())
    sy = make_systems(n_systems, device)
    learned, chi, flags = learned_arm(net, sy, table, n_learned, sch, seed, log)
    plain = plain_arm(sy, table, n_plain, sch, seed + 1, None, log)
    return summarize(sy, table, learned, chi, flags, plain, sch, n_learned, n_plain, seed, log)


def main(argv=None):
    """Stages (each one GPU process; state in --state, read from --load):
      train    simulate the training set, train, save the network
      learned  learned arm on all systems (+ reduced chi^2 of its best particles)
      plain    plain arm on group --part of --parts groups of systems
      finish   fallback reruns, polishing, statistics -> --out
    """
    import argparse
    import os
    ap = argparse.ArgumentParser(description="Train the learned initializer and compare time-to-MAP")
    ap.add_argument("stage", choices=["train", "learned", "plain", "finish"])
    ap.add_argument("--state", required=True)
    ap.add_argument("--load", default=None)
    ap.add_argument("--train-images", type=int, default=200000)
    ap.add_argument("--val-images", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--systems", type=int, default=100)
    ap.add_argument("--learned", type=int, default=512)
    ap.add_argument("--plain", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--lr", type=float, default=3e-2)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--hold", type=float, default=0.7)
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", type=str, default=None)
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    os.makedirs(args.state, exist_ok=True)
    load = args.load or args.state
    sch = Schedule(args.steps, args.lr, args.lr_final, args.hold)
    table = synth.prior_table(synth.paper_prior_dists())

    def log(msg):
        print(msg, flush=True)

    if args.stage == "train":
        t0 = time.perf_counter()
        theta, images = simulate(args.train_images, synth.SEED_CNN_TRAIN, dev)
        vtheta, vimages = simulate(args.val_images, synth.SEED_CNN_VAL, dev)
        t_sim = time.perf_counter() - t0
        log(f"simulated {args.train_images} + {args.val_images} images in {t_sim:.1f} s")
        mean, std = target_standardization(theta)
        net = lens.Cnn(args.batch, 1, dev)
        rep = train(net, images, theta, mean, std, args.epochs, args.batch, lr=2e-3, lr_final=1e-4, log=log,
                    val=(vtheta, vimages))
        np.save(os.path.join(args.state, "cnn_params.npy"), net.get_params().cpu().numpy())
        np.save(os.path.join(args.state, "cnn_mean.npy"), mean)
        np.save(os.path.join(args.state, "cnn_std.npy"), std)
        with open(os.path.join(args.state, "training.json"), "w") as f:
            json.dump({"images": rep.images, "epochs": rep.epochs, "batch": rep.batch, "seconds": rep.seconds,
                       "images_per_s": rep.images_per_s, "simulate_s": t_sim, "loss_first": rep.loss_first,
                       "loss_last": rep.loss_last, "val_nll": rep.val_nll, "val_rmse_std": rep.val_rmse_std}, f)
        return
    sy = make_systems(args.systems, dev)
    if args.stage == "learned":
        net = lens.Cnn(256, 1, dev)
        net.set_params(torch.tensor(np.load(os.path.join(load, "cnn_params.npy")), device=dev))
        configure(net, np.load(os.path.join(load, "cnn_mean.npy")), np.load(os.path.join(load, "cnn_std.npy")))
        run, chi, flags = learned_arm(net, sy, table, args.learned, sch, args.seed, log)
        _save_arm(os.path.join(args.state, "learned.npz"), run, chi=chi, flags=flags)
        log(f"learned arm: {run.t_step * 1e3:.2f} ms/step, reduced chi^2 median {np.median(chi):.3f}")
    elif args.stage == "plain":
        idx = np.array_split(np.arange(args.systems), args.parts)[args.part]
        run = plain_arm(sy, table, args.plain, sch, args.seed + 1, idx, log)
        _save_arm(os.path.join(args.state, f"plain_{args.part}_of_{args.parts}.npz"), run, idx=idx)
        log(f"plain arm part {args.part}: {run.t_step * 1e3:.2f} ms/step")
    else:
        learned, extra = _load_arm(os.path.join(load, "learned.npz"), dev)
        parts = [_load_arm(os.path.join(load, f"plain_{p}_of_{args.parts}.npz"), dev)[0] for p in range(args.parts)]
        res = summarize(sy, table, learned, extra["chi"], extra["flags"], _concat_arms(parts), sch, args.learned,
                        args.plain, args.seed, log, save_dir=args.state)
        tj = os.path.join(load, "training.json")
        if os.path.exists(tj):
            res["training"] = json.load(open(tj))
        if args.out:
            with open(args.out, "w") as f:
                f.write(json.dumps(res) + "\n")
        print(json.dumps({k: v for k, v in res.items() if k != "per_system"}), flush=True)


if __name__ == "__main__":
    main()
