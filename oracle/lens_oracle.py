"""FP64 CPU oracle of the batched strong-lens forward model and likelihood.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain definition that the
GPU path is checked against.  Only the test-suite, the package smoke check
and the benchmark's CPU-baseline leg may import it; the product never does,
and it imports nothing from the product.  It shares no code with the HIP
kernels.

Everything is written with plain PyTorch CPU operations in float64 on whole
sub-pixel grids; the gradient is PyTorch autograd applied to this same plain
definition (no hand-written derivative).  Inputs that arrive as float32 are
promoted once, so the oracle evaluates exactly the values the GPU sees.

What is computed (paper Sec. 3, "Methodology"; Sec. 4.2 footnote on
supersampling).  The paper names the model components and defers their
formulas to the GIGA-Lens 1.0 paper, which is not available here, so each
formula below is a published lensing result, restated:

  grid        integer-supersampled pixel grid centred on the cutout
  ellipticity (e1, e2) -> axis ratio q = (1-c)/(1+c), angle phi = atan2(e2,e1)/2,
              c = |e|; profiles are evaluated in the frame rotated by phi
              about each component's own centre
  EPL         deflection of kappa = (2-t)/2 (b/R)^t, R = sqrt(q^2 x'^2 + y'^2),
              t = gamma - 1, b = theta_E sqrt(q), by the hypergeometric series
              of Tessore & Metcalf (2015, A&A 580, A79)
  SIE         the same profile at t = 1 in closed form (Kormann et al. 1994)
  shear       alpha = (g1 x + g2 y, g2 x - g1 y) about the origin
  lens eq.    beta = theta - alpha_mass - alpha_shear
  Sersic      I_e exp(-b_n[(R/R_e)^(1/n) - 1]), R = sqrt(q x'^2 + y'^2/q),
              b_n = 1.9992 n - 0.3271; lens light at theta, sources at beta
  shapelets   optional shapelet source at beta: sum_k c_k phi_k(x - xc, y - yc;
              beta), the Cartesian basis of Refregier (2003) up to order n_max
  downsample  mean over the s x s sub-pixels of each pixel
  PSF         zero-padded 'same' 2-D convolution with an odd K x K kernel
  logL        -1/2 sum w (d - m)^2  (Gaussian, w = inverse variance)
  stages      prior and bijection, Adam, HMC with Philox draws, and SVI: a
              full-covariance Gaussian surrogate, its Monte-Carlo ELBO with
              the pathwise gradient, Adam or AdaBelief updates

Pins: tests/test_oracle_*.py check these functions against closed forms,
invariants, library routines and brute force (SIS, EPL->SIE at gamma = 2,
Poisson equation, Keeton's 1-D integral, Sersic flux via the incomplete
gamma function, delta-PSF, chi-square statistics, finite differences; for
SVI the closed-form KL of a Gaussian target and the AdaBelief closed form
under a constant gradient; for shapelets numpy's Hermite polynomials, the
basis's orthonormality and 1-D fluxes, superposition with the Sersic model,
least-squares recovery of the coefficients).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

DT = torch.float64
R_MIN = 1e-6             # arcsec; radii are clamped to this (both profiles)
SERIES_REL_TOL = 1e-17   # EPL series stops once every term is below this x |sum|
SERIES_MAX_TERMS = 500

PRIOR_UNIFORM, PRIOR_NORMAL, PRIOR_LOGNORMAL, PRIOR_TRUNCNORMAL = 0, 1, 2, 3


def _t(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(DT)
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=DT)


# ---------------------------------------------------------------------------
# Parameter layout (Sec. 3 lists the parameters of each component)
# ---------------------------------------------------------------------------
def n_shapelet_coeffs(spec) -> int:
    """Coefficients of the shapelet source, (n_max + 1)(n_max + 2)/2, or 0."""
    if not getattr(spec, "n_shapelet", 0):
        return 0
    n = spec.shapelet_nmax
    return (n + 1) * (n + 2) // 2


def n_params(spec) -> int:
    nsh = n_shapelet_coeffs(spec)
    return ((8 if spec.mass_model == "EPL" else 7) + 7 * (spec.n_lens_light + spec.n_source)
            + (3 + nsh if getattr(spec, "n_shapelet", 0) else 0))


def unpack(theta: torch.Tensor, spec) -> Dict[str, object]:
    """Split one parameter vector into named components (canonical order)."""
    i = 0
    out: Dict[str, object] = {}
    out["theta_E"] = theta[i]; i += 1
    if spec.mass_model == "EPL":
        out["gamma"] = theta[i]; i += 1
    else:
        out["gamma"] = None
    out["m_e1"], out["m_e2"], out["m_x"], out["m_y"] = theta[i], theta[i + 1], theta[i + 2], theta[i + 3]
    i += 4
    out["g1"], out["g2"] = theta[i], theta[i + 1]
    i += 2
    lights, sources = [], []
    for _ in range(spec.n_lens_light):
        lights.append(tuple(theta[i + k] for k in range(7))); i += 7
    for _ in range(spec.n_source):
        sources.append(tuple(theta[i + k] for k in range(7))); i += 7
    out["lights"], out["sources"] = lights, sources
    # optional shapelet source (Sec. 3: Sersic profiles and/or shapelets for
    # the source light): (beta, x, y, coefficients in shapelet_indices order)
    out["shapelet"] = None
    if getattr(spec, "n_shapelet", 0):
        nb = n_shapelet_coeffs(spec)
        out["shapelet"] = (theta[i], theta[i + 1], theta[i + 2], theta[i + 3:i + 3 + nb])
        i += 3 + nb
    return out


# ---------------------------------------------------------------------------
# Step 1: supersampled grid (Sec. 4.2 footnote: integer supersampling)
# ---------------------------------------------------------------------------
def subpixel_grid(nx: int, ny: int, pix: float, s: int) -> Tuple[torch.Tensor, torch.Tensor]:
    """Sub-pixel centre coordinates, arrays [ny*s, nx*s] (row = y, column = x).

    Pixel (i, j) is centred at x_j = (j - (nx-1)/2) pix, y_i = (i - (ny-1)/2) pix;
    its sub-pixel (a, b) is offset by ((b + 1/2)/s - 1/2) pix in x and
    ((a + 1/2)/s - 1/2) pix in y.
    """
    xc = (torch.arange(nx, dtype=DT) - (nx - 1) / 2.0) * pix
    yc = (torch.arange(ny, dtype=DT) - (ny - 1) / 2.0) * pix
    off = ((torch.arange(s, dtype=DT) + 0.5) / s - 0.5) * pix
    xs = (xc[:, None] + off[None, :]).reshape(-1)
    ys = (yc[:, None] + off[None, :]).reshape(-1)
    Y, X = torch.meshgrid(ys, xs, indexing="ij")
    return X, Y


# ---------------------------------------------------------------------------
# Step 2: ellipticity and rotated frame (Sec. 3: eccentricities e1, e2)
# ---------------------------------------------------------------------------
def ellipticity_to_q_phi(e1, e2):
    c = torch.sqrt(e1 * e1 + e2 * e2)
    q = (1.0 - c) / (1.0 + c)
    phi = 0.5 * torch.atan2(e2, e1)
    return q, phi


def to_frame(x, y, x0, y0, phi):
    dx, dy = x - x0, y - y0
    cp, sp = torch.cos(phi), torch.sin(phi)
    return cp * dx + sp * dy, -sp * dx + cp * dy


def from_frame(ax, ay, phi):
    cp, sp = torch.cos(phi), torch.sin(phi)
    return cp * ax - sp * ay, sp * ax + cp * ay


# ---------------------------------------------------------------------------
# Step 3: EPL deflection, Tessore & Metcalf (2015) series
# ---------------------------------------------------------------------------
def epl_deflection(x, y, theta_E, gamma, e1, e2, x0, y0, n_terms: Optional[int] = None,
                   return_terms: bool = False):
    """Deflection of the elliptical power law, in the image frame.

    In the rotated frame, with R = sqrt(q^2 x'^2 + y'^2) and
    e^{i phi_R} = (q x' + i y') / R:
        alpha' = 2b/(1+q) (b/R)^(t-1) e^{i phi_R} sum_n W_n,
        W_0 = 1,  W_n = W_{n-1} * [-f (2n - 2 + t)/(2n + 2 - t)] e^{2 i phi_R},
    f = (1-q)/(1+q).  The series is summed until every term is below
    SERIES_REL_TOL of the running sum (or exactly ``n_terms`` terms beyond
    W_0 if given).  alpha = 0 where R < R_MIN.
    """
    q, phi = ellipticity_to_q_phi(e1, e2)
    t = gamma - 1.0
    b = theta_E * torch.sqrt(q)
    f = (1.0 - q) / (1.0 + q)
    xp, yp = to_frame(x, y, x0, y0, phi)
    R2 = q * q * xp * xp + yp * yp
    inside = R2 < R_MIN * R_MIN
    R = torch.sqrt(torch.where(inside, torch.full_like(R2, R_MIN * R_MIN), R2))
    ec, es = q * xp / R, yp / R                    # e^{i phi_R}
    c2, s2 = ec * ec - es * es, 2.0 * ec * es      # e^{2 i phi_R}
    wr, wi = torch.ones_like(R), torch.zeros_like(R)
    sr, si = wr, wi
    n = 1
    used = 0
    while True:
        ratio = -f * (2.0 * n - 2.0 + t) / (2.0 * n + 2.0 - t)
        wr, wi = ratio * (wr * c2 - wi * s2), ratio * (wr * s2 + wi * c2)
        sr, si = sr + wr, si + wi
        used = n
        if n_terms is not None:
            if n >= n_terms:
                break
        else:
            with torch.no_grad():
                mag_t = torch.sqrt(wr * wr + wi * wi).max()
                mag_s = torch.sqrt(sr * sr + si * si).min()
            if mag_t <= SERIES_REL_TOL * mag_s or n >= SERIES_MAX_TERMS:
                break
        n += 1
    pref = 2.0 * b / (1.0 + q) * torch.pow(b / R, t - 1.0)
    axp = pref * (ec * sr - es * si)
    ayp = pref * (ec * si + es * sr)
    zero = torch.zeros_like(axp)
    axp = torch.where(inside, zero, axp)
    ayp = torch.where(inside, zero, ayp)
    ax, ay = from_frame(axp, ayp, phi)
    if return_terms:
        return ax, ay, used
    return ax, ay


def sie_deflection(x, y, theta_E, e1, e2, x0, y0):
    """Singular isothermal ellipsoid (t = 1) in closed form.

    With psi = sqrt(q^2 x'^2 + y'^2) and s = sqrt(1 - q^2):
        alpha'_x = b/s atan(s x'/psi),  alpha'_y = b/s atanh(s y'/psi),
    b = theta_E sqrt(q); the q -> 1 limit is b (x', y')/psi.  alpha = 0 where
    psi < R_MIN.
    """
    q, phi = ellipticity_to_q_phi(e1, e2)
    b = theta_E * torch.sqrt(q)
    xp, yp = to_frame(x, y, x0, y0, phi)
    R2 = q * q * xp * xp + yp * yp
    inside = R2 < R_MIN * R_MIN
    psi = torch.sqrt(torch.where(inside, torch.full_like(R2, R_MIN * R_MIN), R2))
    s = torch.sqrt(1.0 - q * q)
    if float(s.detach()) > 1e-7:
        axp = b / s * torch.atan(s * xp / psi)
        ayp = b / s * torch.atanh(s * yp / psi)
    else:
        axp = b * xp / psi
        ayp = b * yp / psi
    zero = torch.zeros_like(axp)
    axp = torch.where(inside, zero, axp)
    ayp = torch.where(inside, zero, ayp)
    return from_frame(axp, ayp, phi)


def shear_deflection(x, y, g1, g2):
    """External shear about the origin: alpha = (g1 x + g2 y, g2 x - g1 y)."""
    return g1 * x + g2 * y, g2 * x - g1 * y


# ---------------------------------------------------------------------------
# Step 6: elliptical Sersic surface brightness
# ---------------------------------------------------------------------------
def sersic_bn(n):
    """Capaccioli (1989) linear approximation of the Sersic b_n."""
    return 1.9992 * n - 0.3271


def sersic(x, y, R_e, n, e1, e2, xc, yc, I_e):
    """I_e exp(-b_n [(R/R_e)^(1/n) - 1]), R = sqrt(q x'^2 + y'^2/q) >= R_MIN."""
    q, phi = ellipticity_to_q_phi(e1, e2)
    xp, yp = to_frame(x, y, xc, yc, phi)
    R2 = q * xp * xp + yp * yp / q
    R = torch.sqrt(torch.clamp(R2, min=R_MIN * R_MIN))
    return I_e * torch.exp(-sersic_bn(n) * (torch.pow(R / R_e, 1.0 / n) - 1.0))


# ---------------------------------------------------------------------------
# Steps 7-10: sub-pixel image, downsample, PSF, likelihood
# ---------------------------------------------------------------------------
def ellipticity_valid(theta: torch.Tensor, spec) -> bool:
    """False if any component has |e| >= 1 (q <= 0: no valid profile), or a
    shapelet source has a scale beta <= 0 (no valid basis)."""
    p = unpack(theta.detach(), spec)
    es = [(p["m_e1"], p["m_e2"])] + [(c[2], c[3]) for c in p["lights"] + p["sources"]]
    ok = all(float(a * a + b * b) < 1.0 for a, b in es)
    if p["shapelet"] is not None:
        ok = ok and float(p["shapelet"][0]) > 0.0
    return ok


def subpixel_image(theta: torch.Tensor, spec, n_terms: Optional[int] = None) -> torch.Tensor:
    """Surface brightness on the supersampled grid, [ny*s, nx*s]."""
    X, Y = subpixel_grid(spec.nx, spec.ny, spec.pix_scale, spec.supersample)
    p = unpack(theta, spec)
    if spec.mass_model == "EPL":
        ax, ay = epl_deflection(X, Y, p["theta_E"], p["gamma"], p["m_e1"], p["m_e2"],
                                p["m_x"], p["m_y"], n_terms=n_terms)
    else:
        ax, ay = sie_deflection(X, Y, p["theta_E"], p["m_e1"], p["m_e2"], p["m_x"], p["m_y"])
    sx, sy = shear_deflection(X, Y, p["g1"], p["g2"])
    bx, by = X - ax - sx, Y - ay - sy
    v = torch.zeros_like(X)
    for c in p["lights"]:
        v = v + sersic(X, Y, *c)
    for c in p["sources"]:
        v = v + sersic(bx, by, *c)
    if p["shapelet"] is not None:
        beta, xc, yc, coeffs = p["shapelet"]
        v = v + shapelet_source(bx, by, xc, yc, beta, coeffs)
    return v


def downsample(v: torch.Tensor, s: int) -> torch.Tensor:
    """Mean over each s x s block: [ny*s, nx*s] -> [ny, nx]."""
    ny, nx = v.shape[0] // s, v.shape[1] // s
    return v.reshape(ny, s, nx, s).mean(dim=(1, 3))


def convolve_psf(img: torch.Tensor, psf) -> torch.Tensor:
    """m[i, j] = sum_{u,v} P[u, v] img[i - u + h, j - v + h], zero outside, h = (K-1)/2."""
    P = _t(psf)
    K = P.shape[0]
    h = (K - 1) // 2
    ny, nx = img.shape
    pad = torch.zeros((ny + 2 * h, nx + 2 * h), dtype=img.dtype)
    pad[h:h + ny, h:h + nx] = img
    out = torch.zeros_like(img)
    for u in range(K):
        for v in range(K):
            r0, c0 = 2 * h - u, 2 * h - v
            out = out + P[u, v] * pad[r0:r0 + ny, c0:c0 + nx]
    return out


def model_image(theta, spec, psf, n_terms: Optional[int] = None) -> torch.Tensor:
    """PSF-convolved, downsampled model image [ny, nx] (float64)."""
    th = _t(theta)
    return convolve_psf(downsample(subpixel_image(th, spec, n_terms), spec.supersample), psf)


def chi2(model: torch.Tensor, data, invvar) -> torch.Tensor:
    d, w = _t(data), _t(invvar)
    return (w * (d - model) ** 2).sum()


def loglike(theta, spec, psf, data, invvar) -> float:
    th = _t(theta)
    if not ellipticity_valid(th, spec):
        return -math.inf
    with torch.no_grad():
        return float(-0.5 * chi2(model_image(th, spec, psf), data, invvar))


def loglike_and_grad(theta, spec, psf, data, invvar, n_terms: Optional[int] = None):
    """(logL, dlogL/dtheta[d]) by autograd through the plain definition."""
    th = _t(theta).clone().requires_grad_(True)
    if not ellipticity_valid(th, spec):
        return -math.inf, np.zeros(th.shape[0])
    L = -0.5 * chi2(model_image(th, spec, psf, n_terms), data, invvar)
    (g,) = torch.autograd.grad(L, th)
    return float(L.detach()), g.numpy()


def gradient_scale(theta, spec, psf, data, invvar) -> np.ndarray:
    """S_j = sum_pix |r_pix * dm_pix/dtheta_j| with r = w (d - m).

    The L1 size of the terms whose sum is the gradient component j; the
    parity tolerance of a gradient component is relative to |g_j| + S_j.
    The Jacobian dm/dtheta is taken in forward mode (one tangent per
    parameter).
    """
    th = _t(theta)
    with torch.no_grad():
        m = model_image(th, spec, psf)
    r = (_t(invvar) * (_t(data) - m)).reshape(-1, 1)
    J = torch.autograd.functional.jacobian(lambda z: model_image(z, spec, psf).reshape(-1), th,
                                           strategy="forward-mode", vectorize=True)
    return (r.abs() * J.abs()).sum(0).numpy()


# ---------------------------------------------------------------------------
# Batched helpers (one particle at a time: slow by design)
# ---------------------------------------------------------------------------
def batch_model_images(thetas, spec, psf) -> np.ndarray:
    return np.stack([model_image(th, spec, psf).numpy() for th in np.asarray(thetas)])


def batch_loglike(thetas, spec, psf, data, invvar) -> np.ndarray:
    return np.array([loglike(th, spec, psf, data, invvar) for th in np.asarray(thetas)])


def batch_loglike_grad(thetas, spec, psf, data, invvar):
    L, G = [], []
    for th in np.asarray(thetas):
        l, g = loglike_and_grad(th, spec, psf, data, invvar)
        L.append(l); G.append(g)
    return np.array(L), np.stack(G)


# ---------------------------------------------------------------------------
# Prior and bijection to the unconstrained space (Sec. 3.1: tilde quantities;
# Sec. 4.2 eq. sim-dist: uniform, normal, log-normal, truncated normal)
# ---------------------------------------------------------------------------
def _log_ndtr(z):
    return torch.special.log_ndtr(z)


def to_constrained(u: torch.Tensor, table) -> Tuple[torch.Tensor, torch.Tensor]:
    """theta = T(u) per parameter, and log|dtheta/du| summed over parameters.

    uniform / truncnormal on [lo, hi]: theta = lo + (hi - lo) sigmoid(u)
    normal: theta = u;  lognormal: theta = exp(u)
    """
    tab = _t(table)
    out = []
    logj = torch.zeros((), dtype=DT)
    for k in range(tab.shape[0]):
        kind = int(tab[k, 0])
        uk = u[k]
        if kind in (PRIOR_UNIFORM, PRIOR_TRUNCNORMAL):
            lo, hi = (tab[k, 1], tab[k, 2]) if kind == PRIOR_UNIFORM else (tab[k, 3], tab[k, 4])
            sgm = torch.sigmoid(uk)
            out.append(lo + (hi - lo) * sgm)
            logj = logj + torch.log(hi - lo) + torch.nn.functional.logsigmoid(uk) + torch.nn.functional.logsigmoid(-uk)
        elif kind == PRIOR_NORMAL:
            out.append(uk)
        elif kind == PRIOR_LOGNORMAL:
            out.append(torch.exp(uk))
            logj = logj + uk
        else:
            raise ValueError(kind)
    return torch.stack(out), logj


def to_unconstrained(theta: torch.Tensor, table) -> torch.Tensor:
    tab = _t(table)
    out = []
    for k in range(tab.shape[0]):
        kind = int(tab[k, 0])
        x = theta[k]
        if kind in (PRIOR_UNIFORM, PRIOR_TRUNCNORMAL):
            lo, hi = (tab[k, 1], tab[k, 2]) if kind == PRIOR_UNIFORM else (tab[k, 3], tab[k, 4])
            p = (x - lo) / (hi - lo)
            out.append(torch.log(p) - torch.log1p(-p))
        elif kind == PRIOR_NORMAL:
            out.append(x)
        elif kind == PRIOR_LOGNORMAL:
            out.append(torch.log(x))
        else:
            raise ValueError(kind)
    return torch.stack(out)


def log_prior(theta: torch.Tensor, table) -> torch.Tensor:
    """Sum of the per-parameter log densities on the constrained values."""
    tab = _t(table)
    lp = torch.zeros((), dtype=DT)
    half_log_2pi = 0.5 * math.log(2.0 * math.pi)
    for k in range(tab.shape[0]):
        kind = int(tab[k, 0])
        x = theta[k]
        a, b = tab[k, 1], tab[k, 2]
        if kind == PRIOR_UNIFORM:
            lp = lp - torch.log(b - a)
        elif kind == PRIOR_NORMAL:
            lp = lp - 0.5 * ((x - a) / b) ** 2 - torch.log(b) - half_log_2pi
        elif kind == PRIOR_LOGNORMAL:
            lx = torch.log(x)
            lp = lp - 0.5 * ((lx - a) / b) ** 2 - torch.log(b) - half_log_2pi - lx
        elif kind == PRIOR_TRUNCNORMAL:
            lo, hi = tab[k, 3], tab[k, 4]
            z = torch.special.ndtr((hi - a) / b) - torch.special.ndtr((lo - a) / b)
            lp = lp - 0.5 * ((x - a) / b) ** 2 - torch.log(b) - half_log_2pi - torch.log(z)
        else:
            raise ValueError(kind)
    return lp


def log_posterior_unconstrained(u, spec, psf, data, invvar, table, with_jacobian: bool,
                                theta_float32: bool = False):
    """logL(T(u)) + log prior(T(u)) [+ log|J|] and its gradient w.r.t. u.

    The HMC target includes the Jacobian of the bijection; the MAP objective
    (multi-start gradient descent) does not, so its optimum is the MAP of
    the constrained parameters.  With ``theta_float32`` the likelihood is
    evaluated at T(u) rounded to float32 (the parameter vector a float32
    likelihood interface receives); the prior, the Jacobian and the chain
    rule dT/du stay at the float64 T(u).
    """
    uu = _t(u).clone().requires_grad_(True)
    th, logj = to_constrained(uu, table)
    if not ellipticity_valid(th, spec):
        return -math.inf, np.zeros(uu.shape[0])
    lp = log_prior(th, table)
    if theta_float32:
        th_f = th.detach().to(torch.float32).to(DT)
        L, gL = loglike_and_grad(th_f, spec, psf, data, invvar)
        dth = torch.autograd.grad(th.sum(), uu, retain_graph=True)[0]   # elementwise map
        rest = lp + (logj if with_jacobian else 0.0)
        gr = None
        if rest.requires_grad:
            (gr,) = torch.autograd.grad(rest, uu, allow_unused=True)
        gr = torch.zeros_like(uu) if gr is None else gr
        return float(L) + float(rest.detach()), (torch.tensor(gL) * dth.detach() + gr).numpy()
    L = -0.5 * chi2(model_image(th, spec, psf), data, invvar) + lp
    if with_jacobian:
        L = L + logj
    (g,) = torch.autograd.grad(L, uu)
    return float(L.detach()), g.numpy()


# ---------------------------------------------------------------------------
# Optimiser and sampler (Sec. 3: multi-start MAP with Adam; HMC)
# ---------------------------------------------------------------------------
def adam_step(x, g, m, v, k: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) minimising a loss with gradient g.

    k is the 1-based step number used in the bias corrections.
    """
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return x - lr * mh / (np.sqrt(vh) + eps), m, v


def leapfrog(u, p, grad_fn, eps: float, L: int, inv_mass):
    """L leapfrog steps of Hamiltonian dynamics with diagonal mass matrix.

    grad_fn(u) returns the gradient of log p(u).  Half kick, drift, half
    kick per step (Neal 2011).
    """
    u = np.array(u, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    g = grad_fn(u)
    for _ in range(L):
        p = p + 0.5 * eps * g
        u = u + eps * inv_mass * p
        g = grad_fn(u)
        p = p + 0.5 * eps * g
    return u, p


def hamiltonian(logp: float, p, inv_mass) -> float:
    p = np.asarray(p, dtype=np.float64)
    return -logp + 0.5 * float(np.sum(p * p * inv_mass))


# ---------------------------------------------------------------------------
# Counter-based RNG: Philox (Salmon et al. 2011, "Parallel random numbers:
# as easy as 1, 2, 3").  Each round multiplies words 0 and 2 by the round
# multipliers, swaps the halves of the products into the four output words
# xor-ed with the odd words and the key, and the key is bumped by the Weyl
# constants between rounds.
# ---------------------------------------------------------------------------
_PHILOX_CONST = {
    32: (0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85),
    64: (0xD2E7470EE14C6C93, 0xCA5A826395121157, 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B),
}


def philox4(counter: Sequence[int], key: Sequence[int], width: int = 32, rounds: int = 10) -> List[int]:
    """One Philox4xW block: 4 counter words, 2 key words -> 4 output words."""
    m0, m1, w0, w1 = _PHILOX_CONST[width]
    mask = (1 << width) - 1
    c0, c1, c2, c3 = (int(w) & mask for w in counter)
    k0, k1 = (int(w) & mask for w in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & mask, lo1, (hi0 ^ c3 ^ k1) & mask, lo0
    return [c0, c1, c2, c3]


def philox4x32(counter: Sequence[int], key: Sequence[int], rounds: int = 10) -> List[int]:
    return philox4(counter, key, 32, rounds)


def uniform_from_bits(w: int) -> float:
    """((w >> 8) + 1/2) * 2^-24: a uniform in (0, 1), exact in float32."""
    return ((w >> 8) + 0.5) * (2.0 ** -24)


def box_muller(a: float, b: float) -> Tuple[float, float]:
    """Two standard normals from two uniforms (Box & Muller 1958)."""
    r = math.sqrt(-2.0 * math.log(a))
    return r * math.cos(2.0 * math.pi * b), r * math.sin(2.0 * math.pi * b)


def philox_normals(d: int, seed: int, w0: int, w1: int, tag: int) -> np.ndarray:
    """d standard normals from Philox4x32-10 with key (seed low word, seed
    high word) and counters (w0, w1, block, tag); each block's four words give
    two Box-Muller pairs."""
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    z = []
    for blk in range((d + 3) // 4):
        w = philox4x32([w0, w1, blk, tag], key)
        z += list(box_muller(uniform_from_bits(w[0]), uniform_from_bits(w[1])))
        z += list(box_muller(uniform_from_bits(w[2]), uniform_from_bits(w[3])))
    return np.array(z[:d])


def hmc_momenta(d: int, seed: int, chain: int, t: int) -> np.ndarray:
    """Standard normals for one chain and transition: counters (chain, t, block, 0)."""
    return philox_normals(d, seed, chain, t, 0)


def hmc_accept_uniform(d: int, seed: int, chain: int, t: int) -> float:
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return uniform_from_bits(philox4x32([chain, t, (d + 3) // 4, 0], key)[0])


def hmc_transition(u, logp_grad_fn, inv_mass, eps: float, L: int, seed: int, chain: int, t: int):
    """One HMC transition (Neal 2011) with Philox momenta and Metropolis accept.

    logp_grad_fn(u) -> (logp, dlogp/du).  Momenta p = z / sqrt(inv_mass);
    H = -logp + p^T M^-1 p / 2; accept iff log(uniform) < H0 - H1.
    Returns (u_next, logp_next, accepted, H0, H1, log_uniform).
    """
    u = np.asarray(u, dtype=np.float64)
    inv_mass = np.asarray(inv_mass, dtype=np.float64)
    d = u.shape[0]
    # a coordinate with zero inverse mass is frozen: no momentum, no motion
    z = hmc_momenta(d, seed, chain, t)
    p = np.where(inv_mass > 0, z / np.sqrt(np.where(inv_mass > 0, inv_mass, 1.0)), 0.0)
    lp0, _ = logp_grad_fn(u)
    H0 = hamiltonian(lp0, p, inv_mass)
    u1, p1 = leapfrog(u, p, lambda z: logp_grad_fn(z)[1], eps, L, inv_mass)
    lp1, _ = logp_grad_fn(u1)
    H1 = hamiltonian(lp1, p1, inv_mass) if np.isfinite(lp1) else math.inf
    lu = math.log(hmc_accept_uniform(d, seed, chain, t))
    acc = bool(np.isfinite(H1) and lu < H0 - H1)
    return (u1 if acc else u), (lp1 if acc else lp0), acc, H0, H1, lu


# ---------------------------------------------------------------------------
# Stochastic variational inference (Sec. 3: the SVI stage, eq. vi, eq. elbo,
# eq. elbo-grad; Sec. 3.2: AdaBelief for SVI)
#
# Surrogate: q(u) = N(u; mu, L L^T) in the unconstrained space, L lower
# triangular with a positive diagonal.  Parameter vector phi, length
# d + d(d+1)/2: mu, then the lower triangle of L row by row; each diagonal
# entry is stored as rho with L_ii = softplus(rho) + SVI_DIAG_SHIFT.
# Samples u_i = mu + L eps_i, eps_i standard normal.  The target is the
# log posterior in the unconstrained space with the bijection's Jacobian
# (the density of u).
# ---------------------------------------------------------------------------
SVI_DIAG_SHIFT = 1e-10
SVI_RNG_TAG = 1          # counter word 3 of the surrogate draws (HMC's is 0)


def svi_n_params(d: int) -> int:
    return d + d * (d + 1) // 2


def svi_unpack(phi: torch.Tensor, d: int) -> Tuple[torch.Tensor, torch.Tensor]:
    """phi -> (mu [d], L [d, d]) as float64 tensors (differentiable)."""
    mu = phi[:d]
    rows, cols = torch.tril_indices(d, d)
    vals = phi[d:]
    diag = rows == cols
    vals = torch.where(diag, torch.nn.functional.softplus(vals) + SVI_DIAG_SHIFT, vals)
    L = torch.zeros(d, d, dtype=phi.dtype).index_put((rows, cols), vals)
    return mu, L


def svi_pack(mu, L) -> np.ndarray:
    """(mu, L) -> phi: the inverse of svi_unpack (diagonal through the inverse softplus)."""
    mu = np.asarray(mu, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    d = mu.shape[0]
    r, c = np.tril_indices(d)
    vals = L[r, c].copy()
    dg = r == c
    x = vals[dg] - SVI_DIAG_SHIFT
    vals[dg] = x + np.log(-np.expm1(-x))       # softplus^-1(x) = log(e^x - 1)
    return np.concatenate([mu, vals])


def svi_normals(d: int, seed: int, sample: int, step: int) -> np.ndarray:
    """The standard normals of surrogate sample `sample` at SVI step `step`
    (0-based): Philox counters (sample, step, block, SVI_RNG_TAG)."""
    return philox_normals(d, seed, sample, step, SVI_RNG_TAG)


def svi_frozen_mask(d: int, frozen) -> np.ndarray:
    """Entries of phi held fixed when the coordinates in `frozen` are not
    parameters (backward modelling): mu_j and every entry of L in row or
    column j, for j in frozen."""
    fz = set(int(j) for j in frozen)
    r, c = np.tril_indices(d)
    tri = np.array([(a in fz) or (b in fz) for a, b in zip(r, c)], dtype=bool)
    return np.concatenate([np.array([j in fz for j in range(d)], dtype=bool), tri])


def svi_elbo_grad(phi, eps, logp_grad_fn, round_u: bool = True, frozen=()):
    """Monte-Carlo ELBO of eq. elbo over the samples u_i = mu + L eps_i, and its
    gradient with respect to phi.

    eps [n, d]; logp_grad_fn(u [n, d]) -> (logp [n], dlogp/du [n, d]).  With
    round_u the target is evaluated at u rounded to float32 (the points a
    float32 interface receives).  ELBO = mean_i [log q(u_i) - logp(u_i)] with
    log q(u_i) = -|eps_i|^2/2 - sum log L_jj - (d/2) log 2 pi.

    The gradient is the reparameterised (pathwise) estimator: the derivative
    of that sample mean with the eps_i held fixed; the target enters only
    through its gradient at u_i.  Its expectation is the gradient of eq.
    elbo-grad.  With `frozen` coordinates (not parameters of the target) the
    gradient entries of svi_frozen_mask are 0.  Returns (elbo, grad
    [len(phi)], u [n, d]).
    """
    eps = np.asarray(eps, dtype=np.float64)
    n, d = eps.shape
    ph = torch.tensor(np.asarray(phi, dtype=np.float64), requires_grad=True)
    mu, L = svi_unpack(ph, d)
    E = torch.tensor(eps)
    u = mu[None, :] + E @ L.T
    u_eval = u.detach().numpy()
    if round_u:
        u_eval = u_eval.astype(np.float32).astype(np.float64)
    lp, g = logp_grad_fn(u_eval)
    lp = np.asarray(lp, dtype=np.float64)
    g = torch.tensor(np.asarray(g, dtype=np.float64))
    logq = -0.5 * (E * E).sum(1) - torch.log(torch.diagonal(L)).sum() - 0.5 * d * math.log(2 * math.pi)
    elbo = float((logq.detach() - torch.tensor(lp)).mean())
    # d(-logp(u_i))/dphi = -dlogp/du . du/dphi, with du/dphi from autograd
    obj = logq.mean() - (g * u).sum(1).mean()
    (gr,) = torch.autograd.grad(obj, ph)
    gr = gr.numpy()
    if len(frozen):
        gr = np.where(svi_frozen_mask(d, frozen), 0.0, gr)
    return elbo, gr, u_eval


def adabelief_step(x, g, m, s, k: int, lr: float, b1=0.9, b2=0.999, eps=1e-16):
    """One AdaBelief update (Zhuang et al. 2020) minimising a loss with gradient g.

    Like Adam, but the second moment follows the squared deviation of the
    gradient from its moving average, (g - m)^2, plus eps; both moments are
    bias-corrected with the 1-based step number k.
    """
    m = b1 * m + (1 - b1) * g
    s = b2 * s + (1 - b2) * (g - m) ** 2 + eps
    mh = m / (1 - b1 ** k)
    sh = s / (1 - b2 ** k)
    return x - lr * mh / (np.sqrt(sh) + eps), m, s


SVI_ADAM, SVI_ADABELIEF = 0, 1


def svi_run(phi0, n: int, n_steps: int, seed: int, logp_grad_fn, optimizer: int = SVI_ADABELIEF,
            lr: float = 1e-4, b1: float = 0.95, b2: float = 0.99, eps: float = 1e-16, step0: int = 0,
            round_u: bool = True, frozen=()):
    """n_steps SVI iterations from phi0 with n surrogate samples per step.

    Step t (0-based, counted from step0 for the draws and the bias correction)
    draws eps with svi_normals(d, seed, i, step0 + t), evaluates the ELBO and
    its gradient, and applies one Adam or AdaBelief update (moments start at
    zero).  Returns (phi, elbo per step [n_steps], gradient per step [n_steps, len(phi)]).
    """
    phi = np.asarray(phi0, dtype=np.float64).copy()
    npar = phi.shape[0]
    d = int(round((math.sqrt(9 + 8 * npar) - 3) / 2))
    assert svi_n_params(d) == npar
    m = np.zeros(npar)
    s = np.zeros(npar)
    elbos, grads = [], []
    for t in range(n_steps):
        k = step0 + t
        E = np.stack([svi_normals(d, seed, i, k) for i in range(n)])
        elbo, g, _ = svi_elbo_grad(phi, E, logp_grad_fn, round_u, frozen)
        elbos.append(elbo)
        grads.append(g)
        if optimizer == SVI_ADABELIEF:
            phi, m, s = adabelief_step(phi, g, m, s, k + 1, lr, b1, b2, eps)
        else:
            phi, m, s = adam_step(phi, g, m, s, k + 1, lr, b1, b2, eps)
    return phi, np.array(elbos), np.array(grads)


def svi_moments(phi, d: int) -> Tuple[np.ndarray, np.ndarray]:
    """Mean and covariance L L^T of the surrogate."""
    mu, L = svi_unpack(torch.tensor(np.asarray(phi, dtype=np.float64)), d)
    return mu.numpy(), (L @ L.T).numpy()


# ---------------------------------------------------------------------------
# "Backward" modelling (Sec. 3: the lens and source intensities solved by
# linear inversion instead of being parameters).  For fixed nonlinear
# parameters the model is linear in the intensities A_k of the K light
# components: m = sum_k A_k B_k with B_k the model image of component k at
# unit intensity.  A = argmin_A sum w (d - m)^2 solves the weighted normal
# equations M A = b, M_kl = sum w B_k B_l, b_k = sum w B_k d.  The intensity
# entries of the parameter vector are ignored.
# ---------------------------------------------------------------------------
BACKWARD_PIVOT_REL = 1e-12


def intensity_slots(spec) -> List[int]:
    """Indices of the linear light amplitudes in the parameter vector: the
    Sersic intensities I_e, then the shapelet coefficients (if any)."""
    base = 8 if spec.mass_model == "EPL" else 7
    slots = [base + 7 * k + 6 for k in range(spec.n_lens_light + spec.n_source)]
    if getattr(spec, "n_shapelet", 0):
        c0 = base + 7 * (spec.n_lens_light + spec.n_source) + 3
        slots += list(range(c0, c0 + n_shapelet_coeffs(spec)))
    return slots


def component_images(theta, spec, psf) -> torch.Tensor:
    """[K, ny, nx]: the model image of each light component at unit intensity
    (the others at zero)."""
    th = _t(theta)
    slots = intensity_slots(spec)
    keep = torch.ones(th.shape[0], dtype=DT)
    keep[slots] = 0.0
    out = []
    for s in slots:
        e = torch.zeros(th.shape[0], dtype=DT)
        e[s] = 1.0
        out.append(model_image(th * keep + e, spec, psf))
    return torch.stack(out)


def solve_normal_equations(M: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Solve M A = b (M symmetric positive semi-definite) by Cholesky in index
    order.  A component whose pivot is not above BACKWARD_PIVOT_REL x the
    largest diagonal entry of M (its image is zero, or a combination of the
    earlier components' images) is left out with A_k = 0."""
    K = M.shape[0]
    tol = BACKWARD_PIVOT_REL * float(torch.max(torch.diagonal(M)).detach())
    Lc = [[None] * K for _ in range(K)]
    active: List[int] = []
    for j in range(K):
        s = M[j, j] - sum((Lc[j][i] * Lc[j][i] for i in active), torch.zeros((), dtype=M.dtype))
        if not float(s.detach()) > tol:
            continue
        Lc[j][j] = torch.sqrt(s)
        for r in range(j + 1, K):
            Lc[r][j] = (M[r, j] - sum((Lc[r][i] * Lc[j][i] for i in active), torch.zeros((), dtype=M.dtype))) / Lc[j][j]
        active.append(j)
    y = {}
    for j in active:                       # L y = b
        y[j] = (b[j] - sum((Lc[j][i] * y[i] for i in active if i < j), torch.zeros((), dtype=M.dtype))) / Lc[j][j]
    x = {}
    for j in reversed(active):             # L^T x = y
        x[j] = (y[j] - sum((Lc[r][j] * x[r] for r in active if r > j), torch.zeros((), dtype=M.dtype))) / Lc[j][j]
    return torch.stack([x[j] if j in x else torch.zeros((), dtype=M.dtype) for j in range(K)])


def loglike_backward(theta, spec, psf, data, invvar, with_grad: bool = True):
    """logL at the solved intensities, its gradient with respect to the
    parameter vector (zero in the intensity entries) and the intensities.

    Returns (logL, grad [d] or None, A [K]); (-inf, zeros, nan) when a
    component's ellipticity is invalid."""
    th = _t(theta).clone().requires_grad_(with_grad)
    K = len(intensity_slots(spec))
    if not ellipticity_valid(th, spec):
        return -math.inf, (np.zeros(th.shape[0]) if with_grad else None), np.full(K, np.nan)
    B = component_images(th, spec, psf).reshape(K, -1)
    w = _t(invvar).reshape(-1)
    dd = _t(data).reshape(-1)
    M = (B * w) @ B.T
    b = (B * w) @ dd
    A = solve_normal_equations(M, b)
    m = (A[:, None] * B).sum(0)
    L = -0.5 * (w * (dd - m) ** 2).sum()
    g = None
    if with_grad:
        (g,) = torch.autograd.grad(L, th)
        g = g.numpy()
    return float(L.detach()), g, A.detach().numpy()


# ---------------------------------------------------------------------------
# HMC adaptation during burn-in (Sec. 3.3: the mass matrix fitted to burn-in
# samples; the step size by dual averaging, Hoffman & Gelman 2014, "The
# No-U-Turn Sampler", Sec. 3.2.1, with their constants gamma, t0, kappa).
# All chains share one step size; the adaptation statistic of a transition is
# the chain mean of min(1, exp(H0 - H1)) (0 for a non-finite energy).
# ---------------------------------------------------------------------------
DA_GAMMA, DA_T0, DA_KAPPA = 0.05, 10.0, 0.75


def dual_averaging_init(eps0: float) -> Dict[str, float]:
    """State before the first update: mu = log(10 eps0), log eps = log eps0,
    log eps_bar = 0, H_bar = 0, m = 0."""
    return {"mu": math.log(10.0 * eps0), "log_eps": math.log(eps0), "log_eps_bar": 0.0, "H_bar": 0.0, "m": 0}


def dual_averaging_update(st: Dict[str, float], alpha: float, delta: float) -> Dict[str, float]:
    """One update after a transition with adaptation statistic alpha, target delta."""
    m = st["m"] + 1
    eta = 1.0 / (m + DA_T0)
    H_bar = (1.0 - eta) * st["H_bar"] + eta * (delta - alpha)
    log_eps = st["mu"] - math.sqrt(m) / DA_GAMMA * H_bar
    w = m ** (-DA_KAPPA)
    log_eps_bar = w * log_eps + (1.0 - w) * st["log_eps_bar"]
    return {"mu": st["mu"], "log_eps": log_eps, "log_eps_bar": log_eps_bar, "H_bar": H_bar, "m": m}


def accept_prob(H0: float, H1: float) -> float:
    if not (math.isfinite(H0) and math.isfinite(H1)):
        return 0.0
    return min(1.0, math.exp(H0 - H1))


def hmc_adapt(U0, logp_grad_fn, inv_mass, eps0: float, delta: float, L: int, n_transitions: int,
              window_start: int, seed: int, transition0: int = 0, eps_float32: bool = True):
    """Burn-in of C chains with a shared, dual-averaged step size.

    Transition t (0-based) uses eps_t = exp(log eps) (rounded to float32 with
    eps_float32: the step size a float32 interface receives) and the Philox
    counters of transition transition0 + t; after it the step size is
    updated.  Positions after transitions t >= window_start are collected
    and their variance per coordinate (over chains and transitions, ddof 1)
    is returned as the fitted inverse mass matrix.
    Returns (U [C, d], eps per transition [T], adapted eps = exp(log eps_bar),
    variance [d] or None, chain-mean acceptance statistic per transition [T],
    the smallest |log u - (H0 - H1)| of any accept decision).
    """
    U = np.array(U0, dtype=np.float64)
    C, d = U.shape
    st = dual_averaging_init(eps0)
    eps_trace, alphas, window = [], [], []
    margin = math.inf
    for t in range(n_transitions):
        eps = math.exp(st["log_eps"])
        if eps_float32:
            eps = float(np.float32(eps))
        eps_trace.append(eps)
        al = []
        for c in range(C):
            U[c], _, _, H0, H1, lu = hmc_transition(U[c], logp_grad_fn, inv_mass, eps, L, seed, c, transition0 + t)
            al.append(accept_prob(H0, H1))
            if math.isfinite(H1):
                margin = min(margin, abs(lu - (H0 - H1)))
        alpha = float(np.mean(al))
        alphas.append(alpha)
        st = dual_averaging_update(st, alpha, delta)
        if t >= window_start:
            window.append(U.copy())
    var = np.concatenate(window).var(axis=0, ddof=1) if len(window) * C > 1 else None
    return U, np.array(eps_trace), math.exp(st["log_eps_bar"]), var, np.array(alphas), margin


def log_posterior_backward(u, spec, psf, data, invvar, table, with_jacobian: bool,
                           theta_float32: bool = False):
    """Backward-modelling posterior in the unconstrained space: logL at the
    solved intensities (loglike_backward) of T(u), plus the log prior and,
    optionally, the log-Jacobian of the nonlinear parameters only (the
    intensities are not parameters); gradient w.r.t. u, zero in the intensity
    entries.  With theta_float32 the likelihood sees T(u) rounded to float32.
    """
    tab = np.asarray(_t(table).numpy())
    d = tab.shape[0]
    slots = intensity_slots(spec)
    keep = [j for j in range(d) if j not in slots]
    uu = _t(u).clone().requires_grad_(True)
    th, _ = to_constrained(uu, tab)
    thk, logj = to_constrained(uu[keep], tab[keep])
    if not ellipticity_valid(th.detach(), spec):
        return -math.inf, np.zeros(d)
    rest = log_prior(thk, tab[keep]) + (logj if with_jacobian else 0.0)
    th_eval = th.detach()
    if theta_float32:
        th_eval = th_eval.to(torch.float32).to(DT)
    L, gL, _ = loglike_backward(th_eval, spec, psf, data, invvar)
    (dth,) = torch.autograd.grad(th.sum(), uu, retain_graph=True)
    gr = None
    if torch.is_tensor(rest) and rest.requires_grad:
        (gr,) = torch.autograd.grad(rest, uu, allow_unused=True)
    gr = torch.zeros_like(uu) if gr is None else gr
    g = torch.tensor(gL) * dth.detach() + gr
    g[slots] = 0.0
    return float(L) + float(rest.detach()), g.numpy()


# ---------------------------------------------------------------------------
# Shapelet sources (Sec. 3 names shapelets beside Sersic profiles for the
# source light; the basis is the Cartesian one of Refregier 2003, MNRAS 338,
# 35, also used by Birrer et al. 2015).  A spec with n_shapelet = 1 carries
# one such source after its Sersic sources (unpack, subpixel_image).
#   phi_n(x; beta) = [2^n sqrt(pi) n! beta]^(-1/2) H_n(x / beta) exp(-x^2 / (2 beta^2)),
#   H_n the physicists' Hermite polynomials; the 2-D basis is
#   phi_n1(x) phi_n2(y) for n1 + n2 <= n_max, ordered by n = n1 + n2, then n2.
# ---------------------------------------------------------------------------
def hermite_phys(n: int, x: torch.Tensor) -> torch.Tensor:
    """H_n(x) by the recurrence H_{k+1} = 2x H_k - 2k H_{k-1}."""
    h0 = torch.ones_like(x)
    if n == 0:
        return h0
    h1 = 2.0 * x
    for k in range(1, n):
        h0, h1 = h1, 2.0 * x * h1 - 2.0 * k * h0
    return h1


def shapelet_1d(n: int, x: torch.Tensor, beta) -> torch.Tensor:
    norm = 1.0 / math.sqrt((2.0 ** n) * math.sqrt(math.pi) * math.factorial(n))
    u = x / beta
    return norm / torch.sqrt(torch.as_tensor(beta, dtype=DT)) * hermite_phys(n, u) * torch.exp(-0.5 * u * u)


def shapelet_indices(n_max: int) -> List[Tuple[int, int]]:
    return [(n - n2, n2) for n in range(n_max + 1) for n2 in range(n + 1)]


def shapelet_basis(x: torch.Tensor, y: torch.Tensor, beta, n_max: int) -> torch.Tensor:
    """[n_basis, *x.shape]: every 2-D basis function at (x, y)."""
    return torch.stack([shapelet_1d(a, x, beta) * shapelet_1d(b, y, beta) for a, b in shapelet_indices(n_max)])


def shapelet_source(x, y, xc, yc, beta, coeffs) -> torch.Tensor:
    """Surface brightness sum_k c_k phi_k(x - xc, y - yc; beta); the number of
    coefficients fixes n_max ((n_max + 1)(n_max + 2) / 2 of them)."""
    c = _t(coeffs)
    nb = c.shape[0]
    n_max = int(round((math.sqrt(8 * nb + 1) - 3) / 2))
    assert (n_max + 1) * (n_max + 2) // 2 == nb
    B = shapelet_basis(x - xc, y - yc, beta, n_max)
    return torch.einsum("k...,k->...", B, c)


def lensed_shapelet_image(theta, spec, psf, xc, yc, beta, coeffs) -> torch.Tensor:
    """Model image [ny, nx] of one shapelet source seen through the lens of
    the parameter vector theta (its mass and shear entries; its light
    components are not used): the source is evaluated at the lens-equation
    positions of the sub-pixel grid, then downsampled and PSF-convolved like
    the Sersic components."""
    th = _t(theta)
    X, Y = subpixel_grid(spec.nx, spec.ny, spec.pix_scale, spec.supersample)
    p = unpack(th, spec)
    if spec.mass_model == "EPL":
        ax, ay = epl_deflection(X, Y, p["theta_E"], p["gamma"], p["m_e1"], p["m_e2"], p["m_x"], p["m_y"])
    else:
        ax, ay = sie_deflection(X, Y, p["theta_E"], p["m_e1"], p["m_e2"], p["m_x"], p["m_y"])
    sx, sy = shear_deflection(X, Y, p["g1"], p["g2"])
    v = shapelet_source(X - ax - sx, Y - ay - sy, xc, yc, beta, coeffs)
    return convolve_psf(downsample(v, spec.supersample), psf)
