"""Seeded synthetic inputs for the batched strong-lens likelihood.

This module only *draws* inputs: model layouts, parameter vectors from the
stated distributions, PSF kernels, Gaussian noise and inverse-variance maps.
It holds none of the lensing forward model's arithmetic; the observed image
of a system is made by the caller (forward model at the truth + the noise
drawn here), so both the GPU path and the CPU checker can consume the same
arrays.

Workload shapes follow the paper's simulated systems (Sec. 4.2, eq. sim-dist:
EPL + external shear mass, Sersic lens light, Sersic source, supersampling,
Table 100sysparams): the parity system (60x60, SIE), the 100x100 EPL system
with two sources, and the uneven batch of 100 systems.  Every generator takes an explicit seed and uses
``numpy.random.default_rng``; values are produced in float64 and rounded to
float32 once, so every consumer sees identical bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np
from scipy import special as _sp

# --------------------------------------------------------------------------
# Model layout
# --------------------------------------------------------------------------
MASS_SIE = "SIE"
MASS_EPL = "EPL"

SERSIC_NAMES = ("R_e", "n", "e1", "e2", "x", "y", "I_e")


@dataclass(frozen=True)
class ModelSpec:
    """Image geometry and model composition of one lens system.

    Canonical parameter order (Sec. 3 lists the parameters): mass block
    (theta_E, [gamma,] e1, e2, x, y), external shear (g1, g2), then the
    Sersic lens-light components, then the Sersic source components, each
    (R_e, n, e1, e2, x, y, I_e), then an optional shapelet source
    (beta, x, y, c_0 .. c_{nb-1}; Sec. 3: Sersic profiles and/or shapelets
    for the source light).
    """

    nx: int
    ny: int
    pix_scale: float
    supersample: int
    psf_size: int
    mass_model: str = MASS_EPL
    n_lens_light: int = 1
    n_source: int = 1
    n_shapelet: int = 0          # 0 or 1 shapelet source (after the Sersic sources)
    shapelet_nmax: int = 0       # its order: (n_max + 1)(n_max + 2)/2 coefficients

    def __post_init__(self):
        # the pixel scale is a float32 input of the GPU path: keep it float32-exact
        object.__setattr__(self, "pix_scale", float(np.float32(self.pix_scale)))

    @property
    def n_mass(self) -> int:
        return 8 if self.mass_model == MASS_EPL else 7

    @property
    def n_shapelet_coeffs(self) -> int:
        return (self.shapelet_nmax + 1) * (self.shapelet_nmax + 2) // 2 if self.n_shapelet else 0

    @property
    def n_params(self) -> int:
        return self.n_mass + 7 * (self.n_lens_light + self.n_source) + (
            3 + self.n_shapelet_coeffs if self.n_shapelet else 0)

    def param_names(self) -> List[str]:
        names = ["theta_E"]
        if self.mass_model == MASS_EPL:
            names.append("gamma")
        names += ["m_e1", "m_e2", "m_x", "m_y", "g1", "g2"]
        for k in range(self.n_lens_light):
            names += [f"l{k}_{s}" for s in SERSIC_NAMES]
        for k in range(self.n_source):
            names += [f"s{k}_{s}" for s in SERSIC_NAMES]
        if self.n_shapelet:
            names += ["sh_beta", "sh_x", "sh_y"] + [f"sh_c{k}" for k in range(self.n_shapelet_coeffs)]
        return names


# --------------------------------------------------------------------------
# Priors / parameter distributions (kind, a, b, c, d)
#   uniform(a, b) | normal(mu, sigma) | lognormal(mu, sigma): log x ~ N(mu, sigma)
#   truncnormal(mu, sigma, lo, hi)
# --------------------------------------------------------------------------
PRIOR_UNIFORM = 0
PRIOR_NORMAL = 1
PRIOR_LOGNORMAL = 2
PRIOR_TRUNCNORMAL = 3


@dataclass(frozen=True)
class Dist:
    kind: int
    a: float
    b: float
    c: float = 0.0
    d: float = 0.0

    def row(self) -> Tuple[float, float, float, float, float]:
        return (float(self.kind), self.a, self.b, self.c, self.d)


def U(a, b):
    return Dist(PRIOR_UNIFORM, a, b)


def N(mu, sigma):
    return Dist(PRIOR_NORMAL, mu, sigma)


def LN(mu, sigma):
    return Dist(PRIOR_LOGNORMAL, mu, sigma)


def TN(mu, sigma, lo, hi):
    return Dist(PRIOR_TRUNCNORMAL, mu, sigma, lo, hi)


def draw(dist: Dist, rng: np.random.Generator, size) -> np.ndarray:
    """Draw from one distribution (float64)."""
    if dist.kind == PRIOR_UNIFORM:
        return rng.uniform(dist.a, dist.b, size)
    if dist.kind == PRIOR_NORMAL:
        return rng.normal(dist.a, dist.b, size)
    if dist.kind == PRIOR_LOGNORMAL:
        return np.exp(rng.normal(dist.a, dist.b, size))
    if dist.kind == PRIOR_TRUNCNORMAL:
        lo = _sp.ndtr((dist.c - dist.a) / dist.b)
        hi = _sp.ndtr((dist.d - dist.a) / dist.b)
        u = rng.uniform(lo, hi, size)
        return dist.a + dist.b * _sp.ndtri(u)
    raise ValueError(dist.kind)


def prior_table(dists: Sequence[Dist]) -> np.ndarray:
    """[d, 5] float32 table (kind, a, b, c, d) consumed by both sides."""
    return np.asarray([d.row() for d in dists], dtype=np.float32)


def uniform_box_dists(spec: ModelSpec, src_center=0.3) -> List[Dist]:
    """Uniform ranges of the small parity / headline workloads."""
    d = [U(0.8, 1.8)]
    if spec.mass_model == MASS_EPL:
        d.append(U(1.5, 2.5))
    d += [U(-0.3, 0.3), U(-0.3, 0.3), U(-0.1, 0.1), U(-0.1, 0.1),
          U(-0.1, 0.1), U(-0.1, 0.1)]
    sers_l = [U(0.05, 1.0), U(0.5, 5.0), U(-0.3, 0.3), U(-0.3, 0.3),
              U(-0.1, 0.1), U(-0.1, 0.1), U(0.1, 1.0)]
    sers_s = [U(0.05, 1.0), U(0.5, 5.0), U(-0.3, 0.3), U(-0.3, 0.3),
              U(-src_center, src_center), U(-src_center, src_center), U(0.1, 1.0)]
    for _ in range(spec.n_lens_light):
        d += sers_l
    for _ in range(spec.n_source):
        d += sers_s
    return d


# The paper's 22-parameter simulation distribution and modeling prior
# (eq. sim-dist).  Intensities are divided by 1000 so that sigma = 0.01
# noise gives lens-like S/N at surface-brightness pixel units.
_I_SCALE = 1e-3


def paper_sim_dists() -> List[Dist]:
    return [
        LN(math.log(1.25), 0.25), TN(2.0, 0.25, 1.0, 3.0),
        N(0.0, 0.1), N(0.0, 0.1), N(0.0, 0.03), N(0.0, 0.03),
        N(0.0, 0.05), N(0.0, 0.05),
        LN(math.log(1.6), 0.15), U(2.0, 6.0),
        TN(0.0, 0.05, -0.15, 0.15), TN(0.0, 0.05, -0.15, 0.15),
        N(0.0, 0.01), N(0.0, 0.01), LN(math.log(300 * _I_SCALE), 0.3),
        LN(math.log(0.25), 0.15), U(0.5, 4.0),
        TN(0.0, 0.15, -0.5, 0.5), TN(0.0, 0.15, -0.5, 0.5),
        N(0.0, 0.25), N(0.0, 0.25), LN(math.log(150 * _I_SCALE), 0.5),
    ]


def paper_prior_dists() -> List[Dist]:
    return [
        LN(math.log(1.25), 0.4), TN(2.0, 0.5, 1.0, 3.0),
        N(0.0, 0.2), N(0.0, 0.2), N(0.0, 0.06), N(0.0, 0.06),
        N(0.0, 0.1), N(0.0, 0.1),
        LN(math.log(1.6), 0.25), U(0.5, 8.0),
        TN(0.0, 0.1, -0.15, 0.15), TN(0.0, 0.1, -0.15, 0.15),
        N(0.0, 0.02), N(0.0, 0.02), LN(math.log(300 * _I_SCALE), 0.5),
        LN(math.log(0.25), 0.25), U(0.5, 8.0),
        TN(0.0, 0.3, -0.5, 0.5), TN(0.0, 0.3, -0.5, 0.5),
        N(0.0, 0.5), N(0.0, 0.5), LN(math.log(150 * _I_SCALE), 0.9),
    ]


def draw_params(dists: Sequence[Dist], n: int, seed: int) -> np.ndarray:
    """[n, d] float32 parameter vectors, one column per distribution."""
    rng = np.random.default_rng(seed)
    cols = [draw(dd, rng, n) for dd in dists]
    return np.stack(cols, axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# PSF kernels and noise
# --------------------------------------------------------------------------
FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def gaussian_psf(k: int, fwhm_arcsec: float, pix_scale: float) -> np.ndarray:
    """Odd k x k pixel-centre-sampled circular Gaussian, normalised to sum 1."""
    assert k % 2 == 1
    sig = fwhm_arcsec * FWHM_TO_SIGMA / pix_scale
    h = (k - 1) // 2
    u = np.arange(k, dtype=np.float64) - h
    g = np.exp(-0.5 * (u[:, None] ** 2 + u[None, :] ** 2) / sig ** 2)
    return (g / g.sum()).astype(np.float32)


def double_gaussian_psf(k: int, pix_scale: float) -> np.ndarray:
    """0.8 G(FWHM 0.1") + 0.2 G(FWHM 0.3"), normalised to sum 1."""
    a = gaussian_psf(k, 0.1, pix_scale).astype(np.float64)
    b = gaussian_psf(k, 0.3, pix_scale).astype(np.float64)
    p = 0.8 * a + 0.2 * b
    return (p / p.sum()).astype(np.float32)


def asymmetric_psf(k: int, seed: int) -> np.ndarray:
    """Positive PSF with no symmetry (catches flipped / transposed kernels)."""
    rng = np.random.default_rng(seed)
    base = double_gaussian_psf(k, 0.05).astype(np.float64)
    p = base * (1.0 + 0.5 * rng.uniform(0.0, 1.0, (k, k)))
    p[0, :] += 0.02 * rng.uniform(0.0, 1.0, k)
    p[:, -1] += 0.01 * rng.uniform(0.0, 1.0, k)
    return (p / p.sum()).astype(np.float32)


def noise(shape, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal(shape)).astype(np.float32)


def invvar_map(ny: int, nx: int, sigma: float) -> np.ndarray:
    return np.full((ny, nx), 1.0 / (sigma * sigma), dtype=np.float32)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
SEED_TRUTH = 20260001
SEED_NOISE = 20261001
SEED_PARTICLES = 20262001
SEED_TEST_PSF = 20263001
SEED_CNN_TRAIN = 20264000
SEED_CNN_VAL = 20265000
SEED_HMC = 20266000

SIGMA_NOISE = 0.01


@dataclass
class System:
    """One synthetic lens system: geometry, PSF, truth, noise, weights."""

    spec: ModelSpec
    psf: np.ndarray          # [K, K] float32
    truth: np.ndarray        # [d] float32
    noise: np.ndarray        # [ny, nx] float32 (added to the model at truth)
    invvar: np.ndarray       # [ny, nx] float32
    prior: List[Dist] = field(default_factory=list)


def config1_spec() -> ModelSpec:
    return ModelSpec(60, 60, 0.05, 2, 11, MASS_SIE, 1, 1)


def config2_spec() -> ModelSpec:
    return ModelSpec(100, 100, 0.05, 3, 21, MASS_EPL, 1, 2)


def make_system_box(spec: ModelSpec, k: int = 0, psf: np.ndarray | None = None) -> System:
    """Single system with uniform-box truth (parity / headline workloads)."""
    dists = uniform_box_dists(spec)
    truth = draw_params(dists, 1, SEED_TRUTH + k)[0]
    if psf is None:
        if spec.psf_size == 11 and spec.supersample == 2:
            psf = gaussian_psf(spec.psf_size, 0.1, spec.pix_scale)
        else:
            psf = double_gaussian_psf(spec.psf_size, spec.pix_scale)
    return System(spec, psf, truth,
                  noise((spec.ny, spec.nx), SIGMA_NOISE, SEED_NOISE + k),
                  invvar_map(spec.ny, spec.nx, SIGMA_NOISE), dists)


def config1_system() -> System:
    return make_system_box(config1_spec(), 0)


def config2_system() -> System:
    return make_system_box(config2_spec(), 0)


def particles_box(sys_: System, n: int, k: int = 0) -> np.ndarray:
    return draw_params(sys_.prior, n, SEED_PARTICLES + k)


def paper_spec(side: int, s: int, kpsf: int) -> ModelSpec:
    return ModelSpec(side, side, 0.05, s, kpsf, MASS_EPL, 1, 1)


def large_spec(side: int, s: int = 2, kpsf: int = 21) -> ModelSpec:
    """Large cutout (Sec. 2: O(10^6) pixels for a cluster-scale lens): the
    headline model composition on a side x side grid at 0.05"/px."""
    return ModelSpec(side, side, 0.05, s, kpsf, MASS_EPL, 1, 2)


def large_box_dists(spec: ModelSpec) -> List[Dist]:
    """The headline uniform ranges with every angle scaled by the field width
    over the headline's 5" field: the same morphology resolved by more
    pixels (theta_E 8-18" at 1000 px, a cluster-scale Einstein radius)."""
    f = spec.nx * spec.pix_scale / 5.0
    d = [U(0.8 * f, 1.8 * f), U(1.5, 2.5), U(-0.3, 0.3), U(-0.3, 0.3), U(-0.1 * f, 0.1 * f),
         U(-0.1 * f, 0.1 * f), U(-0.1, 0.1), U(-0.1, 0.1)]
    for k in range(spec.n_lens_light + spec.n_source):
        c = 0.1 * f if k < spec.n_lens_light else 0.3 * f
        d += [U(0.05 * f, 1.0 * f), U(0.5, 5.0), U(-0.3, 0.3), U(-0.3, 0.3), U(-c, c), U(-c, c), U(0.1, 1.0)]
    return d


def make_system_large(spec: ModelSpec, k: int = 0) -> System:
    dists = large_box_dists(spec)
    truth = draw_params(dists, 1, SEED_TRUTH + k)[0]
    return System(spec, double_gaussian_psf(spec.psf_size, spec.pix_scale), truth,
                  noise((spec.ny, spec.nx), SIGMA_NOISE, SEED_NOISE + k),
                  invvar_map(spec.ny, spec.nx, SIGMA_NOISE), dists)


def uneven_batch_specs(n_systems: int = 100, seed: int = SEED_TRUTH) -> List[ModelSpec]:
    """Image sides U{48..160}, supersampling U{2,3,4}, PSF sizes U{11,13,...,31}."""
    rng = np.random.default_rng(seed + 500000)
    sides = rng.integers(48, 161, n_systems)
    ss = rng.integers(2, 5, n_systems)
    ks = 11 + 2 * rng.integers(0, 11, n_systems)
    return [paper_spec(int(a), int(b), int(c)) for a, b, c in zip(sides, ss, ks)]


def make_system_paper(spec: ModelSpec, k: int) -> System:
    truth = draw_params(paper_sim_dists(), 1, SEED_TRUTH + k)[0]
    return System(spec, double_gaussian_psf(spec.psf_size, spec.pix_scale), truth,
                  noise((spec.ny, spec.nx), SIGMA_NOISE, SEED_NOISE + k),
                  invvar_map(spec.ny, spec.nx, SIGMA_NOISE), paper_prior_dists())


def particles_paper(n: int, k: int) -> np.ndarray:
    return draw_params(paper_prior_dists(), n, SEED_PARTICLES + k)
