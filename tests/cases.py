"""Shared seeded test systems: inputs from the generators, data from the oracle."""
import numpy as np

from oracle import lens_oracle as O
from paper_2606_30633_amd import synth


def make_case(spec, k=0, n_particles=8, psf="asym", near_truth=0):
    """System + particles.  Data = oracle model at the truth + seeded noise."""
    if psf == "asym":
        p = synth.asymmetric_psf(spec.psf_size, synth.SEED_TEST_PSF + spec.psf_size)
    elif psf == "gauss":
        p = synth.gaussian_psf(spec.psf_size, 0.1, spec.pix_scale)
    else:
        p = synth.double_gaussian_psf(spec.psf_size, spec.pix_scale)
    sysm = synth.make_system_box(spec, k, psf=p)
    model = O.model_image(sysm.truth, spec, p).numpy()
    data = (model + sysm.noise).astype(np.float32)
    th = synth.particles_box(sysm, n_particles, k)
    if near_truth:
        rng = np.random.default_rng(99 + k)
        near = sysm.truth[None, :] * (1 + 1e-3 * rng.standard_normal((near_truth, spec.n_params)))
        th = np.vstack([th, near.astype(np.float32)])
    return sysm, p, data, th.astype(np.float32)
