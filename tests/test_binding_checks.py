"""The Python binding rejects wrongly shaped, placed or strided arrays before
any copy, allocation or launch.

The kernels read the PSF, data and weights (and every state array of the
samplers) through raw device pointers whose extent the C layer cannot see,
so a short or misplaced buffer must be refused on the host.  Host-only: no
call here reaches the GPU.
"""
import numpy as np
import pytest
import torch

from paper_2606_30633_amd import lens, synth


def _arrays(spec):
    K = spec.psf_size
    return (np.zeros((K, K), np.float32), np.zeros((spec.ny, spec.nx), np.float32),
            np.ones((spec.ny, spec.nx), np.float32))


@pytest.mark.parametrize("which,shape", [
    ("psf", (9, 9)), ("psf", (11, 10)), ("data", (60, 59)), ("data", (3600,)),
    ("invvar", (59, 60)), ("invvar", (60, 60, 1)),
])
def test_plan_rejects_wrong_system_array_shapes(which, shape):
    spec = synth.config1_spec()
    psf, data, invvar = _arrays(spec)
    arrs = {"psf": psf, "data": data, "invvar": invvar}
    arrs[which] = np.zeros(shape, np.float32)
    with pytest.raises(ValueError, match=which):
        lens.LensPlan(spec, arrs["psf"], arrs["data"], arrs["invvar"], 4, "cuda:0")


def test_plan_rejects_transposed_image_of_a_non_square_system():
    import dataclasses
    spec = dataclasses.replace(synth.config1_spec(), nx=40, ny=30)
    psf, data, invvar = _arrays(spec)
    with pytest.raises(ValueError, match="data"):
        lens.LensPlan(spec, psf, data.T.copy(), invvar, 4, "cuda:0")


def test_plan_rejects_a_cpu_device_and_empty_capacity():
    spec = synth.config1_spec()
    psf, data, invvar = _arrays(spec)
    with pytest.raises(ValueError, match="GPU"):
        lens.LensPlan(spec, psf, data, invvar, 4, "cpu")
    with pytest.raises(ValueError, match="max_particles"):
        lens.LensPlan(spec, psf, data, invvar, 0, "cuda:0")


def test_batch_plan_rejects_a_wrong_shape_in_any_system():
    specs = [synth.config1_spec(), synth.config2_spec()]
    arrs = [_arrays(s) for s in specs]
    psfs, datas, invvars = [a[0] for a in arrs], [a[1] for a in arrs], [a[2] for a in arrs]
    bad = list(datas)
    bad[1] = np.zeros((99, 100), np.float32)
    with pytest.raises(ValueError, match="system 1"):
        lens.BatchPlan(specs, psfs, bad, invvars, [4, 4], "cuda:0")
    with pytest.raises(ValueError):
        lens.BatchPlan(specs, psfs[:1], datas, invvars, [4, 4], "cuda:0")


def _fake_plan(d=21, maxp=8):
    """A plan object with no C plan behind it: argument checks run before the
    library is reached, so none of these calls touches it."""
    plan = lens.LensPlan.__new__(lens.LensPlan)
    plan.d = d
    plan.device = torch.device("cuda", 0)
    plan.max_particles = maxp
    plan.handle = None
    plan.spec = synth.config1_spec()
    return plan


def test_sampler_state_on_the_cpu_is_rejected():
    plan = _fake_plan()
    C, d = 4, plan.d
    u = torch.zeros((C, d))
    with pytest.raises(ValueError):
        lens.lens_hmc_run(plan, u, torch.zeros((C, d)), torch.zeros(C, dtype=torch.float64), torch.ones(d),
                          0.1, 3, 1, 0)
    with pytest.raises(ValueError):
        lens.lens_hmc_adapt(plan, u, torch.zeros((C, d)), torch.zeros(C, dtype=torch.float64), torch.ones(d),
                            0.1, 0.8, 3, 4, 0, 0)
    with pytest.raises(ValueError):
        lens.lens_map_adam(plan, u, torch.zeros((C, d)), torch.zeros((C, d)), 1, 1e-2)
    with pytest.raises(ValueError):
        lens.lens_logpost_grad(plan, u, True)


def test_non_contiguous_or_misplaced_outputs_are_rejected():
    """_check_out is the single gate for caller-supplied arrays: dtype, shape,
    device and contiguity are each enforced."""
    dev = torch.device("cuda", 0)
    ok_shape = (4, 21)
    strided = torch.zeros((21, 4)).t()            # right shape, not contiguous
    assert strided.shape == ok_shape and not strided.is_contiguous()
    for bad in (torch.zeros(ok_shape),            # CPU
                torch.zeros(ok_shape, dtype=torch.float64),
                torch.zeros((4, 20)),
                strided):
        with pytest.raises(ValueError):
            lens._check_out(bad, ok_shape, torch.float32, dev)


def test_noalloc_size_and_argument_checks_run_before_any_gpu_call():
    """lens_loglike_grad_noalloc refuses, on the host, a call larger than its
    fixed scratch (LENS_ESCRATCH) and bad arguments (LENS_EINVAL).  The
    pointers are never dereferenced on these paths, so placeholders serve."""
    import ctypes
    lib = lens.load_library()
    spec = synth.config2_spec()
    desc = lens.desc_from_spec(spec)
    fake = ctypes.c_void_p(0x1000)
    per_image = 4 * spec.nx * spec.ny
    P_big = lens.LENS_NOALLOC_SCRATCH_BYTES // per_image + 1
    args = (ctypes.byref(desc), fake, fake, fake)
    out = (fake, fake, fake, None, None)
    assert lib.lens_loglike_grad_noalloc(*args, P_big, *out) == lens.LENS_ESCRATCH
    assert lib.lens_loglike_grad_noalloc(*args, 0, *out) == lens.LENS_EINVAL
    assert lib.lens_loglike_grad_noalloc(ctypes.byref(desc), None, fake, fake, 8, *out) == lens.LENS_EINVAL
    bad = lens.desc_from_spec(spec)
    bad.psf_size = 4
    assert lib.lens_loglike_grad_noalloc(ctypes.byref(bad), fake, fake, fake, 8, *out) == lens.LENS_EINVAL
    assert "scratch" in lens.lens_status_string(lens.LENS_ESCRATCH)


def test_noalloc_binding_rejects_host_tensors():
    spec = synth.config1_spec()
    K, d = spec.psf_size, spec.n_params
    z = torch.zeros
    with pytest.raises(ValueError):
        lens.lens_loglike_grad_noalloc(spec, z((K, K)), z((spec.ny, spec.nx)), z((spec.ny, spec.nx)),
                                       z((4, d)), z(4), z((4, d)))
