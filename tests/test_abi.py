"""The C-ABI library loads and exports every symbol include/*.h declares.

Host-only: no call here touches the GPU.
"""
import ctypes
import glob
import os
import re

import pytest

from paper_2606_30633_amd import lens, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*([a-z_][a-z0-9_]*)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_is_built():
    assert os.path.exists(lens.LIB_PATH), "liblens.so is not built (python -m paper_2606_30633_amd.build)"


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert {"lens_forward", "lens_loglike", "lens_loglike_grad", "lens_plan_create"} <= names
    lib = ctypes.CDLL(lens.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_shapelet_parameter_counts_match_the_oracle():
    import dataclasses
    from oracle import lens_oracle as O
    for nmax in (0, 4, 8):
        for ns in (0, 1):
            spec = dataclasses.replace(synth.config1_spec(), n_source=ns, n_shapelet=1, shapelet_nmax=nmax)
            assert lens.lens_num_params(spec) == O.n_params(spec) == spec.n_params


def test_status_strings_and_param_counts():
    assert lens.lens_status_string(0) == "ok"
    assert "invalid" in lens.lens_status_string(-1)
    assert lens.lens_num_params(synth.config1_spec()) == 21
    assert lens.lens_num_params(synth.config2_spec()) == 29
    assert lens.lens_num_params(synth.paper_spec(80, 2, 11)) == 22


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(pix_scale=0.0), dict(supersample=0), dict(psf_size=4),
    dict(psf_size=33), dict(mass_model="XYZ"), dict(n_lens_light=4), dict(n_source=0),
    dict(nx=2049), dict(n_shapelet=2), dict(n_shapelet=1, shapelet_nmax=9),
    dict(n_shapelet=1, shapelet_nmax=-1), dict(n_shapelet=1, n_source=2),
])
def test_invalid_descriptors_rejected(bad):
    import dataclasses
    spec = dataclasses.replace(synth.config1_spec(), **bad)
    assert lens.lens_num_params(spec) == -1


def test_cnn_parameter_count_matches_oracle_layout():
    from oracle import cnn_oracle
    lib = lens.load_library()
    lib.lens_cnn_num_params.restype = ctypes.c_int64
    assert lib.lens_cnn_num_params() == cnn_oracle.n_params()


def test_svi_parameter_count_matches_oracle_layout():
    from oracle import lens_oracle as O
    lens.load_library()
    for d in (1, 21, 22, 29, 50):
        assert lens.lens_svi_num_params(d) == O.svi_n_params(d)
    for bad in (0, -3, 51):
        with pytest.raises(ValueError):
            lens.lens_svi_num_params(bad)


def test_new_entry_points_reject_null_and_bad_arguments_on_the_host():
    """SVI, HMC adaptation and backward modelling return LENS_EINVAL for a null
    plan or invalid sizes before any GPU call."""
    lib = lens.load_library()
    EINVAL = -1
    P = None
    assert lib.lens_svi_reset(P) == EINVAL
    assert lib.lens_svi_elbo_grad(P, 4, P, 0, 0, P, P, P, P) == EINVAL
    assert lib.lens_svi_run(P, 4, P, P, P, 1, 1, 1e-4, 0.95, 0.99, 1e-16, 0, P, 0, P) == EINVAL
    assert lib.lens_svi_moments(0, P, P, P, P, P) == EINVAL
    assert lib.lens_svi_moments(29, P, P, P, P, P) == EINVAL
    assert lib.lens_hmc_adapt(P, 4, P, P, P, P, 0.1, 0.8, 3, 10, 0, 0, 0, P, P, P, 0, P) == EINVAL
    assert lib.lens_loglike_grad_backward(P, 4, P, P, P, P, P) == EINVAL
    assert lib.lens_plan_set_backward(P, 1) == EINVAL


def test_build_flags_target_gfx950_without_packed_fp32():
    """Every HIP source is compiled for gfx950 with the packed-FP32 target
    feature switched off (the code relies on scalar FP32 FMA only)."""
    from paper_2606_30633_amd import build as B
    flags = " ".join(B.HIPCC_FLAGS)
    assert "--offload-arch=gfx950" in flags
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
    srcs = B.sources()
    assert any(s.endswith("lens_kernels.hip") for s in srcs) and any(s.endswith("lens_backward.hip") for s in srcs)
