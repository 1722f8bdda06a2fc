"""Host-side parts of the benchmark contract: more than one GPU is refused
with a message (the library runs on one GPU), and the flop models behind the
roofline figures are the sums their docstrings state."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_flop_models():
    # render: 4 K_s (series) + 40 + 60 (EPL) + 12 (shear, lens equation) + 18 per Sersic + 1 (downsampling)
    assert bench.render_flops_per_subpixel(20, 1, 2, True) == 80 + 100 + 12 + 54 + 1
    assert bench.render_flops_per_subpixel(20, 1, 1, False) == 80 + 40 + 12 + 36 + 1
    # adjoint: forward and reverse series, mass forward and reverse, shear, 48 per Sersic
    a = bench.adjoint_flops_per_subpixel(20, 12, 1, 2, True)
    assert a == 80 + 4 * 12 * 2 + 100 + 12 + 70 + 3 * 48
