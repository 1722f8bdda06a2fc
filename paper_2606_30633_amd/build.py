"""Builds the HIP library liblens.so for gfx950 in-tree with hipcc.

Each source is compiled to its own object in parallel (objects under
_build/ next to this file), then the objects are linked into liblens.so.
With force=False a source is recompiled only when it, or any header it may
include, is newer than its object.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblens.so")
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: some of their forms have given wrong
    # results on this hardware without any error, and the kernels do not need them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    csrc = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")))


def headers():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h")))


def _filter(stderr: str) -> str:
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def _compile(hipcc, src, obj, verbose, extra=()):
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = _filter(r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({r.returncode}):\n{errs}")
    os.replace(obj + ".tmp", obj)
    return errs


# Host-code sanitizers for the checking build (device code is built as usual):
# AddressSanitizer and UndefinedBehaviorSanitizer on the host pass only.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ASAN_LIB = os.path.join(HERE, "liblens_asan.so")


def build_library(verbose: bool = False, force: bool = True, jobs: int = 8, sanitize: bool = False) -> str:
    """Compiles every source and links liblens.so; with sanitize, the host
    code is instrumented (objects under _build_asan/, liblens_asan.so, loaded
    with the sanitizer runtime preloaded; it is never the library the
    binding loads by default)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = OBJ_DIR + "_asan" if sanitize else OBJ_DIR
    lib_path = ASAN_LIB if sanitize else LIB
    extra = SANITIZE_FLAGS if sanitize else []
    os.makedirs(obj_dir, exist_ok=True)
    hdr_time = max((os.path.getmtime(h) for h in headers()), default=0.0)
    todo, objs = [], []
    for src in sources():
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        stale = (force or not os.path.exists(obj)
                 or os.path.getmtime(obj) < max(os.path.getmtime(src), hdr_time))
        if stale:
            todo.append((src, obj))
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(todo) or 1))) as ex:
        futs = [ex.submit(_compile, hipcc, s, o, verbose, extra) for s, o in todo]
        warnings = [f.result() for f in futs]
    if verbose:
        for w in warnings:
            if w.strip():
                print(w, file=sys.stderr)
    tmp = lib_path + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed ({r.returncode}):\n{_filter(r.stderr)}")
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build_library(verbose=True, force="--incremental" not in sys.argv))
