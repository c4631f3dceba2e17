"""Build libhrir.so (HIP for gfx950) in-tree with hipcc.

Usage: python paper_1502_03162_amd/build.py   (runs without importing the
package, which needs the library this script produces)
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhrir.so")

SOURCES = ["render.hip", "render_quad.hip", "render_rw.hip", "dense.hip", "fftola.hip", "block.hip", "render_moving.hip", "mlp.hip",
           "factorize_device.hip", "l1_device.hip", "autotune.cpp", "server.cpp", "loadgen.cpp", "factorize.cpp", "sparsify.cpp",
           "errors.cpp"]

# Per-file extra flags.  The register-window kernel dispatches taps through a
# tree of wave-uniform scalar branches; the structurizer must leave such
# uniform regions as they are (structurizing them inserts flow blocks whose
# phis copy the accumulators after every tap).
EXTRA = {"render_rw.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=true"],
         # the device factorization keeps the host code's rounding: no fused multiply-adds
         "factorize_device.hip": ["-ffp-contract=off"],
         # likewise the device L1-NNLS solves
         "l1_device.hip": ["-ffp-contract=off"]}

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 VALU ops stay off; plain fp32 fma is what the kernels use
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]

_NOISE = "packed-fp32-ops' is not a recognized feature"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if _NOISE not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append(([hipcc(), *HIPCC_FLAGS, *EXTRA.get(src, []), *inc, "-c", "-o", obj,
                      os.path.join(CSRC, src)], obj))
    with ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o in jobs], "-lhipfft"],
         verbose)
    os.replace(tmp, LIB)
    return LIB


def assemble(src: str, out_path: str) -> str:
    """gfx950 device assembly of one HIP source, with the library's flags
    (for inspection of the generated code)."""
    cmd = [hipcc(), *HIPCC_FLAGS, *EXTRA.get(src, []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "--cuda-device-only", "-S", "-o", out_path, os.path.join(CSRC, src)]
    _run(cmd, False)
    return out_path


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
