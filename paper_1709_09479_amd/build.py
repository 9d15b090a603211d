"""Builds libdualcsc.so (HIP, gfx950) in the package directory.

    python -m paper_1709_09479_amd.build        # or build() from Python
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libdualcsc.so")
BUILD = os.path.join(PKG, "_build")
SOURCES = ["api.hip", "coding.hip", "split.hip", "learning.hip", "fftops.hip", "batched.hip", "diff.hip",
           "nuclear.hip", "dct.hip", "volume.hip", "learnspan.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused where the source writes them in one expression,
    # so a device function gives the same bits in every kernel it is inlined in
    "-ffp-contract=on", "-Wno-unused-result",
    "-I" + os.path.join(os.path.dirname(PKG), "include"),
]


def _compile(src: str, extra=(), build_dir=BUILD) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), res.stderr[-8000:]))
    return obj


def build(verbose: bool = False, extra=(), out=OUT, build_dir=BUILD) -> str:
    """Compile every source with FLAGS (+ ``extra``) and link ``out``."""
    os.makedirs(build_dir, exist_ok=True)
    sys.path.insert(0, CSRC)
    import gen_twiddles  # noqa: E402
    sys.path.pop(0)
    gen_twiddles.main(os.path.join(CSRC, "twiddles.inc"))
    workers = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, extra, build_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s" % res.stderr[-8000:])
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
