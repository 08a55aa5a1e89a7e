"""Build of the HIP library ``libpars3.so`` for gfx950 (hipcc, in-tree).

Every ``csrc/*.hip`` file is compiled to an object in parallel and linked into
``paper_2407_17651_amd/libpars3.so``.  Run ``python -m paper_2407_17651_amd.build``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpars3.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Wno-deprecated-declarations",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
LIBS = ["-L/opt/rocm/lib", "-lrocsparse", "-Wl,-rpath,/opt/rocm/lib"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], check=True, stderr=subprocess.PIPE, text=True)
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        futs = {s: ex.submit(_compile, s) for s in srcs}
        objs = []
        for s, f in futs.items():
            try:
                objs.append(f.result())
            except subprocess.CalledProcessError as e:
                sys.stderr.write(e.stderr or "")
                raise RuntimeError(f"hipcc failed on {os.path.basename(s)}") from None
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs, *LIBS], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
