"""Builds libqnep.so (gfx950) in-tree with hipcc.

    python -m paper_2601_19034_amd.build        # compile every source, link
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqnep.so")

SOURCES = ["nbr.hip", "nep.hip", "mlp.hip", "mlp_bf16.hip", "coul.hip", "fft.hip", "pppm.hip", "finalize.hip", "backward.hip", "batch_setup.hip", "batch_eval.hip", "snes.hip", "md.hip",
           "api.cpp"]

ARCH = os.environ.get("QNEP_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
    # packed FP32 instructions are not emitted (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _newest_header() -> float:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(h) for h in hdrs)


def _compile(src: str, incremental: bool = False) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(out):
        t = os.path.getmtime(out)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _newest_header():
            return out
    cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", out]
    if src.endswith(".cpp"):
        cmd = [hipcc()] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return out


def build(jobs: int = 8, incremental: bool = False) -> str:
    """Compiles every source (or, with incremental, those older than their object
    and the headers) and links libqnep.so."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    print(build(int(args[0]) if args else 8, incremental="--incremental" in sys.argv))
