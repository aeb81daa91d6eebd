"""Compile the HIP sources of the engine into in-tree shared libraries for
gfx950 with hipcc (no JIT cache, no torch extension machinery).

    python -m paper_1809_08857_amd.build        # builds libmg.so and libmgl.so
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
INCLUDE = os.path.join(ROOT, "include")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # keep hand-written float code away from packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
]

LIBS = {
    "libmg.so": ["mg_kern_f64.hip", "mg_kern_f32.hip", "mg_kern_bf16.hip", "mg_misc.hip",
                 "mg_tail.hip", "mg_engine.hip", "mg_batched.hip", "mg_autotune.hip", "mg_noalloc.hip", "mg_krylov.hip", "mg_amr.hip", "mg_eb.hip"],
    "libmgl.so": ["nn_kernels.hip", "nn_net.hip"],
}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if msgs:
        print(msgs, file=sys.stderr)
    return obj


def build(jobs: int | None = None) -> list[str]:
    """Compile every source and link every library; always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    out = []
    for lib, srcs in LIBS.items():
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(_compile, srcs))
        target = os.path.join(PKG, lib)
        tmp = target + f".tmp{os.getpid()}"
        subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       check=True)
        os.replace(tmp, target)
        out.append(target)
    return out


if __name__ == "__main__":
    for p in build():
        print(p)
