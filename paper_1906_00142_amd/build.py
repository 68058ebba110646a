"""Build librpfit.so in-tree with hipcc for gfx950.

Every HIP translation unit under csrc/ is compiled in parallel, then linked
into paper_1906_00142_amd/librpfit.so.  Run ``python -m paper_1906_00142_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librpfit.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("RP_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-lambda-capture", "-Wno-pass-failed",
]


def sources():
    """Every HIP unit, the largest shape units first so that the parallel
    build is not left waiting on one of them at the end."""
    import re

    def weight(name):
        m = re.match(r"rp_shape_v(\d)_d(\d)\.hip$", name)
        if m:
            return -(int(m.group(1)) * int(m.group(2)))
        m = re.match(r"rp_shape_v(\d)_n(\d)q(\d)\.hip$", name)
        return -(int(m.group(1)) * max(int(m.group(2)), int(m.group(3)))) if m else 0
    names = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in sorted(names, key=weight)]


def _fresh(src: str, obj: str) -> bool:
    """The object is newer than its unit and every header of csrc/ and include/."""
    if not os.path.exists(obj):
        return False
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".inc"))]
    inc = os.path.join(os.path.dirname(HERE), "include")
    deps += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and _fresh(src, obj):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every unit and link.  incremental: keep the objects that are
    newer than their unit and every header (a development shortcut; the
    default rebuilds everything)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), srcs))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources")
    return OUT


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
