"""Compile the HIP library (liblbm.so) for gfx950, in-tree.

Every ``csrc/*.hip`` file is compiled to an object under ``_build/`` and
linked into ``paper_1906_05448_amd/liblbm.so``. Packed-FP32 instruction
selection is switched off for all device code.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
BUILD = PKG / "_build"
LIB = PKG / "liblbm.so"
ARCH = "gfx950"

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Geometry and particle arithmetic must round exactly like the FP64 recipe
# they implement (no fused multiply-add), so classification is reproducible.
PER_FILE_FLAGS = {"dense.hip": []}
DEFAULT_EXTRA = ["-ffp-contract=off"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: Path, obj: Path) -> None:
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-c",
           *DEVICE_FLAGS, *PER_FILE_FLAGS.get(src.name, DEFAULT_EXTRA), "-Wall", "-Wno-unused-function",
           f"-I{INCLUDE}", f"-I{CSRC}", str(src), "-o", str(obj)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src.name}\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    warn = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l
                     and "target-feature" not in l and l.strip())
    if warn:
        sys.stderr.write(warn + "\n")


def build(jobs: int = 8) -> Path:
    BUILD.mkdir(exist_ok=True)
    sources = sorted(CSRC.glob("*.hip"))
    objs = [BUILD / (s.stem + ".o") for s in sources]
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(sources))) as ex:
        list(ex.map(lambda so: _compile(*so), zip(sources, objs)))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
