"""Build libpfresample.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1301_4019_amd.build          # compile every source
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
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpfresample.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["pfr_api.hip", "pfr_alt.hip", "pfr_scan.hip", "pfr_fscan.hip", "pfr_aux.hip", "pfr_filter.hip",
           "pfr_util.hip", "pfr_check.hip"]

ARCH = os.environ.get("PFR_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-fvisibility=hidden",
    # packed fp32 instructions stay disabled
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unknown-pragmas",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# The product library uses Philox4x32-10.  build_philox_variant() compiles a
# second copy with another round count, for the round-count study only.
VARIANT_ROUNDS = 7


def variant_path(rounds: int = VARIANT_ROUNDS) -> str:
    return os.path.join(HERE, f"libpfresample_philox{rounds}.so")


def _compile(src: str, build_dir: str, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def _build(out: str, build_dir: str, defines=(), verbose: bool = False) -> str:
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


def build(verbose: bool = False) -> str:
    return _build(LIB, BUILD_DIR, (), verbose)


def build_philox_variant(rounds: int = VARIANT_ROUNDS, verbose: bool = False) -> str:
    return _build(variant_path(rounds), BUILD_DIR + f"_philox{rounds}",
                  (f"-DPFR_PHILOX_ROUNDS={rounds}",), verbose)


if __name__ == "__main__":
    build(verbose=True)
    build_philox_variant(verbose=True)
    sys.exit(0)
