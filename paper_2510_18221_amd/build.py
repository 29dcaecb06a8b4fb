"""Compile libeco.so (HIP kernels for gfx950 + the C-ABI runtime) in-tree.

    python -m paper_2510_18221_amd.build

Objects go to paper_2510_18221_amd/_build/, the library to
paper_2510_18221_amd/libeco.so.  Translation units compile in parallel.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libeco.so")
ARCH = os.environ.get("ECO_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(HERE, "..", "include")]
# Device code: no packed-FP32 instructions; IEEE-correct FP32 divide/sqrt.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fhip-fp32-correctly-rounded-divide-sqrt", "-munsafe-fp-atomics"]


def _units():
    units = []
    for wdt in (0, 1, 2):
        units.append((os.path.join(CSRC, "eco_forward.hip"), os.path.join(OBJ, f"eco_forward_w{wdt}.o"),
                      DEVICE + [f"-DECO_FWD_WDT={wdt}"]))
    units.append((os.path.join(CSRC, "eco_step.hip"), os.path.join(OBJ, "eco_step.o"), DEVICE))
    units.append((os.path.join(CSRC, "eco_runtime.cpp"), os.path.join(OBJ, "eco_runtime.o"), []))
    return units


def _compile(src, obj, extra, verbose):
    cmd = [HIPCC] + COMMON + extra + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u[0], u[1], u[2], verbose), units))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
