"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's C source is built a second time with -fsanitize=address,undefined
(into a temporary directory), and its hand-traced pins, invariants and the
property-based cross-check with the Python statement of the rules run in a
child process against that build: any out-of-bounds access, use after free or
undefined behaviour (signed overflow, bad shift, misaligned access) aborts the
child.  Leak detection is off: the Python interpreter itself keeps memory to the
end.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-fopenmp", "-o", lib,
                    os.path.join(ROOT, "oracle", "eco_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ECO_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    # the child first shows that it runs the sanitized build with the runtime in place
    probe = ("import ctypes; from oracle import oracle as o; l = o.lib(); "
             "assert o._LIB_PATH == %r; ctypes.CDLL(None).__asan_init; print('sanitized oracle loaded')" % lib)
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and "sanitized oracle loaded" in r.stdout, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_pins.py", "tests/test_oracle_fuzz.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout
