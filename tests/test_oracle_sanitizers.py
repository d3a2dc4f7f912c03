"""The oracle under sanitizers (CPU): tests/oracle_sanitize_driver.c calls
every entry point of the oracle on a small scene (maps, bubbly pane, photon
map, both intersection walks, item ranges, the slab Monte Carlo and the
network) and is built with the oracle's sources

- with gcc and AddressSanitizer + UndefinedBehaviorSanitizer (leak checks
  on, undefined behaviour fatal);
- with ROCm's clang, its OpenMP runtime and ThreadSanitizer, the runtime's
  Archer tool making the OpenMP synchronisation visible (so the parallel
  render loops are checked for data races without the false reports an
  uninstrumented OpenMP runtime gives).

Each run must end with exit status 0 and no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")
SOURCES = [os.path.join(ROOT, "oracle", s) for s in ("sdm_oracle.c", "slab_mc.c", "mlp.c")]
LLVM = "/opt/rocm/llvm"


def run(cmd, env=None, timeout=600):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_asan")
    b = run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
             "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", DRIVER, *SOURCES, "-lm", "-o", exe])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
    r = run([exe], env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "all calls ran" in r.stdout


def test_oracle_under_tsan(tmp_path):
    clang = os.path.join(LLVM, "bin", "clang")
    archer = os.path.join(LLVM, "lib", "libarcher.so")
    if not (os.path.exists(clang) and os.path.exists(archer)):
        pytest.skip("ROCm clang with the OpenMP runtime's Archer tool not available")
    exe = str(tmp_path / "orc_tsan")
    lib = os.path.join(LLVM, "lib")
    b = run([clang, "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=thread", DRIVER,
             *SOURCES, "-lm", f"-L{lib}", f"-Wl,-rpath,{lib}", "-o", exe])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", OMP_TOOL_LIBRARIES=archer,
               TSAN_OPTIONS="ignore_noninstrumented_modules=1:halt_on_error=1")
    r = run([exe], env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "all calls ran" in r.stdout
