"""Sanitizer builds of the host code (CPU only).

* The oracle's C, built with AddressSanitizer and UndefinedBehaviorSanitizer
  (undefined behaviour aborts), under its pin tests: the same tests that
  hold its arithmetic, loaded into a Python process with the sanitizer
  runtimes preloaded.
* The library's host BVH builder, built with ThreadSanitizer and then with
  AddressSanitizer + UndefinedBehaviorSanitizer into a small driver
  (tests/c/bvh_threads.cpp) that builds a triangle soup on one thread and on
  many, compares the trees byte for byte, and builds a two-level layout.
  The builder's parallel thresholds are lowered for these builds so that a
  small soup reaches every threaded stage.

Each test needs gcc / g++ with the sanitizer runtimes; it is skipped where
they are missing."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_20061_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _runtime(name):
    cc = shutil.which("gcc")
    if not cc:
        return None
    p = subprocess.run([cc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _need(*names):
    paths = [_runtime(n) for n in names]
    if not shutil.which("g++") or not all(paths):
        pytest.skip("gcc sanitizer runtimes not available")
    return paths


ORACLE_PIN_TESTS = ["test_oracle_rng.py", "test_oracle_sincos.py", "test_oracle_geometry.py", "test_oracle_bsdf.py",
                    "test_oracle_env.py", "test_oracle_render.py", "test_oracle_nif.py",
                    "test_oracle_nif_precision.py", "test_oracle_nif_train_q.py", "test_oracle_sround.py"]


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _need("libasan.so", "libubsan.so")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-fPIC", "-shared", os.path.join(ROOT, "oracle", "npt_oracle.c"), "-o", lib, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", NPT_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", t) for t in ORACLE_PIN_TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def _driver(tmp_path, name, sanitize):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", *sanitize,
                    "-D__HIP_PLATFORM_AMD__", "-DNPT_BVH_PARALLEL_PRIMS=8000u", "-DNPT_BVH_PARALLEL_BIN=16384u",
                    "-DNPT_BVH_PARALLEL_RANGE=4096u", f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}",
                    f"-I{CSRC}", os.path.join(ROOT, "tests", "c", "bvh_threads.cpp"),
                    os.path.join(CSRC, "bvh_build.cpp"), "-o", exe], check=True)
    return exe


def test_bvh_builder_under_tsan(tmp_path):
    _need("libtsan.so")
    exe = _driver(tmp_path, "bvh_tsan", ["-fsanitize=thread"])
    r = subprocess.run([exe, "30000"], env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"),
                       capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ThreadSanitizer" not in r.stderr
    assert r.stdout.count("identical") == 4


def test_bvh_builder_under_asan_and_ubsan(tmp_path):
    _need("libasan.so", "libubsan.so")
    exe = _driver(tmp_path, "bvh_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    r = subprocess.run([exe, "60000"], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"),
                       capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.count("identical") == 4
