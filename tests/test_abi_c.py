"""The C ABI from plain C: tests/c/host_only.c is compiled as C99 against
include/npt.h with every warning an error, linked against libnpt.so and run
on a host-only context (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

from paper_2305_20061_amd import npt

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_plain_c_client_builds_and_runs(tmp_path):
    npt.lib()  # the library is built
    exe = str(tmp_path / "host_only")
    libdir = os.path.dirname(npt.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.dirname(npt.HEADER),
           os.path.join(HERE, "c", "host_only.c"), "-o", exe, "-L", libdir, "-lnpt", f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_binding_structs_match_the_c_layout(tmp_path):
    # every ctypes mirror in the binding has the size the C compiler gives the
    # header's struct (a field added on one side only would show here)
    import ctypes

    exe = str(tmp_path / "struct_sizes")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.dirname(npt.HEADER),
           os.path.join(HERE, "c", "struct_sizes.c"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout.split("\n")
    sizes = dict(line.split() for line in out if line.strip())
    assert len(sizes) == 9
    for name, size in sizes.items():
        assert ctypes.sizeof(getattr(npt, name)) == int(size), name
