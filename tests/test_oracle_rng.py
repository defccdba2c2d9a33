"""Pins for the oracle's Philox4x32-10 and U01 (counter-based stand-in for the
IPU hardware RNG of Sec. 3.1.3 / App. A.1).

The independent reference is rocRAND's header-only philox4x32_10 engine
(a separate implementation of Salmon et al., SC'11), compiled here on the
host with g++; counter words (x, y) map to the engine's offset/4 and (z, w)
to its subsequence."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O

ROCRAND = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long key = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(key, sub, off);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_exe():
    if not os.path.exists(ROCRAND) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    d = tempfile.mkdtemp()
    src, exe = os.path.join(d, "p.cpp"), os.path.join(d, "p")
    open(src, "w").write(_PROG)
    subprocess.check_call(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", src, "-o", exe])
    yield exe
    shutil.rmtree(d)


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(123)
    rows = rng.integers(0, 2**32, size=(400, 6), dtype=np.uint64)
    rows[:, 1] %= 2**30  # offset*4 must not overflow 64 bits in the engine's API
    rows[:4] = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0],
                [0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    inp = "\n".join(" ".join(str(int(x)) for x in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], np.uint64)
    for r, e in zip(rows, ref):
        got = O.philox(r[:4].astype(np.uint32), r[4:].astype(np.uint32))
        assert got.tolist() == e.tolist(), (r, got, e)


def test_philox_zero_vector():
    # counter 0, key 0: the all-zero known answer of Philox4x32-10 (also what
    # the rocRAND engine yields for seed 0, subsequence 0, offset 0)
    assert O.philox([0, 0, 0, 0], [0, 0]).tolist() == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


def test_philox_avalanche():
    # flipping any single counter bit changes about half of the 128 output bits
    base = O.philox([1, 2, 3, 4], [5, 6])
    flips = []
    for w in range(4):
        for b in (0, 7, 31):
            c = [1, 2, 3, 4]
            c[w] ^= 1 << b
            o = O.philox(c, [5, 6])
            flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(o, base)))
    assert 40 < np.mean(flips) < 88


def test_u01_closed_form():
    assert O.u01(0) == 0.0
    assert O.u01(0xFF) == 0.0
    assert O.u01(0x100) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert O.u01(0x80000000) == 0.5
    xs = np.random.default_rng(0).integers(0, 2**32, 2000, dtype=np.uint64)
    for x in xs:
        assert O.u01(int(x)) == (int(x) >> 8) / 2.0 ** 24
