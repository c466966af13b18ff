"""Pins of the oracle's random-number primitives.

* Philox4x32-10 against PyTorch's open-source engine (an independent
  implementation of Salmon et al., SC'11), over edge and random counters.
* ``mulhi`` (the map of a 32-bit word onto [0, n)) against its closed form:
  value v is taken by exactly the words w with ceil(v*2^32/n) <= w <
  ceil((v+1)*2^32/n), so each value is hit floor(2^32/n) or ceil(2^32/n)
  times.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    import torch.utils.cpp_extension as ext
    for d in ext.include_paths():
        if os.path.exists(os.path.join(d, "ATen", "core", "PhiloxRNGEngine.h")):
            return d
    return None


@pytest.fixture(scope="module")
def torch_kat(tmp_path_factory):
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("PyTorch headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("kat") / "torch_philox_kat")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc,
                    os.path.join(HERE, "torch_philox_kat.cpp"), "-o", exe],
                   check=True)

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True,
                             check=True).stdout.split("\n")
        return [tuple(int(x) for x in line.split()) for line in out if line.strip()]
    return run


def test_philox_matches_pytorch_engine(orc, torch_kat):
    rng = np.random.default_rng(12345)
    rows = [(0, 0, 0, 0, 0),
            (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFFFFFFFFFF),
            (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0x299F31D0A4093822),
            (1, 0, 0, 0, 1), (0, 1, 0, 0, 1), (0, 0, 1, 0, 1), (0, 0, 0, 1, 1)]
    # the counter shapes the GA uses: (slot, island, generation, purpose)
    for purpose in range(4):
        rows.append((31, 524287, 9999, purpose, 1))
        rows.append((0, 65535, 19999, purpose, 64))
    for _ in range(200):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        s = int(rng.integers(0, 2**63, dtype=np.uint64)) * 2 + int(rng.integers(0, 2))
        rows.append((int(c[0]), int(c[1]), int(c[2]), int(c[3]), s))
    expect = torch_kat(rows)
    got = [orc.philox(*r) for r in rows]
    assert got == expect


def test_philox_is_counter_sensitive(orc):
    base = orc.philox(5, 6, 7, 0, 1)
    assert orc.philox(5, 6, 7, 1, 1) != base
    assert orc.philox(5, 6, 8, 0, 1) != base
    assert orc.philox(5, 6, 7, 0, 2) != base


@pytest.mark.parametrize("n", [1, 2, 3, 4, 16, 17, 31, 32, 33, 63, 64, 1000, 4097])
def test_mulhi_boundaries_match_closed_form(orc, n):
    two32 = 1 << 32
    vals = list(range(min(n, 80))) + list(range(max(0, n - 5), n))
    for v in vals:
        first = -(-v * two32 // n)            # ceil(v * 2^32 / n)
        nxt = -(-(v + 1) * two32 // n)
        assert orc.mulhi(first, n) == v
        if first > 0:
            assert orc.mulhi(first - 1, n) == v - 1
        assert orc.mulhi(nxt - 1, n) == v
        assert nxt - first in (two32 // n, -(-two32 // n))


def test_mutation_threshold_is_one_percent():
    # p = 0.01 as a threshold on a uniform 32-bit word: floor(0.01 * 2^32)
    thr = 42949672
    assert thr == int(0.01 * 2**32)
    assert abs(thr / 2**32 - 0.01) < 1e-9
