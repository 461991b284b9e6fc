"""Pins of the oracle's randomness against definitions it does not share.

* Philox4x32-10 block-for-block against rocRAND's host-callable engine, a
  library implementation of the same published generator (Salmon et al.,
  SC'11), compiled here with g++.
* The (0, 1] uniform map on its extreme words and its exact mean.
* Box-Muller normals against the N(0, 1) CDF (Kolmogorov-Smirnov).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("g++ or rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "helpers", "rocrand_philox.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(oracle, rocrand_ref):
    rng = np.random.default_rng(1234)
    rows = []
    for _ in range(400):
        k0, k1, c0, c2, c3 = (int(x) for x in rng.integers(0, 2**32, size=5, dtype=np.uint64))
        c1 = int(rng.integers(0, 2**30))  # keeps rocRAND's 64-bit offset (4 per block) in range
        rows.append((k0, k1, c0, c1, c2, c3))
    rows += [(0, 0, 0, 0, 0, 0), (2**32 - 1, 2**32 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1)]
    inp = "".join(" ".join(map(str, r)) + "\n" for r in rows)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([list(map(int, line.split())) for line in out.strip().splitlines()], dtype=np.uint64)
    got = np.array([oracle.philox4x32_10([c0, c1, c2, c3], [k0, k1]) for k0, k1, c0, c1, c2, c3 in rows],
                   dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


def test_philox_blocks_counter_layout(oracle):
    # block j of (seed, tag, id, c0) is the Philox of counter (c0 + j, id_lo, id_hi, tag)
    seed, tag, ident = 0x1234_5678_9ABC_DEF0, 7, (5 << 32) | 17
    blocks = oracle.philox_blocks(seed, tag, ident, 40, 3)
    for j in range(3):
        exp = oracle.philox4x32_10([40 + j, 17, 5, tag], [0x9ABC_DEF0, 0x1234_5678])
        np.testing.assert_array_equal(blocks[j], exp)


def test_u01_range_and_mean(oracle):
    assert oracle.u01(0) == 2.0**-24
    assert oracle.u01(0xFFFFFFFF) == 1.0
    assert oracle.u01(0x000000FF) == 2.0**-24  # low 8 bits are dropped
    # mean over the 2^24 equally likely values is 1/2 + 2^-25 exactly
    k = np.arange(1, 2**24 + 1, dtype=np.float64)
    assert np.mean(k * 2.0**-24) == 0.5 + 2.0**-25
    # the oracle's map agrees with that closed form on a random sample of words
    words = np.random.default_rng(0).integers(0, 2**32, 2000, dtype=np.uint64)
    for w in words:
        assert oracle.u01(int(w)) == ((int(w) >> 8) + 1) * 2.0**-24


def test_uniformity_chi_square(oracle):
    words = oracle.philox_blocks(0, 0, 99, 0, 50000).reshape(-1)
    u = ((words >> 8) + 1) * 2.0**-24
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2, p = stats.chisquare(hist)
    assert p > 1e-4, (chi2, p)


def test_box_muller_normals(oracle):
    import ctypes as C
    L = oracle.lib()
    L.or_normal4.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_void_p]
    vals = np.zeros((20000, 4))
    for i in range(20000):
        L.or_normal4(3, 5, i, 0, vals[i].ctypes.data)
    x = vals.reshape(-1)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1) < 5 * np.sqrt(2 / x.size)
