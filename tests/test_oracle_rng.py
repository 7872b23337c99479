"""Pins for the oracle's random stream: Philox4x32-10 against the rocRAND
library's engine, and the uniform lattice that feeds -ln(u) (the inverse
transform of Sec. 2 and the Gumbel draws of Sec. 3.2 need u strictly inside
(0, 1))."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = str(tmp_path_factory.mktemp("kat") / "rocrand_philox")
    subprocess.check_call([hipcc, "-O1", os.path.join(HERE, "golden", "rocrand_philox.cpp"),
                           "-o", exe], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    g = np.random.default_rng(123)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6],
             [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0]]
    cases += g.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint64)
    assert ref.shape == (len(cases), 4)
    mine = np.array([orc.philox4x32_10(c[:4], c[4:]) for c in cases], np.uint64)
    assert np.array_equal(mine, ref)


def test_step_word_layout(orc):
    """Word w of step k of trajectory i is lane w%4 of block w//4 with counter
    (w//4, k, i, purpose<<24 | epoch) and key (lo32(seed), hi32(seed))."""
    seed = 0x0123456789ABCDEF
    u = orc.step_uniforms(seed, 2, 77, 1234, 99, 11)
    for w in range(11):
        blk = orc.philox4x32_10([w // 4, 99, 1234, (2 << 24) | 77], [seed & 0xFFFFFFFF, seed >> 32])
        assert u[w] == ((2 * (int(blk[w % 4]) >> 9) + 1) * 2.0 ** -24)


def test_uniform_lattice_exhaustive(orc):
    """All 2^23 lattice points are exact in FP32, lie in [2^-24, 1-2^-24], are
    distinct, and are symmetric about 1/2 (u(m) + u(2^23-1-m) = 1)."""
    m = np.arange(2 ** 23, dtype=np.int64)
    u64 = (2 * m + 1) * 2.0 ** -24
    assert np.all(u64.astype(np.float32).astype(np.float64) == u64)
    assert u64.min() == 2.0 ** -24 and u64.max() == 1 - 2.0 ** -24
    assert np.all(np.diff(u64) > 0)
    assert np.all(u64 + u64[::-1] == 1.0)
    # the oracle's conversion agrees on words spanning the whole 32-bit range
    for x in [0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFE00, 0xFFFFFFFF, 123456789]:
        assert orc.uniform(x) == (2 * (x >> 9) + 1) * 2.0 ** -24
    # -ln(u) is finite and positive everywhere on the lattice
    e = -np.log(u64)
    assert np.all(np.isfinite(e)) and np.all(e > 0)
