"""Pins of the oracle's counter-based generator (Philox4x32-10 of Salmon et
al., SC'11) and of the Box-Muller normals built on it."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats as sst

from inputs import rand
from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h") or not shutil.which("g++"):
        pytest.skip("rocRAND header or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    subprocess.check_call(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe])
    return exe


def test_philox_equals_rocrand_header(rocrand_ref):
    r = rand.rng(11)
    n = 2000
    words = r.integers(0, 2 ** 32, (n, 6), dtype=np.uint64)
    words[:4] = [[0] * 6, [2 ** 32 - 1] * 6, [1, 2, 3, 4, 5, 6], [0, 7, 0, 1, 0x22031185, 0]]
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in words) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    got = np.stack(philox.philox4x32_10(*[words[:, i] for i in range(6)]), axis=1).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_source_bits_layout(rocrand_ref):
    """Bit i of codeword b is bit i%32 of word (i//32)%4 of block i//128."""
    seed, cw0, B, k = 0x2203118500000102, 5, 3, 300
    u = philox.source_bits(seed, cw0, B, k)
    lines = []
    for b in range(B):
        for j in range(-(-k // 128)):
            lines.append(f"{j} {cw0 + b} 0 0 {seed & 0xffffffff} {seed >> 32}")
    out = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split()
    words = np.array([int(t) for t in out], dtype=np.uint64).reshape(B, -1)
    for b in range(B):
        for i in range(k):
            assert u[b, i] == (int(words[b, i // 32]) >> (i % 32)) & 1


def test_bits_balanced():
    u = philox.source_bits(123, 0, 400, 2500).astype(np.int64)
    n = u.size
    ones = int(u.sum())
    chi2 = (ones - n / 2) ** 2 / (n / 4)
    assert chi2 < sst.chi2.ppf(0.999, 1)


def test_normals_moments():
    g = philox.normals(77, 0, 1000, 2000).reshape(-1)
    x = np.concatenate([g.real, g.imag])
    n = x.size
    assert abs(x.mean()) < 4.5 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 4.5 * math.sqrt(2.0 / n)
    kurt = np.mean(x ** 4) / np.mean(x ** 2) ** 2
    assert abs(kurt - 3.0) < 4.5 * math.sqrt(24.0 / n)
    # real and imaginary parts uncorrelated
    assert abs(np.mean(g.real * g.imag)) < 4.5 / math.sqrt(g.size)


def test_normals_are_box_muller_of_the_stream(rocrand_ref):
    seed, b, S = 99, 7, 6
    g = philox.normals(seed, b, 1, S)[0]
    lines = [f"{j} {b} 0 1 {seed} 0" for j in range(S // 2)]
    out = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split()
    w = [int(t) for t in out]
    for s in range(S):
        xa, xb = w[4 * (s // 2) + 2 * (s % 2)], w[4 * (s // 2) + 2 * (s % 2) + 1]
        rho = math.sqrt(-2 * math.log((xa + 1) / 2 ** 32))
        ang = 2 * math.pi * xb / 2 ** 32
        assert abs(g[s] - complex(rho * math.cos(ang), rho * math.sin(ang))) < 1e-12
