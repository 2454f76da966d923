"""Pins for the oracle's random numbers and point map.

Philox4x32-10 (Salmon et al., SC'11) is checked bit for bit against an
independent implementation: PyTorch's header-only ``at::philox_engine``, compiled
here from source.  The point map (one extent per dimension, paper section 3) is
checked in exact rational arithmetic on dyadic boxes.
"""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe,
                    os.path.join(HERE, "philox_torch_ref.cpp")], check=True)

    def run(triples):
        txt = "".join(f"{s} {b} {o}\n" for s, b, o in triples)
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint32)
    return run


def test_philox_block_matches_pytorch_engine(oracle_lib, torch_philox):
    rng = np.random.Generator(np.random.PCG64(7))
    triples = [(0, 0, 0), (1, 1, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1), (1, 16, 5 * 12345)]
    triples += [tuple(int(v) for v in rng.integers(0, 2**63, size=3, dtype=np.uint64))
                for _ in range(60)]
    ref = torch_philox(triples)
    for (seed, sub, off), want in zip(triples, ref):
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = oracle.philox4x32_10(ctr, key)
        assert np.array_equal(got, want), (seed, sub, off)


@pytest.mark.parametrize("d", [1, 3, 4, 8, 20, 64])
def test_words_layout(oracle_lib, torch_philox, d):
    """Word 4j+t of sample i is output t of the block with offset i*ceil(d/4)+j,
    subsequence = subvolume id, key = seed."""
    nb = (d + 3) // 4
    seed, sub = 1, 1037
    for index in (0, 1, 2**20 - 1, 2**33 + 5):
        triples = [(seed, sub, index * nb + j) for j in range(nb)]
        want = torch_philox(triples).reshape(-1)[:d]
        assert np.array_equal(oracle.words(d, seed, sub, index), want)


def test_words_are_uniform_bits(oracle_lib):
    """Sanity of the stream: the top bit of each word is a fair coin over samples."""
    w = np.stack([oracle.words(20, 1, 16, i) for i in range(4000)])
    frac = (w >> 31).mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 4 * 0.5 / np.sqrt(4000))


def _exact_point(x, lo, hi):
    return Fraction(lo) + (Fraction(int(x)) + Fraction(1, 2)) * (Fraction(hi) - Fraction(lo)) / 2**32


@pytest.mark.parametrize("box", [(-4.0, 4.0), (-1.0, 0.0), (0.5, 0.75), (-3.0, 3.0)])
def test_point_map_exact_rational(oracle_lib, box):
    """u = lo + (x + 1/2)(hi - lo)/2^32 holds exactly when the box is dyadic
    (for [-3,3] the product stays within 53 bits)."""
    d = 8
    lo = np.full(d, box[0])
    hi = np.full(d, box[1])
    for index in (0, 1, 99, 2**31 + 3):
        x = oracle.words(d, 1, 3, index)
        u = oracle.point(d, 1, 3, lo, hi, index)
        for k in range(d):
            assert Fraction(float(u[k])) == _exact_point(x[k], box[0], box[1])
            assert box[0] < u[k] < box[1]


def test_point_map_extreme_words_stay_inside():
    """x = 0 and x = 2^32-1 map strictly inside (lo, hi) for the bisected boxes
    of the workloads, and the upper half of the box is exactly the words with the
    top bit set.  fma(x, scale, base) is the correctly rounded value of
    x*scale + base, which float(Fraction(...)) reproduces."""
    for lo, hi in [(-4.0, 4.0), (0.0, 4.0), (-4.0, -3.9921875), (-3.0, 3.0), (1.5, 3.0)]:
        scale = (hi - lo) * 2.0**-32
        base = lo + 0.5 * scale
        for x in (0, 1, 2**31 - 1, 2**31, 2**32 - 1):
            u = float(Fraction(x) * Fraction(scale) + Fraction(base))
            assert lo < u < hi
            assert (u >= 0.5 * (lo + hi)) == (x >= 2**31)
