"""Pins of the oracle's random numbers (counter-based Philox, uniforms, normals).

The paper only asks for pseudo-random numbers that can be drawn in parallel
(Sec. 2.2); the stream layout is the reading this library fixes.  Pins:
the Philox words against an independent implementation (rocRAND's engine,
built for the host), the bit layout of a block's six 21-bit fields (hand
blocks, and every bit moving exactly one field), exact representability of
the uniforms in float, and the normal law of the Box-Muller pairs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_words(tmp_path, seeds_ctrs):
    exe = str(tmp_path / "rocrand_words")
    cxx = shutil.which("g++")
    if cxx is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or g++ missing")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    os.path.join(HERE, "pins", "rocrand_words.cpp"), "-o", exe], check=True)
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in seeds_ctrs) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand_engine(ref, tmp_path):
    rng = np.random.default_rng(7)
    rows = []
    for seed in (0, 1, 5, 0x123456789ABCDEF, 2**64 - 1):
        for _ in range(400):
            c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
            c[1] %= 2**30
            rows.append([seed, *c])
        rows.append([seed, 0, 0, 0, 0])
        rows.append([seed, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1])
    rows = np.array(rows, dtype=np.uint64)
    want = _rocrand_words(tmp_path, rows)
    got = np.concatenate([
        ref.philox(rows[rows[:, 0] == s][:, 1:].astype(np.uint32), [int(s) & 0xFFFFFFFF, int(s) >> 32])
        for s in dict.fromkeys(rows[:, 0].tolist())])
    assert got.shape == want.shape
    assert np.array_equal(got.astype(np.uint64), want)


def test_block_fields_hand_blocks(ref):
    # fields: steps 3m, 3m+1 take words (0,1), (2,3) >> 11; step 3m+2 takes
    # (w0 & 0x7ff) | (w1 & 0x3ff) << 11 and (w2 & 0x7ff) | (w3 & 0x3ff) << 11
    blk = np.array([[0xFFFFF800, 0x000007FF, 0x00000400, 0x00000400]], dtype=np.uint32)
    u = ref.block_uniforms(blk)[0]
    f = 2.0**-21
    want = [((2**21 - 1) + 0.5) * f, 0.5 * f, 0.5 * f, 0.5 * f, (0x3FF * 2**11 + 0.5) * f, (0x400 + 0.5) * f]
    assert list(u) == want


def test_block_fields_partition_the_bits(ref):
    # every bit of a block moves exactly one of the six uniforms, except bit
    # 10 of words 1 and 3, which moves none
    rng = np.random.default_rng(11)
    base = rng.integers(0, 2**32, size=(1, 4), dtype=np.uint64).astype(np.uint32)
    u0 = ref.block_uniforms(base)[0]
    for w in range(4):
        for bit in range(32):
            blk = base.copy()
            blk[0, w] ^= np.uint32(1 << bit)
            moved = int(np.sum(ref.block_uniforms(blk)[0] != u0))
            assert moved == (0 if (w in (1, 3) and bit == 10) else 1), (w, bit)


def test_uniforms_exact_in_float_and_open_interval(ref):
    rng = np.random.default_rng(3)
    blocks = rng.integers(0, 2**32, size=(50000, 4), dtype=np.uint64).astype(np.uint32)
    uu = ref.block_uniforms(blocks).ravel()
    assert np.all(uu > 0) and np.all(uu < 1)
    assert uu.min() >= 2.0**-22 and uu.max() <= 1 - 2.0**-22
    assert np.array_equal(uu.astype(np.float32).astype(np.float64), uu)
    # 2^21 equally likely levels: mean 1/2, variance ~1/12
    assert abs(uu.mean() - 0.5) < 4 * np.sqrt(1 / 12 / uu.size)
    assert abs(uu.var() - 1 / 12) < 4 * np.sqrt(1 / 180 / uu.size)


def _fields(ref, blocks):
    """The 21-bit fields [n*3][2] of blocks, from the oracle's own uniforms."""
    u = ref.block_uniforms(blocks).reshape(-1, 2)
    return np.rint(u * 2**21 - 0.5).astype(np.uint32)


def test_normals_are_standard_normal(ref):
    n = 1 << 19
    ctr = np.zeros((n // 4, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n // 4)
    ctr[:, 2] = 17
    words = _fields(ref, ref.philox(ctr, [99, 0]))
    z = ref.normals64(words).ravel()
    N = z.size
    assert abs(z.mean()) < 4.3 / np.sqrt(N)
    assert abs(z.var() - 1.0) < 4.3 * np.sqrt(2.0 / N)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # pairs are uncorrelated and the radius is the Rayleigh law
    zz = ref.normals64(words)
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 4.3 / np.sqrt(zz.shape[0])
    r2 = (zz**2).sum(1)
    assert stats.kstest(r2, "expon", args=(0, 2)).pvalue > 1e-3


def test_box_muller_special_angles(ref):
    # u_b = 1/4 + 2^-22 is close to a quarter turn: z0 ~ 0, z1 ~ radius
    fa, fb = 2**20, 2**19          # u_a = (2^20 + 1/2) 2^-21, u_b = (2^19 + 1/2) 2^-21
    z = ref.normals64(np.array([[fa, fb]], dtype=np.uint32))[0]
    ua = (fa + 0.5) * 2.0**-21
    ub = (fb + 0.5) * 2.0**-21
    R = np.sqrt(-2 * np.log(ua))
    assert z[0] == pytest.approx(R * np.cos(2 * np.pi * ub), abs=1e-15)
    assert z[1] == pytest.approx(R * np.sin(2 * np.pi * ub), abs=1e-15)
    assert abs(z[0]) < 4e-6 and abs(z[1] - R) < 1e-10

