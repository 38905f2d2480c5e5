"""Pins of the oracle's random numbers (counter-based Philox, uniforms, normals).

The paper only asks for pseudo-random numbers that can be drawn in parallel
(Sec. 2.2); the stream layout is the reading this library fixes.  Pins:
the Philox words against an independent implementation (rocRAND's engine,
built for the host), exact representability of the uniforms in float, and
the normal law of the Box-Muller pairs.
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


def test_uniforms_exact_in_float_and_open_interval(ref):
    # the low 23 bits of the word select one of 2^23 equally spaced points
    w = np.array([0, 1, 2**23, 2**23 + 1, 2**31, 2**32 - 1, 2**23 - 1, 12345678], dtype=np.uint32)
    u = ref.uniforms(w)
    assert u[0] == 2.0**-24 and u[2] == 2.0**-24 and u[4] == 2.0**-24
    assert u[1] == 3 * 2.0**-24 and u[3] == 3 * 2.0**-24
    assert u[5] == 1.0 - 2.0**-24 and u[6] == 1.0 - 2.0**-24
    assert u[7] == ((12345678 % 2**23) + 0.5) * 2.0**-23
    rng = np.random.default_rng(3)
    words = rng.integers(0, 2**32, size=200000, dtype=np.uint64).astype(np.uint32)
    uu = ref.uniforms(words)
    assert np.all(uu > 0) and np.all(uu < 1)
    assert np.array_equal(uu.astype(np.float32).astype(np.float64), uu)
    # 2^23 equally likely levels: mean 1/2, variance ~1/12
    assert abs(uu.mean() - 0.5) < 4 * np.sqrt(1 / 12 / uu.size)


def test_normals_are_standard_normal(ref):
    n = 1 << 19
    ctr = np.zeros((n // 4, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n // 4)
    ctr[:, 2] = 17
    words = ref.philox(ctr, [99, 0]).reshape(-1, 2)
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
    # u_b = 1/4 + 2^-24 is close to a quarter turn: z0 ~ 0, z1 ~ radius
    ra = np.uint32(0x00400000)      # u_a = (2^22 + 1/2) 2^-23
    rb = np.uint32(0x00200000)      # u_b = (2^21 + 1/2) 2^-23
    z = ref.normals64(np.array([[ra, rb]], dtype=np.uint32))[0]
    ua = (2**22 + 0.5) * 2.0**-23
    ub = (2**21 + 0.5) * 2.0**-23
    R = np.sqrt(-2 * np.log(ua))
    assert z[0] == pytest.approx(R * np.cos(2 * np.pi * ub), abs=1e-15)
    assert z[1] == pytest.approx(R * np.sin(2 * np.pi * ub), abs=1e-15)
    assert abs(z[0]) < 1e-6 and abs(z[1] - R) < 1e-12
