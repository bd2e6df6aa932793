"""Pins of the oracle's random-number pieces (CPU only).

Philox4x32-10 is pinned against rocRAND's engine, run as an independent
implementation (its public device API compiled for the host); the uniform
conversions against their exact ranges; Box-Muller against its defining
polar identities and the normal distribution.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_engine():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp(prefix="ppf_rr_")
    exe = os.path.join(d, "rocrand_engine")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_ref", "rocrand_engine.cpp")],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_independent_engine(orc, rocrand_engine):
    rng = np.random.default_rng(12345)
    rows = []
    for _ in range(3000):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        c = rng.integers(0, 2**32, 4, dtype=np.uint64)
        c[1] >>= 2  # the engine's 64-bit offset reaches counter word 1 only below 2^30
        rows.append((seed, c))
    # the counters the filter actually uses: small indices, purpose words, track 0
    for i in range(64):
        for purpose in (1, 2, 3, 4):
            rows.append((1, np.array([i, i % 7, (purpose << 24) | (i & 1), 0], dtype=np.uint64)))
    inp = "".join("%x %x %x %x %x\n" % (s, *[int(x) for x in c]) for s, c in rows)
    out = subprocess.run([rocrand_engine], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(x, 16) for x in line.split()] for line in out.stdout.strip().split("\n")],
                   dtype=np.uint64)
    mine = np.stack([orc.philox(s, np.array(c, dtype=np.uint32))[0] for s, c in rows]).astype(np.uint64)
    assert ref.shape == mine.shape
    assert np.array_equal(ref, mine)


def test_philox_uniformity_and_avalanche(orc):
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    out = orc.philox(7, ctr)
    # byte histogram of all words: chi-square against uniform
    b = out.view(np.uint8).ravel()
    hist = np.bincount(b, minlength=256)
    _, p = stats.chisquare(hist)
    assert p > 1e-4
    # flipping one counter bit flips about half of the 128 output bits
    flipped = ctr.copy()
    flipped[:, 2] ^= 1
    d = np.unpackbits((out ^ orc.philox(7, flipped)).view(np.uint8)).reshape(n, -1).sum(1)
    assert abs(d.mean() - 64.0) < 0.5


def test_uniform_conversions_exact(orc):
    assert orc.u24_open_hi(0) == 0.0
    assert orc.u24_open_hi(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert orc.u24_open_lo(0) == 2.0**-24
    assert orc.u24_open_lo(0xFFFFFFFF) == 1.0
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    rng = np.random.default_rng(3)
    for a in rng.integers(0, 2**32, 200, dtype=np.uint64):
        a = int(a)
        for u in (orc.u24_open_hi(a), orc.u24_open_lo(a)):
            assert float(np.float32(u)) == u  # exactly representable in fp32
        # only the top 24 bits matter
        assert orc.u24_open_hi(a) == orc.u24_open_hi(a | 0xFF)
    # u53 is a strictly increasing function of (a, b >> 11)
    assert orc.u53(1, 0) == 2.0**-32
    assert orc.u53(0, 1 << 11) == 2.0**-53
    assert orc.u53(0, (1 << 11) - 1) == 0.0


WIDTHS = (24, 18, 24, 18, 24, 18)  # radius 0, angle 0, radius 1, angle 1, radius 2, angle 2


def fields_flat(orc, words):
    rad, ang = orc.normal_fields(np.array(words, dtype=np.uint32))
    return [rad[0], ang[0], rad[1], ang[1], rad[2], ang[2]]


def test_normal_fields_partition_the_block(orc):
    # every one of the low 126 bits of the block moves exactly one bit of
    # exactly one field, in order; the top two bits move nothing
    rng = np.random.default_rng(8)
    base = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
    f0 = fields_flat(orc, base)
    for f, w in zip(f0, WIDTHS):
        assert 0 <= f < (1 << w)
    seen = []
    for bit in range(128):
        words = list(base)
        words[bit // 32] ^= 1 << (bit % 32)
        diff = [(i, a ^ b) for i, (a, b) in enumerate(zip(f0, fields_flat(orc, words))) if a != b]
        if bit >= 126:
            assert diff == []
            continue
        assert len(diff) == 1 and bin(diff[0][1]).count("1") == 1
        seen.append((diff[0][0], diff[0][1].bit_length() - 1))
    # bits 0..125 map to (field, bit) in lexicographic order: a bijection
    assert seen == [(i, b) for i, w in enumerate(WIDTHS) for b in range(w)]
    # the same fields read from the block as one 128-bit integer
    for words in rng.integers(0, 2**32, (50, 4), dtype=np.uint64):
        X = sum(int(v) << (32 * j) for j, v in enumerate(words))
        off, ref = 0, []
        for w in WIDTHS:
            ref.append((X >> off) & ((1 << w) - 1))
            off += w
        assert fields_flat(orc, [int(v) for v in words]) == ref


def test_box_muller_polar_identities(orc):
    rng = np.random.default_rng(5)
    for rad, ang in zip(rng.integers(0, 2**24, 500), rng.integers(0, 2**18, 500)):
        rad, ang = int(rad), int(ang)
        z0, z1 = orc.box_muller(rad, ang)
        u1, u2 = (rad + 1) / 2.0**24, ang / 2.0**18
        assert math.isclose(z0 * z0 + z1 * z1, -2.0 * math.log(u1), rel_tol=1e-12, abs_tol=1e-300)
        if z0 * z0 + z1 * z1 > 1e-20:
            a = math.atan2(z1, z0) % (2 * math.pi)
            d = abs(a - 2 * math.pi * u2)
            assert min(d, 2 * math.pi - d) < 1e-9
    # the extreme fields: radius field 2^24 - 1 is u = 1 (z = 0), field 0 the
    # largest radius; angle field 0 is angle 0
    assert orc.box_muller(2**24 - 1, 12345) == (0.0, 0.0)
    z0, z1 = orc.box_muller(0, 0)
    assert z1 == 0.0 and math.isclose(z0, math.sqrt(-2.0 * math.log(2.0**-24)), rel_tol=1e-15)


def test_box_muller_is_standard_normal(orc):
    n = 20000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    w = orc.philox(11, ctr)
    z = []
    for r in w:
        rad, ang = orc.normal_fields(r)
        for j in range(3):
            z.extend(orc.box_muller(rad[j], ang[j]))
    z = np.array(z)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.02
    # truncation of the tail at sqrt(-2 log 2^-24)
    assert np.abs(z).max() <= math.sqrt(-2.0 * math.log(2.0**-24)) + 1e-12
