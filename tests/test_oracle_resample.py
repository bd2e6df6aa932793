"""Pins of the oracle's systematic and RNA resampling (CPU only): offspring
invariants, special cases, and exact rational enumeration over the uniform on
tiny inputs (the brute-force enumerator is itself pinned by the exact
identity E_u[o_j] = N w_j)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute


def dyadic_weights(rng, n, bits=20, zeros=0):
    """Random weights exactly representable in fp64 and summing to 1 exactly."""
    k = rng.integers(1, 1 << 10, n).astype(np.int64)
    if zeros:
        k[rng.choice(n, zeros, replace=False)] = 0
    # scale so the total is a power of two: w = k / 2^bits with sum 2^bits
    tot = int(k.sum())
    scale = (1 << bits) // tot
    k = k * scale
    k[np.argmax(k)] += (1 << bits) - int(k.sum())
    fr = [Fraction(int(v), 1 << bits) for v in k]
    return np.array([float(f) for f in fr]), fr


def test_systematic_offspring_invariants(orc):
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 100, 4096):
        for _ in range(20):
            w = rng.exponential(size=n) ** 3
            w[rng.random(n) < 0.2] = 0.0
            if w.sum() == 0:
                w[0] = 1
            w /= w.sum()
            u = rng.random()
            anc = orc.resample_systematic(w, u)
            assert np.all(np.diff(anc) >= 0)
            o = np.bincount(anc, minlength=n)
            assert o.sum() == n
            nw = n * w
            # floor/ceil up to fp rounding of the running CDF
            assert np.all(o >= np.floor(nw - 1e-9)) and np.all(o <= np.ceil(nw + 1e-9))
            assert np.all(o[w == 0] == 0)


def test_systematic_special_cases(orc):
    # with exactly representable uniform weights even u = 0 sits exactly on
    # the CDF steps and still gives the identity; with 1/1000 only u away
    # from the steps is decided exactly (the steps carry fp rounding)
    for n, us in ((1024, (0.0, 0.3, 0.999999)), (1000, (0.3, 0.7))):
        for u in us:
            assert np.array_equal(orc.resample_systematic(np.full(n, 1.0 / n), u), np.arange(n))
    n = 1000
    w = np.zeros(n)
    w[417] = 1.0
    assert np.all(orc.resample_systematic(w, 0.5) == 417)


def test_brute_force_enumerator_is_unbiased():
    rng = np.random.default_rng(1)
    for n in range(1, 9):
        _, fr = dyadic_weights(rng, n, zeros=min(2, n - 1))
        e = brute.expected_offspring(fr)
        assert e == [n * x for x in fr]
        # every outcome has offspring counts floor/ceil of N w
        for lo, hi, anc in brute.systematic_pieces(fr):
            o = [anc.count(j) for j in range(n)]
            for j in range(n):
                assert math.floor(n * fr[j]) <= o[j] <= math.ceil(n * fr[j])


def test_systematic_matches_brute_force(orc):
    rng = np.random.default_rng(2)
    for n in range(1, 9):
        for trial in range(10):
            w, fr = dyadic_weights(rng, n, zeros=int(trial % 3 == 0) * min(2, n - 1))
            for lo, hi, anc in brute.systematic_pieces(fr):
                mid = float((lo + hi) / 2)
                assert tuple(orc.resample_systematic(w, mid)) == anc
                assert tuple(orc.resample_systematic(w, float(lo))) == anc


def test_post_resample_mean_is_unbiased_exactly():
    rng = np.random.default_rng(3)
    for n in (3, 5, 8):
        _, fr = dyadic_weights(rng, n)
        xs = [Fraction(int(v)) for v in rng.integers(-50, 50, n)]
        e = Fraction(0)
        for lo, hi, anc in brute.systematic_pieces(fr):
            e += (hi - lo) * sum(xs[a] for a in anc) / n
        assert e == sum(w * x for w, x in zip(fr, xs))


# ----------------------------------------------------------------- RNA
def test_rna_single_group_equals_systematic(orc):
    rng = np.random.default_rng(4)
    n = 256
    w = rng.exponential(size=n) ** 4
    w /= w.sum()
    for moved in (0, 25, 100):
        anc, lwg, lws = orc.resample_rna(w, n, moved, np.array([0.37]))
        assert np.array_equal(anc, orc.resample_systematic(w, 0.37))
        assert np.allclose(lws, math.log(w.sum() / n), rtol=1e-14)


def test_rna_group_invariants(orc):
    rng = np.random.default_rng(5)
    n, grp = 4096, 256
    G = n // grp
    moved = 25
    w = rng.exponential(size=n) ** 3
    w[512:768] = 0.0  # an empty group keeps the identity map and weight 0
    w /= w.sum()
    ug = rng.random(G)
    anc, lwg, lws = orc.resample_rna(w, grp, moved, ug)
    W = w.reshape(G, grp).sum(1)
    for g in range(G):
        sl = slice(g * grp, (g + 1) * grp - moved)
        own = anc[sl]
        assert np.all((own >= g * grp) & (own < (g + 1) * grp))  # local resampling
        assert np.all(np.diff(own) >= 0)
        prev = (g - 1) % G
        recv = anc[(g + 1) * grp - moved:(g + 1) * grp]
        assert np.all((recv >= prev * grp) & (recv < (prev + 1) * grp))
        if W[g] > 0:
            assert np.allclose(np.exp(lws[sl]), W[g] / grp, rtol=1e-13)
        else:
            assert np.array_equal(own, np.arange(g * grp, (g + 1) * grp - moved))
            assert np.all(np.isneginf(lws[sl]))
    # particle count per group fixed, total weight conserved
    assert math.isclose(math.fsum(np.exp(lws)), 1.0, rel_tol=1e-12)
    # ancestors of the received slots are the ones group g-1 drew for them
    anc0, _, _ = orc.resample_rna(w, grp, 0, ug)
    for g in range(G):
        prev = (g - 1) % G
        assert np.array_equal(anc[(g + 1) * grp - moved:(g + 1) * grp],
                              anc0[(prev + 1) * grp - moved:(prev + 1) * grp])


def test_rna_matches_brute_force(orc):
    rng = np.random.default_rng(6)
    n, grp = 8, 4
    for trial in range(6):
        w, fr = dyadic_weights(rng, n, zeros=trial % 3)
        for moved in (0, 1, 2):
            pieces = brute.rna_pieces(fr, grp, moved)
            assert sum(p for p, _, _ in pieces) == 1
            # weight per slot is conserved exactly in every outcome
            for prob, anc, wslot in pieces:
                assert sum(wslot) == 1
            G = n // grp
            per_group = [brute.systematic_pieces([x / sum(fr[g * grp:(g + 1) * grp]) for x in
                                                  fr[g * grp:(g + 1) * grp]])
                         if sum(fr[g * grp:(g + 1) * grp]) > 0 else [(Fraction(0), Fraction(1), None)]
                         for g in range(G)]
            for a in per_group[0]:
                for b in per_group[1]:
                    us = [(a[0] + a[1]) / 2, (b[0] + b[1]) / 2]
                    anc_b, wslot = brute.rna_at(fr, grp, moved, us)
                    anc_o, _, lws = orc.resample_rna(w, grp, moved, np.array([float(v) for v in us]))
                    assert tuple(anc_o) == anc_b
                    assert np.allclose(np.exp(lws), [float(x) for x in wslot], rtol=1e-14)
