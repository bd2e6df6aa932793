"""Pins of the oracle's ARNA (adaptive RNA, Section 6.4), whose rules the
paper names without defining them; the reading implemented (design notes):
  - a group tracks when its share of the normalised weight is at least
    theta / G;
  - the exchange shrinks with the share of tracking groups: mu = mu_min +
    floor((mu_max - mu_min) (G - G_t) / G) slots per group;
  - the ring order is redrawn as a keyed permutation whenever the object is
    lost: the frame's log-likelihood increment falls more than kappa P below
    that of the last frame that was not lost; it is kept until the next loss
    (key 0, before any loss: the index order, RNA's ring).
Pinned against: exact rational enumeration (brute.arna_at), RNA (itself
pinned by enumeration) as the special case mu_min = mu_max with the index
ring, hand-worked exchange sizes, the total weight carried through any ring,
the permutation's bijectivity and spread over keys, and the lost test's
closed form on noise-free frames."""
import itertools
import math
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from paper_1310_5045_amd import synth


def test_ring_order_is_a_keyed_bijection(orc):
    m = orc.Model()
    for G in list(range(1, 70)) + [255, 256, 257, 4096, 5000]:
        for key in (1, 2, 99, 2**31 - 1):
            o = orc.ring_order(m, key, G)
            assert np.array_equal(np.sort(o), np.arange(G)), (G, key)
            assert np.array_equal(o, orc.ring_order(m, key, G))  # a pure function of the key
        assert np.array_equal(orc.ring_order(m, 0, G), np.arange(G))  # before any loss
    # the key, the seed and the track all change the order
    base = orc.ring_order(m, 5, 64)
    assert not np.array_equal(base, orc.ring_order(m, 6, 64))
    assert not np.array_equal(base, orc.ring_order(orc.Model(seed=2), 5, 64))
    assert not np.array_equal(base, orc.ring_order(orc.Model(track=3), 5, 64))


def test_ring_orders_spread_over_all_permutations(orc):
    """Over 3000 keys every ordering of 5 groups occurs, and each group
    takes each ring position about equally often (chi-square, 16 dof,
    far below its 0.001 quantile of 39.3)."""
    m = orc.Model(seed=11)
    G, K = 5, 3000
    seen = Counter()
    pos = np.zeros((G, G))
    for key in range(1, K + 1):
        o = orc.ring_order(m, key, G)
        seen[tuple(o)] += 1
        pos[o, np.arange(G)] += 1
    assert len(seen) == math.factorial(G)
    chi2 = ((pos - K / G) ** 2 / (K / G)).sum()
    assert chi2 < 39.3, chi2


def rational_weights(rng, n, zero_frac=0.2):
    k = rng.integers(1, 40, n)
    k[rng.random(n) < zero_frac] = 0
    if k.sum() == 0:
        k[0] = 1
    return [Fraction(int(v), int(k.sum())) for v in k], k / k.sum()


def test_arna_matches_brute_force(orc):
    rng = np.random.default_rng(4)
    for trial in range(40):
        group = int(rng.integers(2, 5))
        G = int(rng.integers(2, 5))
        n = group * G
        fr, w = rational_weights(rng, n)
        mu_max = int(rng.integers(0, group + 1))
        mu_min = int(rng.integers(0, mu_max + 1))
        theta = Fraction(int(rng.integers(1, 9)), 8)
        order = rng.permutation(G)
        # uniforms at the middle of a piece of each group's local map
        us = []
        for g in range(G):
            ws = fr[g * group:(g + 1) * group]
            W = sum(ws, Fraction(0))
            pieces = brute.systematic_pieces([x / W for x in ws]) if W else [(0, 1, None)]
            lo, hi, _ = pieces[int(rng.integers(0, len(pieces)))]
            us.append(Fraction(lo + hi) / 2)
        anc_b, ws_b, t_b, mu_b = brute.arna_at(fr, group, mu_min, mu_max, theta, us, order)
        anc, lwg, lws, t, mu = orc.resample_arna(w, group, mu_min, mu_max, float(theta),
                                                 np.array([float(u) for u in us]), order)
        # a group weight exactly at theta / G is decided alike up to rounding
        near = any(abs(float(sum(fr[g * group:(g + 1) * group], Fraction(0)) - theta / G)) < 1e-12
                   for g in range(G))
        if not near:
            assert (t, mu) == (t_b, mu_b), trial
            assert tuple(anc) == anc_b, trial
            with np.errstate(divide="ignore"):
                assert np.allclose(np.exp(lws), [float(x) for x in ws_b], rtol=1e-12, atol=0)


def test_arna_equals_rna_with_a_fixed_exchange_and_the_index_ring(orc):
    rng = np.random.default_rng(2)
    for n, group, moved in ((4096, 256, 25), (1024, 4, 1), (600, 60, 30)):
        w = rng.gamma(0.3, 1.0, n)
        w[: group] = 0.0  # an empty group keeps the identity map
        w /= w.sum()
        ug = rng.random(n // group)
        a0, g0, s0 = orc.resample_rna(w, group, moved, ug)
        a1, g1, s1, t, mu = orc.resample_arna(w, group, moved, moved, 0.5, ug,
                                              np.arange(n // group))
        assert mu == moved
        assert np.array_equal(a0, a1)
        assert np.array_equal(g0, g1) and np.array_equal(s0, s1)


def test_exchange_size_hand_worked(orc):
    # G = 8 groups of 10; groups 2 and 5 hold all the weight: G_t = 2 at any
    # theta <= 4, so mu = 1 + floor((5 - 1) * 6 / 8) = 4
    n, group = 80, 10
    w = np.zeros(n)
    w[20:30] = 0.05
    w[50:60] = 0.05
    ug = np.full(8, 0.5)
    anc, lwg, lws, t, mu = orc.resample_arna(w, group, 1, 5, 0.5, ug, np.arange(8))
    assert (t, mu) == (2, 4)
    # every group tracking: the least exchange
    w = np.full(n, 1.0 / n)
    assert orc.resample_arna(w, group, 1, 5, 0.5, ug, np.arange(8))[3:] == (8, 1)
    # one group holding all the weight (at least one group always tracks: the
    # largest share is at least 1/G): mu = 1 + floor(4 * 7 / 8) = 4
    w = np.zeros(n)
    w[3] = 1.0
    assert orc.resample_arna(w, group, 1, 5, 1.0, ug, np.arange(8))[3:] == (1, 4)


def test_arna_routes_along_the_ring_and_keeps_the_weight(orc):
    rng = np.random.default_rng(9)
    n, group = 64 * 37, 64
    G = n // group
    w = rng.gamma(0.5, 1.0, n)
    w /= w.sum()
    ug = rng.random(G)
    order = orc.ring_order(orc.Model(), 13, G)
    anc, lwg, lws, t, mu = orc.resample_arna(w, group, 3, 20, 0.7, ug, order)
    assert 3 <= mu <= 20
    pos = np.empty(G, dtype=np.int64)
    pos[order] = np.arange(G)
    pred = order[(pos - 1) % G]
    for g in range(G):
        own = anc[g * group: (g + 1) * group - mu]
        tail = anc[(g + 1) * group - mu: (g + 1) * group]
        assert np.all(own // group == g)
        assert np.all(tail // group == pred[g])
    # the slot weights of all groups still sum to one: the ring is a permutation
    assert math.isclose(math.fsum(np.exp(lws)), 1.0, rel_tol=1e-12)
    assert t == int(np.sum(w.reshape(G, group).sum(1) >= 0.7 / G))


def test_lost_test_closed_form(orc):
    """Noise-free frames: a particle exactly on the spot fits with residual 0,
    so its log-likelihood is -P^2 log(sigma sqrt(2 pi)); on a frame without
    the spot the same particle leaves I^2 sum g^2 / (2 sigma^2) unexplained, a
    drop far beyond kappa P: lost. The threshold is strict."""
    W = H = 64
    s, I, b, sig = 1.5, 30.0, 10.0, 3.0
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    x0, y0 = 31.0, 30.0
    g = np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / (2 * s * s))
    frame = (b + I * g).astype(np.float32)
    blank = np.full((H, W), b, dtype=np.float32)
    m = orc.Model(n=1, width=W, height=H, s=s, b=b, sigma=sig, resample=2, arna_lost=3.0)
    P = m.P
    x = np.array([[x0], [y0], [0.0], [0.0], [I]])
    l_on = orc.loglik(m, frame, x)[0]
    lognorm = P * P * math.log(sig * math.sqrt(2 * math.pi))
    assert abs(l_on + lognorm) < 1e-9
    l_off = orc.loglik(m, blank, x)[0]
    h = (P - 1) // 2
    patch = g[30 - h:30 + h + 1, 31 - h:31 + h + 1]
    assert math.isclose(l_on - l_off, I * I * (patch ** 2).sum() / (2 * sig * sig), rel_tol=1e-9)
    assert not orc.arna_lost(m, l_on, -math.inf)  # the first frame has no reference
    assert not orc.arna_lost(m, l_on, l_on)
    assert orc.arna_lost(m, l_off, l_on)
    thr = l_on - 3.0 * P
    assert not orc.arna_lost(m, thr, l_on) and orc.arna_lost(m, np.nextafter(thr, -np.inf), l_on)


def test_arna_run_equals_rna_when_nothing_adapts(orc):
    mv = synth.render_movie(128, 128, 6, intensity=30.0, sigma=1.5, seed=6,
                            start_box=(32, 96, 32, 96))
    kw = dict(n=4096, init_a=(32, 32, -1, -1, 15), init_b=(96, 96, 1, 1, 45), rna_group=256,
              rna_exchange=0.1, ess_threshold=2048.0)
    r0 = orc.run(orc.Model(resample=1, **kw), mv.frames)
    r1 = orc.run(orc.Model(resample=2, arna_min=0.1, arna_lost=math.inf, **kw), mv.frames)
    assert np.array_equal(r0.mean, r1.mean) and np.array_equal(r0.anc, r1.anc)
    assert np.array_equal(r0.ess, r1.ess) and np.array_equal(r0.delta, r1.delta)
    assert np.all(r1.extra["arna"][:, 0] == 0)


def test_arna_run_redraws_the_ring_when_the_object_is_lost(orc):
    """A movie whose spot vanishes at frame 4: that frame's increment drops,
    the ring key becomes 4 and stays (the following frames are explained as
    well as before, by particles whose intensity has fallen, so none is lost
    again); the exchange stays within its bounds."""
    mv = synth.render_movie(128, 128, 8, intensity=30.0, sigma=1.5, seed=6,
                            start_box=(48, 80, 48, 80))
    frames = mv.frames.copy()
    rng = np.random.default_rng(0)
    for k in (3, 4):  # frames 4 and 5: background and noise only
        frames[k] = (10.0 + 3.0 * rng.standard_normal(frames[k].shape)).astype(np.float32)
    m = orc.Model(n=1 << 14, resample=2, rna_group=256, rna_exchange=0.5, arna_min=0.05,
                  init_a=(40, 40, -1, -1, 15), init_b=(88, 88, 1, 1, 45))
    r = orc.run(m, frames)
    keys = r.extra["arna"][:, 0]
    ref, lost = -math.inf, []
    for d in r.delta:
        lost.append(orc.arna_lost(m, d, ref))
        if not lost[-1]:
            ref = d
    assert lost == [False, False, False, True, False, False, False, False]
    assert list(keys) == [0, 0, 0, 4, 4, 4, 4, 4]
    mu = r.extra["arna"][:, 2]
    assert np.all((mu >= m.arna_mu_min) & (mu <= m.rna_moved))
    # the ring of key 4 differs from the index ring
    assert not np.array_equal(orc.ring_order(m, 4, 64), np.arange(64))
