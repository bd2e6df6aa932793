"""Pins of the oracle's initialisation, dynamics, likelihood and
normalisation (CPU only). Each check uses a property the paper's definitions
or plain mathematics fix, not a retyped copy of the oracle's formula."""
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_1310_5045_amd import synth


def model(orc, **kw):
    return orc.Model(**kw)


# ------------------------------------------------------------------ init
def test_uniform_init_in_box_and_weights(orc):
    m = model(orc, n=20000, init_a=(10, 20, -1, -2, 5), init_b=(30, 25, 1, 2, 15))
    x, lw = orc.init(m)
    for d in range(5):
        assert x[d].min() >= m.init_a[d] and x[d].max() < m.init_b[d]
        assert stats.kstest((x[d] - m.init_a[d]) / (m.init_b[d] - m.init_a[d]), "uniform").pvalue > 1e-3
    assert np.all(lw == -math.log(m.n))
    # components come from distinct random words: near-zero correlation
    c = np.corrcoef(x)
    assert np.abs(c - np.eye(5)).max() < 0.05


def test_stratified_init_cells_and_marginals(orc):
    n = 4096 * 3 + 5
    m = model(orc, n=n, init_kind=2, init_a=(10, 20, -1, -2, 5), init_b=(74, 52, 1, 2, 15))
    x, lw = orc.init(m)
    t = int(math.floor(math.log2(n))) - 2
    ax, ay = (t + 1) // 2, t // 2
    # every (x, y) cell of the 2^ax x 2^ay grid holds floor/ceil(n / 2^t) particles
    cx = np.floor((x[0] - 10) / 64 * 2**ax).astype(int)
    cy = np.floor((x[1] - 20) / 32 * 2**ay).astype(int)
    counts = np.bincount(cx * 2**ay + cy, minlength=2**t)
    assert counts.min() >= n // 2**t and counts.max() <= -(-n // 2**t)
    for d in range(5):
        assert x[d].min() >= m.init_a[d] and x[d].max() < m.init_b[d]
        assert stats.kstest((x[d] - m.init_a[d]) / (m.init_b[d] - m.init_a[d]), "uniform").pvalue > 1e-3
    # locality: 256 consecutive particles cover a small part of the box
    span = [np.ptp(x[0][j:j + 256]) * np.ptp(x[1][j:j + 256]) for j in range(0, n - 256, 256)]
    assert np.median(span) < 64 * 32 * 0.1  # i.i.d. draws would span nearly all of it
    assert np.all(lw == -math.log(n))


def test_gaussian_init_moments(orc):
    m = model(orc, n=40000, init_kind=1, init_a=(1, 2, 3, 4, 5), init_b=(0.5, 1, 2, 3, 4))
    x, _ = orc.init(m)
    for d in range(5):
        z = (x[d] - m.init_a[d]) / m.init_b[d]
        assert stats.kstest(z, "norm").pvalue > 1e-3


# -------------------------------------------------------------- dynamics
def test_propagate_zero_noise_is_exact_ncv(orc):
    n = 1000
    m = model(orc, n=n, q=(0, 0, 0, 0, 0))
    rng = np.random.default_rng(0)
    xp = rng.normal(size=(5, n)) * 10
    parent = np.sort(rng.integers(0, n, n)).astype(np.int32)
    xn = orc.propagate(m, 3, xp, parent)
    p = xp[:, parent]
    assert np.array_equal(xn[0], p[0] + p[2])
    assert np.array_equal(xn[1], p[1] + p[3])
    assert np.array_equal(xn[2:], p[2:])
    assert np.array_equal(orc.propagate(m, 3, xp, None)[0], xp[0] + xp[2])


def test_propagate_noise_is_independent_standard_normal(orc):
    n = 20000
    q = (0.5, 0.25, 0.1, 0.2, 1.0)
    m = model(orc, n=n, q=q)
    xn = orc.propagate(m, 5, np.zeros((5, n)))
    qf = np.asarray(q, dtype=np.float32).astype(np.float64)
    z = xn / qf[:, None]
    for d in range(5):
        assert stats.kstest(z[d], "norm").pvalue > 1e-3
    assert np.abs(np.corrcoef(z) - np.eye(5)).max() < 0.04
    # a different frame index gives fresh noise, the same index repeats it
    assert np.array_equal(orc.propagate(m, 5, np.zeros((5, n))), xn)
    assert abs(np.corrcoef(orc.propagate(m, 6, np.zeros((5, n)))[0], xn[0])[0, 1]) < 0.05


# ------------------------------------------------------------ likelihood
def _frame_with_spot(W, H, x0, y0, I, s, b):
    """A noiseless frame: Eq. 3 rendered by the input generator's own code."""
    mv = synth.render_movie(W, H, 1, intensity=I, sigma=s, background=b, noise_sd=0.0,
                            vmax=0.0, jitter=0.0, start_box=(x0, x0, y0, y0), seed=0)
    return mv.frames[0]


def test_likelihood_noiseless_spot_has_zero_residual(orc):
    s, b, sig, I = 1.5, 10.0, 3.0, 30.0
    frame = _frame_with_spot(64, 48, 20.25, 30.75, I, s, b)
    m = model(orc, n=1, width=64, height=48, s=s, b=b, sigma=sig)
    x = np.array([[20.25], [30.75], [0.0], [0.0], [I]])
    ll = orc.loglik(m, frame, x)[0]
    const = -(m.P ** 2) * math.log(sig * math.sqrt(2 * math.pi))
    # the frame is stored in fp32: residuals of ~1e-6 per pixel remain
    assert abs(ll - const) < 1e-9 * abs(const) + 1e-8
    # moving the particle off the spot lowers the likelihood
    x2 = x.copy()
    x2[0] += 0.5
    assert orc.loglik(m, frame, x2)[0] < ll - 1.0


def test_likelihood_layout_is_row_major_y_x(orc):
    s, b, I = 1.5, 10.0, 30.0
    frame = _frame_with_spot(64, 64, 15.0, 40.0, I, s, b)
    m = model(orc, n=2, width=64, height=64, s=s, b=b)
    x = np.array([[15.0, 40.0], [40.0, 15.0], [0, 0], [0, 0], [I, I]])
    ll = orc.loglik(m, frame, x)
    assert ll[0] > ll[1] + 100


def test_likelihood_far_outside_frame_is_separable_sum(orc):
    # all pixels of the patch outside the frame: Z - b := 0, so the residual
    # is -I g, and sum g^2 factorises into two 1-D sums
    s, sig, I = 1.7, 2.5, 12.0
    m = model(orc, n=3, width=32, height=32, s=s, sigma=sig)
    xs = np.array([-50.3, 1e4 + 0.2, 77.45])
    ys = np.array([12.1, -300.4, 5000.0])
    x = np.array([xs, ys, [0] * 3, [0] * 3, [I] * 3], dtype=np.float64)
    ll = orc.loglik(m, np.zeros((32, 32), np.float32), x)
    sf, sgf, If = (float(np.float32(v)) for v in (s, sig, I))
    h = (m.P - 1) // 2
    for i in range(3):
        fx = xs[i] - math.floor(xs[i] + 0.5)
        fy = ys[i] - math.floor(ys[i] + 0.5)
        gx2 = math.fsum(math.exp(-((d - fx) ** 2) / sf**2) for d in range(-h, h + 1))
        gy2 = math.fsum(math.exp(-((d - fy) ** 2) / sf**2) for d in range(-h, h + 1))
        expect = -If * If * gx2 * gy2 / (2 * sgf**2) - m.P**2 * math.log(sgf * math.sqrt(2 * math.pi))
        assert math.isclose(ll[i], expect, rel_tol=1e-12)


def test_likelihood_constant_frame_no_spot(orc):
    m = model(orc, n=1, width=40, height=40, s=2.0, b=10.0, sigma=3.0)
    frame = np.full((40, 40), 14.0, np.float32)  # Z - b = 4 everywhere
    x = np.array([[20.3], [19.6], [0], [0], [0.0]])
    ll = orc.loglik(m, frame, x)[0]
    P = m.P
    assert P == 13
    assert math.isclose(ll, -P * P * 16.0 / 18.0 - P * P * math.log(3 * math.sqrt(2 * math.pi)),
                        rel_tol=1e-14)


def test_likelihood_translation_invariant_and_border_reading(orc):
    rng = np.random.default_rng(1)
    m = model(orc, n=1, width=50, height=50, s=1.5, b=10.0)
    frame = (10 + 3 * rng.standard_normal((50, 50))).astype(np.float32)
    x = np.array([[20.3], [30.1], [0], [0], [25.0]])
    ll = orc.loglik(m, frame, x)[0]
    # shift content and particle by (+3, -2)
    sh = np.full((50, 50), 10.0, np.float32)
    sh[:48, 3:] = frame[2:, :47]
    xs = x.copy()
    xs[0] += 3
    xs[1] -= 2
    assert math.isclose(orc.loglik(m, sh, xs)[0], ll, rel_tol=1e-13)
    # a particle on the border sees background (Z - b = 0) outside the frame:
    # the same as a larger frame padded with b
    xb = np.array([[1.2], [48.6], [0], [0], [25.0]])
    big = np.full((60, 60), 10.0, np.float32)
    big[5:55, 5:55] = frame
    mb = model(orc, n=1, width=60, height=60, s=1.5, b=10.0)
    xbb = xb.copy()
    xbb[0] += 5
    xbb[1] += 5
    assert math.isclose(orc.loglik(m, frame, xb)[0], orc.loglik(mb, big, xbb)[0], rel_tol=1e-13)


def test_linear_gaussian_likelihood(orc):
    m = model(orc, n=4, obs_model=1, lg_r=(0.5, 2.0, 1.5))
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 4))
    z = np.array([0.3, -0.7, 1.1], np.float32)
    ll = orc.loglik(m, z, x)
    r = np.asarray(m.lg_r, np.float32).astype(np.float64)
    expect = (stats.norm.logpdf(z[0], x[0], r[0]) + stats.norm.logpdf(z[1], x[1], r[1])
              + stats.norm.logpdf(z[2], x[4], r[2]))
    assert np.allclose(ll, expect, rtol=1e-13)


# --------------------------------------------------------- normalisation
def test_normalize_special_cases(orc):
    w, st = orc.normalize(np.full(1000, -3.7))
    assert np.allclose(w, 1e-3, rtol=1e-14)
    assert math.isclose(st["ess"], 1000.0, rel_tol=1e-12)
    assert math.isclose(st["delta"], -3.7 + math.log(1000), rel_tol=1e-14)
    l = np.full(50, -np.inf)
    l[17] = 2.5
    w, st = orc.normalize(l)
    assert w[17] == 1.0 and w.sum() == 1.0 and st["ess"] == 1.0 and st["delta"] == 2.5
    with pytest.raises(FloatingPointError):
        orc.normalize(np.full(10, -np.inf))
    l = np.zeros(10)
    l[3] = np.nan
    with pytest.raises(FloatingPointError):
        orc.normalize(l)


def test_normalize_matches_exact_sums(orc):
    rng = np.random.default_rng(4)
    l = rng.normal(-500, 20, 5000)
    w, st = orc.normalize(l)
    assert math.isclose(st["delta"], special.logsumexp(l), rel_tol=1e-14)
    assert math.isclose(math.fsum(w), 1.0, rel_tol=1e-13)
    ess = 1.0 / math.fsum(x * x for x in w)
    assert math.isclose(st["ess"], ess, rel_tol=1e-12)
    x = rng.normal(size=(5, 5000))
    assert np.allclose(orc.estimate(w, x), np.average(x, axis=1, weights=w), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("init_kind", [0, 1, 2, 3])
def test_indexed_entry_points_agree_with_whole_run(orc, init_kind):
    n = 3001
    m = model(orc, n=n, init_kind=init_kind, init_a=(0, 0, -1, -1, 15), init_b=(64, 32, 1, 1, 45))
    x, _ = orc.init(m)
    idx = np.array([0, 1, 255, 256, 2047, 2048, 3000, 1234])
    ms = model(orc, n=idx.size, init_kind=init_kind, init_a=m.init_a, init_b=m.init_b)
    assert np.array_equal(orc.init_indexed(ms, n, idx), x[:, idx])
    parent = np.sort(np.random.default_rng(0).integers(0, n, n)).astype(np.int32)
    xn = orc.propagate(m, 4, x, parent)
    assert np.array_equal(orc.propagate_indexed(ms, 4, idx, x[:, parent[idx]]), xn[:, idx])


# ------------------------------------------------- init kind 3 (Z-ordered uniform)
def test_zorder_key_hand_worked(orc):
    """The Morton key interleaves the top 16 bits of the x word (even bit
    positions) and of the y word (odd positions); the low 16 bits of each
    word do not enter."""
    assert orc.zorder_key(0xFFFF0000, 0) == 0x55555555
    assert orc.zorder_key(0, 0xFFFF0000) == 0xAAAAAAAA
    assert orc.zorder_key(0x00010000, 0) == 1
    assert orc.zorder_key(0, 0x00010000) == 2
    assert orc.zorder_key(0x80000000, 0x80000000) == 0xC0000000
    assert orc.zorder_key(0x0000FFFF, 0x0000FFFF) == 0
    assert orc.zorder_key(0x00030000, 0x00050000) == 0b100111  # x 011, y 101


def _morton16(x, y):
    k = 0
    for j in range(16):
        k |= ((x >> j) & 1) << (2 * j)
        k |= ((y >> j) & 1) << (2 * j + 1)
    return k


def test_zorder_init_is_the_uniform_cloud_in_key_order(orc):
    """Kind 3 equals kind 0's draws permuted: position j holds the draw
    whose key is j-th in the stable sort by key, the keys re-derived here
    from the generator's words with an interleave written independently."""
    n = 5000
    kw = dict(n=n, init_a=(0, 0, -1, -1, 15), init_b=(128, 96, 1, 1, 45), seed=11, track=3)
    x0, _ = orc.init(model(orc, init_kind=0, **kw))
    x3, lw3 = orc.init(model(orc, init_kind=3, **kw))
    assert np.allclose(lw3, -np.log(n), rtol=0, atol=1e-15)
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 2] = 1 << 24  # the init purpose, block 0
    ctr[:, 3] = 3
    words = orc.philox(11, ctr)
    keys = np.array([_morton16(int(a) >> 16, int(b) >> 16) for a, b in words[:, :2]],
                    dtype=np.int64)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(orc.zorder_perm(model(orc, init_kind=3, **kw), n), order)
    assert np.array_equal(x3, x0[:, order])
    # the order is spatial: keys non-decreasing, ties by draw index
    k_sorted = keys[order]
    assert np.all(np.diff(k_sorted) >= 0)
    ties = np.diff(k_sorted) == 0
    assert np.all(np.diff(order)[ties] > 0)
    # neighbours in the order are neighbours in space (cells of 1/256 of the box)
    step = np.hypot(np.diff(x3[0]) / 128, np.diff(x3[1]) / 96)
    assert np.median(step) < 0.05
