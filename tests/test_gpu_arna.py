"""GPU parity of ARNA (adaptive RNA, Section 6.4; the reading is in the
oracle's pins, tests/test_oracle_arna.py) against the FP64 oracle,
teacher-forced per step: propagation and weights as for every scheme, then
the lost test on the GPU's own log-likelihood increments, the ring key, and
the oracle's ARNA resampling of the GPU's weights with that ring (tracking
count, slots exchanged, ancestors to the band rule)."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_5045_amd import synth

from parity import check_arna, check_propagate, check_weights, pair, snapshot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


def vanishing_spot_movie(T=8, W=128, blank=(3, 4)):
    """A spot that vanishes for frames 4 and 5 (noise and background only)."""
    mv = synth.render_movie(W, W, T, intensity=30.0, sigma=1.5, seed=6,
                            start_box=(48, 80, 48, 80))
    frames = mv.frames.copy()
    rng = np.random.default_rng(0)
    for k in blank:
        frames[k] = (10.0 + 3.0 * rng.standard_normal(frames[k].shape)).astype(np.float32)
    return frames


def run_arna_teacher_forced(ppf, p, m, frames, T):
    f = ppf.Filter(p)
    n = m.n
    obs = torch.from_numpy(frames).cuda()
    prev, _ = snapshot(f, n, np.full(n, -math.log(n)))
    ref, key, rep = -math.inf, 0, []
    for k in range(1, T + 1):
        f.step(obs[k - 1])
        cur, st = snapshot(f, n, None)
        ar = f.arna_state()
        check_propagate(m, k, prev, cur.x)
        check_weights(m, frames[k - 1], prev.lw_next, cur.x, cur.lw, st)
        # the lost test on the GPU's increments (a decision within 1e-6 of
        # the threshold may go either way)
        thr = ref - float(np.float32(m.arna_lost)) * m.P
        if abs(st["delta"] - thr) > 1e-6:
            assert ar["lost"] == (st["delta"] < thr), (k, st["delta"], thr)
        if ar["lost"]:
            key = k
        else:
            ref = st["delta"]
        assert ar["ring_key"] == key, (k, ar, key)
        if cur.resampled:
            nm, lws = check_arna(m, k, np.exp(cur.lw), cur.anc, ar, key)
            cur.lw_next = lws
        else:
            assert np.array_equal(cur.anc, np.arange(n))
            cur.lw_next = cur.lw.copy()
            nm = 0
        rep.append((k, ar["lost"], ar["ring_key"], ar["tracking"], ar["moved"], nm))
        prev = cur
    f.close()
    print(rep, flush=True)
    return rep


ARNA = dict(width=128, height=128, s=1.5, b=10.0, sigma=3.0, resample=3, rna_group=256,
            rna_exchange=0.5, arna_min=0.05, init_a=(40, 40, -1, -1, 15),
            init_b=(88, 88, 1, 1, 45))


def test_arna_redraws_the_ring_when_the_object_is_lost(ppf):
    frames = vanishing_spot_movie()
    p, m = pair(ppf, n=1 << 14, **ARNA)
    rep = run_arna_teacher_forced(ppf, p, m, frames, 8)
    assert any(r[1] for r in rep) and rep[-1][2] > 0  # a loss, and a keyed ring after it
    assert len({r[4] for r in rep}) > 1  # the exchange adapted


@pytest.mark.parametrize("n,group,thr", [(5000, 100, 2500.0), (4096, 64, math.inf)])
def test_arna_ragged_groups_and_ess_threshold(ppf, n, group, thr):
    frames = vanishing_spot_movie(T=6, blank=(2,))
    p, m = pair(ppf, n=n, ess_threshold=thr, **dict(ARNA, rna_group=group, arna_track=0.8))
    run_arna_teacher_forced(ppf, p, m, frames, 6)


def test_arna_without_adaptation_is_rna(ppf):
    """arna_min = rna_exchange and a lost test that never fires: the GPU's
    ARNA and RNA filters agree bit for bit."""
    mv = synth.render_movie(128, 128, 6, intensity=30.0, sigma=1.5, seed=6,
                            start_box=(32, 96, 32, 96))
    kw = dict(n_particles=4096, width=128, height=128, init_a=(32, 32, -1, -1, 15),
              init_b=(96, 96, 1, 1, 45), rna_group=256, rna_exchange=0.1, ess_threshold=2048.0)
    fa = ppf.Filter(ppf.params(resample=3, arna_min=0.1, arna_lost=math.inf, **kw))
    fr = ppf.Filter(ppf.params(resample=1, **kw))
    obs = torch.from_numpy(mv.frames).cuda()
    for k in range(6):
        fa.step(obs[k])
        fr.step(obs[k])
        for u, v in zip(fa.particles(), fr.particles()):
            assert np.array_equal(u, v), k
        assert fa.stats()["cum"] == fr.stats()["cum"]
        assert fa.arna_state()["ring_key"] == 0
    fa.close()
    fr.close()


def test_arna_c2size(ppf):
    """2^20 particles on 512 x 512 frames in 4096 groups of 256, resampling
    when ESS < N/2, the spot gone for frame 5 (a loss: the ring of 4096
    groups is redrawn): every particle checked, ten frames."""
    W = 512
    mv = synth.render_movie(W, W, 10, intensity=30.0, sigma=1.5, background=10.0, noise_sd=3.0,
                            seed=1)
    frames = mv.frames.copy()
    rng = np.random.default_rng(1)
    frames[4] = (10.0 + 3.0 * rng.standard_normal(frames[4].shape)).astype(np.float32)
    n = 1 << 20
    # a 64 px box around the spot's start, and a lost test at 0.8 P: at this
    # size the groups hold the spot loosely (ESS 1-80), so the blank frame's
    # increment drops by about 14, under the default 3 P = 27
    x0, y0 = mv.truth[0, 0]
    p, m = pair(ppf, n=n, width=W, height=W, s=1.5, b=10.0, sigma=3.0, init_kind=0,
                init_a=(x0 - 32, y0 - 32, -1, -1, 15), init_b=(x0 + 32, y0 + 32, 1, 1, 45),
                ess_threshold=float(n // 2), resample=3, rna_group=256, rna_exchange=0.5,
                arna_min=0.05, arna_lost=0.8, seed=1)
    assert n // m.rna_group == 4096
    rep = run_arna_teacher_forced(ppf, p, m, frames, 10)
    assert any(r[1] for r in rep)
