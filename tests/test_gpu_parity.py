"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (teacher-forced per step, see tests/parity.py)."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_5045_amd import synth

from parity import (PATH_BOXES, PATH_ORIGINS, GpuState, box_layout, check_propagate, check_rna,
                    check_step, check_systematic, check_weights, pair, snapshot)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


def run_teacher_forced(ppf, p, m, obs_np, T, rna=False, shape=0):
    f = ppf.Filter(p)
    f.set_shape(shape)
    n = m.n
    obs_t = torch.from_numpy(np.ascontiguousarray(obs_np)).cuda()
    prev, _ = snapshot(f, n, np.full(n, -math.log(n)))
    x0o, _ = oracle.init(m)
    # initial states: the GPU rounds the same fp64 value once to fp32
    assert np.all(np.abs(prev.x - x0o) <= np.spacing(np.abs(x0o).astype(np.float32)) + 1e-12)
    report = []
    for k in range(1, T + 1):
        f.step(obs_t[k - 1])
        cur, st = snapshot(f, n, None)
        report.append(check_step(m, k, prev, cur, st, obs_np[k - 1], rna))
        prev = cur
    f.close()
    return report


SPOT = dict(width=128, height=128, s=1.5, b=10.0, sigma=3.0, init_a=(32, 32, -1, -1, 15),
            init_b=(96, 96, 1, 1, 45))


@pytest.fixture(scope="module")
def movie128():
    return synth.render_movie(128, 128, 8, intensity=30.0, sigma=1.5, background=10.0, noise_sd=3.0,
                              start_box=(32, 96, 32, 96), seed=6)


def test_philox_bit_exact(ppf):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, (50000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:100, 1:] = 0
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        out = ppf.philox(seed, torch.from_numpy(ctr.view(np.int32)).cuda()).cpu().numpy()
        assert np.array_equal(out.view(np.uint32), oracle.philox(seed, ctr))


@pytest.mark.parametrize("init_kind", [0, 1, 2, 3])
def test_init_matches_oracle(ppf, init_kind):
    kw = dict(SPOT, n=5000, init_kind=init_kind)
    if init_kind == 1:
        kw.update(init_a=(64, 64, 0, 0, 30), init_b=(3, 3, 0.5, 0.5, 4))
    p, m = pair(ppf, **kw)
    f = ppf.Filter(p)
    x, lw, anc = f.particles()
    xo, lwo = oracle.init(m)
    tol = np.spacing(np.abs(xo).astype(np.float32)).astype(np.float64)
    if init_kind == 1:  # device fp64 log/sincos may differ from the host's by an ulp
        tol = tol + 1e-12 * np.abs(xo)
    assert np.all(np.abs(x - xo) <= tol)
    assert np.allclose(lw, lwo, rtol=1e-15)
    assert np.array_equal(anc, np.arange(5000))
    f.close()


def test_zorder_init_many_tiles(ppf):
    """The Z-ordered uniform cloud over many sort tiles and a ragged tail:
    every particle equals the oracle's, and a reset draws it again."""
    n = (1 << 20) + 37
    p, m = pair(ppf, **dict(SPOT, n=n, init_kind=3, init_a=(0, 0, -1, -1, 15),
                            init_b=(128, 128, 1, 1, 45)))
    f = ppf.Filter(p)
    x, _, _ = f.particles()
    xo, _ = oracle.init(m)
    assert np.all(np.abs(x - xo) <= np.spacing(np.abs(xo).astype(np.float32)))
    f.step(torch.from_numpy(np.full((128, 128), 10.0, np.float32)).cuda())
    f.reset()
    x2, _, _ = f.particles()
    assert np.array_equal(x, x2)
    f.close()


@pytest.mark.parametrize("n", [4096, 5000, 257])
def test_spot_systematic_every_step(ppf, movie128, n):
    p, m = pair(ppf, n=n, **SPOT)
    rep = run_teacher_forced(ppf, p, m, movie128.frames, 6)
    print(rep)
    assert all(r[3] == 0 for r in rep), rep  # no mismatch beyond the 1e-10 band


@pytest.mark.parametrize("n,s", [(5000, 1.5), (3001, 2.0)])
def test_spot_workgroup_shape_1(ppf, movie128, n, s):
    """The six-wave step kernel (1792-double tile) against the oracle."""
    p, m = pair(ppf, n=n, **dict(SPOT, s=s))
    rep = run_teacher_forced(ppf, p, m, movie128.frames, 5, shape=1)
    assert all(r[3] == 0 for r in rep), rep


def test_spot_stratified_patch13_ess_threshold(ppf):
    mv = synth.render_movie(160, 144, 5, intensity=30.0, sigma=2.0, seed=3)
    p, m = pair(ppf, n=6000, width=160, height=144, s=2.0, b=10.0, sigma=3.0, init_kind=2,
                init_a=(0, 0, -1, -1, 15), init_b=(160, 144, 1, 1, 45), ess_threshold=3000.0)
    assert m.P == 13
    run_teacher_forced(ppf, p, m, mv.frames, 5)


@pytest.mark.parametrize("P", [1, 3, 25])
def test_spot_patch_extremes(ppf, movie128, P):
    p, m = pair(ppf, n=3000, patch=P, **dict(SPOT, s=4.0 if P == 25 else 1.5))
    run_teacher_forced(ppf, p, m, movie128.frames, 3)


def test_spot_log_weights_beyond_2_20(ppf, movie128):
    """A tiny noise sigma (0.02) puts every block maximum of l below -2^20,
    where the block shift is the exact fp64 maximum instead of the fp32 one."""
    p, m = pair(ppf, n=3001, **dict(SPOT, sigma=0.02))
    assert oracle.loglik(m, movie128.frames[0], oracle.init(m)[0]).max() < -2.0**20
    run_teacher_forced(ppf, p, m, movie128.frames, 3)


def test_spot_particles_leaving_frame(ppf):
    # a wide init box: many patches cross the border or lie fully outside
    mv = synth.render_movie(48, 40, 3, seed=2, start_box=(10, 38, 10, 30))
    p, m = pair(ppf, n=4000, width=48, height=40, s=1.5, b=10.0, sigma=3.0,
                init_a=(-100, -80, -3, -3, 0), init_b=(150, 120, 3, 3, 40), q=(2, 2, 0.5, 0.5, 2))
    run_teacher_forced(ppf, p, m, mv.frames, 3)


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("P", [9, 11, 13])
@pytest.mark.parametrize("way", ["sum", "tab", "glob"])
def test_spot_tile_limits(ppf, shape, P, way):
    """Placed particles whose workgroup boxes sit at the limits of the LDS
    tile (the gradient tests' layouts: a small box, a tile filled to its last
    double in shape 0, a box just too large for it), weights flattened so
    that every particle counts; one step against the oracle's weights."""
    s = {9: 1.5, 11: 1.7, 13: 2.0}[P]
    W, H = 96, 80
    mv = synth.render_movie(W, H, 1, intensity=30.0, sigma=s, start_box=(40, 52, 34, 46), seed=8)
    n = 2 * 256 + 37
    p, m = pair(ppf, n=n, width=W, height=H, s=s, b=10.0, sigma=3.0, q=(1e-3,) * 5, seed=3)
    acx, acy = PATH_BOXES[P][way]
    x = box_layout(np.random.default_rng(P), n, acx, acy, *PATH_ORIGINS[way])
    a = -oracle.loglik(m, mv.frames[0], x.astype(np.float64))
    lw = a - a.max() - np.log(np.exp(a - a.max()).sum())
    f = ppf.Filter(p)
    f.set_shape(shape)
    f.set_particles(x, lw)
    f.step(torch.from_numpy(mv.frames[0]).cuda())
    cur, st = snapshot(f, n, None)
    check_propagate(m, 1, GpuState(x, lw, np.arange(n), False, lw), cur.x)
    check_weights(m, mv.frames[0], lw, cur.x, cur.lw, st)
    f.close()


def test_linear_gaussian_filter(ppf):
    LG = dict(obs_model=1, q=(0.5, 0.5, 0.3, 0.3, 1.0), lg_r=(2.0, 2.0, 4.0), init_kind=1,
              init_a=(50.0, 50.0, 0.5, -0.3, 30.0), init_b=(0.5, 0.5, 0.2, 0.2, 1.0))
    tr = synth.linear_gaussian_track(6, LG["init_a"], LG["init_b"], LG["q"], LG["lg_r"], seed=3)
    p, m = pair(ppf, n=4500, ess_threshold=2250.0, **LG)
    run_teacher_forced(ppf, p, m, tr.obs, 6)


def test_rna_filter(ppf, movie128):
    p, m = pair(ppf, n=4096, resample=1, rna_group=256, rna_exchange=0.1, ess_threshold=2048.0,
                **SPOT)
    rep = run_teacher_forced(ppf, p, m, movie128.frames, 6, rna=True)
    assert any(len(r) == 3 for r in rep)


def test_rna_small_groups_and_full_exchange(ppf, movie128):
    p, m = pair(ppf, n=4096, resample=1, rna_group=64, rna_exchange=0.5, **SPOT)
    run_teacher_forced(ppf, p, m, movie128.frames, 4, rna=True)


# ------------------------------------------------- standalone resamplers
def test_systematic_standalone_brute_force(ppf):
    from fractions import Fraction
    from oracle import brute
    rng = np.random.default_rng(1)
    for n in range(1, 9):
        for _ in range(4):
            k = rng.integers(1, 64, n)
            k[rng.random(n) < 0.25] = 0
            if k.sum() == 0:
                k[0] = 1
            fr = [Fraction(int(v), int(k.sum())) for v in k]
            with np.errstate(divide="ignore"):
                lw = torch.tensor(np.log(k / k.sum()).astype(np.float32)).cuda()
            for lo, hi, anc in brute.systematic_pieces(fr):
                if hi - lo < Fraction(1, 10**5):
                    continue  # pieces thinner than the fp32 weight rounding
                u = float((lo + hi) / 2)
                got = ppf.resample_systematic(lw, u).cpu().numpy()
                assert tuple(got) == anc, (n, k, u, got, anc)


@pytest.mark.parametrize("n,kind", [(1, "flat"), (2047, "flat"), (2049, "exp"), (100_000, "exp"),
                                    (1 << 20, "onehot"), (1 << 20, "one_tile"), (300_001, "zeros"),
                                    ((1 << 24) + 77, "onehot")])
def test_systematic_standalone_vs_oracle(ppf, n, kind):
    rng = np.random.default_rng(n)
    if kind == "flat":
        l = np.zeros(n)
    elif kind == "exp":
        l = rng.normal(0, 3, n)
    elif kind == "onehot":
        l = np.full(n, -np.inf)
        l[n // 3] = 0.0
    elif kind == "one_tile":  # nearly all weight on 1000 particles of two segments: the heavy pass
        l = rng.normal(-60, 1, n)
        l[500_000:501_000] = rng.normal(0, 1, 1000)
    else:
        l = rng.normal(0, 1, n)
        l[rng.random(n) < 0.5] = -np.inf
    l32 = l.astype(np.float32)
    for u in (0.0, 0.123456789, 0.999):
        anc = ppf.resample_systematic(torch.from_numpy(l32).cuda(), u).cpu().numpy()
        w = np.exp(l32.astype(np.float64) - l32.max())
        w /= w.sum()
        nm, nm10 = check_systematic(w, u, anc)
        assert nm10 == 0
        o = np.bincount(anc, minlength=n)
        assert o.sum() == n and np.all(o[w == 0] == 0)


@pytest.mark.parametrize("slots", [2048, 3900, 4100, 6200, 9000])
def test_systematic_heavy_segments_around_the_queue_limit(ppf, slots):
    """Segments of 1024 particles whose slots span just under, at and over the
    four tiles one wave writes itself (more go to the queued fill in chunks of
    two tiles: odd and even chunk counts), two such segments side by side, and
    a heavy ragged last segment; ancestors against the oracle (band rule)."""
    S = 1024
    n = 64 * S + 517
    rng = np.random.default_rng(slots)
    heavy = [5, 6, n // S]  # two neighbours and the ragged last segment
    l = rng.normal(0.0, 1.0, n)
    w_rest = np.exp(l).sum()
    for s in heavy:
        lo, hi = s * S, min(n, (s + 1) * S)
        # this segment's weight for about `slots` of the n slots
        a = slots / n * w_rest / (1.0 - len(heavy) * slots / n) / (hi - lo)
        l[lo:hi] = np.log(a) + rng.normal(0.0, 0.3, hi - lo) - 0.045
    l32 = l.astype(np.float32)
    spans = set()
    for u in (0.0, 0.37, 0.999):
        anc = ppf.resample_systematic(torch.from_numpy(l32).cuda(), u).cpu().numpy()
        w = np.exp(l32.astype(np.float64) - l32.max())
        w /= w.sum()
        nm, nm10 = check_systematic(w, u, anc)
        assert nm10 == 0
        assert np.bincount(anc, minlength=n).sum() == n
        # tiles each heavy segment's slots span (tiles start on 4 slots)
        for s in heavy:
            idx = np.nonzero((anc >= s * S) & (anc < (s + 1) * S))[0]
            fs, fe = int(idx.min()), int(idx.max()) + 1
            spans.add(-(-(fe - (fs & ~3)) // S))
    # the case exercises the wave's own limit (3900: four tiles) or the queue
    assert (max(spans) <= 4) == (slots < 4000), spans


def test_rna_standalone_vs_oracle(ppf):
    rng = np.random.default_rng(7)
    for n, group, moved in ((4096, 256, 25), (1024, 4, 1), (8192, 1024, 512), (512, 512, 0)):
        l = rng.normal(0, 2, n).astype(np.float32)
        if n > group:
            l[: group] = -np.inf  # an empty group keeps the identity map
        ug = rng.random(n // group)
        anc, lwg = ppf.resample_rna(torch.from_numpy(l).cuda(), group, moved,
                                    torch.from_numpy(ug).cuda())
        w = np.exp(l.astype(np.float64) - l.max())
        w /= w.sum()
        check_rna(w, group, moved, ug, anc.cpu().numpy())
        W = w.reshape(-1, group).sum(1)
        with np.errstate(divide="ignore"):
            assert np.allclose(lwg.cpu().numpy(), np.log(W / group), rtol=1e-12)


# ------------------------------------------------------------- conventions
def test_nan_frame_rolls_back(ppf, movie128):
    p, m = pair(ppf, n=4096, **SPOT)
    f = ppf.Filter(p)
    fr = torch.from_numpy(movie128.frames).cuda()
    f.step(fr[0])
    x1, lw1, anc1 = f.particles()
    s1 = f.stats()
    f.step(torch.full_like(fr[1], float("nan")))
    with pytest.raises(ppf.PPFError) as e:
        f.sync()
    assert e.value.code == ppf.PPF_ENUMERIC
    x2, lw2, anc2 = f.particles()
    s2 = f.stats()
    assert s2["k"] == s1["k"] == 1
    assert np.array_equal(x1, x2) and np.array_equal(lw1, lw2) and np.array_equal(anc1, anc2)
    f.sync()  # the report was cleared
    f.step(fr[1])  # and the filter continues from the rolled-back state
    assert f.stats()["k"] == 2
    f.close()


def test_set_particles_and_gather(ppf, movie128):
    p, m = pair(ppf, n=3000, **SPOT)
    f = ppf.Filter(p)
    rng = np.random.default_rng(2)
    x = np.stack([rng.uniform(40, 80, 3000), rng.uniform(40, 80, 3000), rng.normal(0, 1, 3000),
                  rng.normal(0, 1, 3000), rng.uniform(20, 40, 3000)]).astype(np.float32)
    lw = rng.normal(0, 1, 3000)
    lw -= np.log(np.exp(lw).sum())
    f.set_particles(x, lw)
    x2, lw2, anc2 = f.particles()
    assert np.array_equal(x2, x) and np.array_equal(lw2, lw)
    fr = torch.from_numpy(movie128.frames).cuda()
    f.step(fr[0])
    cur, st = snapshot(f, 3000, None)
    check_propagate(m, 1, GpuState(x, lw, anc2, False, lw), cur.x)
    check_weights(m, movie128.frames[0], lw, cur.x, cur.lw, st)
    g = f.gather().cpu().numpy()
    assert np.array_equal(g, cur.x[:, cur.anc])
    f.close()


def test_normals_accuracy(ppf, movie128):
    """From zero states with unit process noise the propagated state is the
    five normals themselves: compare 5 x 2^20 of them with the oracle's fp64
    Box-Muller. Bound: the fp32 radius is within about 2 ulp (hardware log2
    and root), sin/cos(2 pi t) within 9e-8 absolute, so |dz| <= 2.5e-7 |z|
    + 5.2e-7 (the absolute part scaled by the radius, at most 5.8)."""
    n = 1 << 20
    p, m = pair(ppf, n=n, q=(1, 1, 1, 1, 1), **SPOT)
    f = ppf.Filter(p)
    f.set_particles(np.zeros((5, n), np.float32), np.full(n, -math.log(n)))
    f.step(torch.from_numpy(movie128.frames[0]).cuda())
    z_gpu = f.particles()[0].astype(np.float64)
    z = oracle.propagate(m, 1, np.zeros((5, n)))
    err = np.abs(z_gpu - z)
    assert np.all(err <= 3e-7 * np.abs(z) + 6e-7), err.max()
    print("normals: max error", err.max(), "relative", (err / np.maximum(np.abs(z), 1)).max())
    f.close()


def test_free_running_matches_until_first_flip(ppf, movie128):
    p, m = pair(ppf, n=4096, **SPOT)
    f = ppf.Filter(p)
    fr = torch.from_numpy(movie128.frames).cuda()
    r = oracle.run(m, movie128.frames, 8)
    for k in range(1, 9):
        f.step(fr[k - 1])
        st = f.stats()
        if abs(st["mean"][0] - r.mean[k - 1, 0]) > 1e-3:
            break
        assert np.abs(st["mean"] - r.mean[k - 1]).max() < 1e-3
    assert k >= 2  # at least the first frame agrees free-running
    f.close()
