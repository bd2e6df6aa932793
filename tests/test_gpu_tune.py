"""Workgroup shapes of the step kernel and the autotuner that picks them:
tuning leaves the filter's state as it was and keeps a shape that a filter
set to it by hand reproduces bit for bit; batches under each shape candidate
equal single filters with the same shapes, bit for bit. (Each shape's
likelihood is checked against the oracle in test_gpu_parity.py.)"""
import numpy as np
import pytest

from paper_1310_5045_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H = 144, 128


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def frames():
    mv = synth.render_movie(W, H, 6, n_spots=4, intensity=(20.0, 40.0), sigma=(1.2, 2.4),
                            start_box=(30, 114, 30, 98), seed=13)
    return torch.from_numpy(mv.frames).cuda()


def fparams(ppf, n, s, **kw):
    return ppf.params(n_particles=n, width=W, height=H, psf_sigma=s, seed=6,
                      init_a=(30, 30, -1, -1, 15), init_b=(114, 98, 1, 1, 45), **kw)


def snapshot(f):
    x, lw, anc = f.particles()
    st = f.stats()
    return x, lw, anc, {k: st[k] for k in ("k", "resampled", "ess", "delta", "cum")}


def same(a, b):
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    assert a[3] == b[3]


@pytest.mark.parametrize("n,s", [(20000, 1.5), (7001, 2.0)])
def test_autotune_keeps_state_and_picks_a_shape(ppf, frames, n, s):
    p = fparams(ppf, n, s)
    f = ppf.Filter(p)
    for k in range(3):
        f.step(frames[k])
    before = snapshot(f)
    ms, chosen = f.autotune(frames[3], reps=3)
    assert len(ms) == ppf.NUM_SHAPES and all(t > 0 for t in ms) and chosen in (0, 1)
    assert ms[chosen] == min(ms)
    same(before, snapshot(f))
    # the same first steps (shape 0), then the chosen shape set by hand
    twin = ppf.Filter(p)
    for k in range(3):
        twin.step(frames[k])
    twin.set_shape(chosen)
    for k in (3, 4):
        f.step(frames[k])
        twin.step(frames[k])
        same(snapshot(f), snapshot(twin))
    f.close()
    twin.close()


def test_autotune_with_one_kernel(ppf, frames):
    f = ppf.Filter(fparams(ppf, 3000, 1.5, grad=1))
    f.step(frames[0])
    ms, chosen = f.autotune(frames[1], reps=2)
    assert len(ms) == 1 and chosen == 0
    f.close()


SIZES = [(1500, 1.2), (4000, 1.5), (2500, 2.0), (700, 2.4), (64, 1.3)]  # P 7, 9, 13, 15, 7


@pytest.mark.parametrize("cand", [0, 1, 2])
def test_batch_shapes_equal_single_filters(ppf, frames, cand):
    ps = [fparams(ppf, n, s, track_id=t) for t, (n, s) in enumerate(SIZES)]
    assert [ppf.patch_size(p) for p in ps] == [7, 9, 13, 15, 7]
    b = ppf.Batch(ps)
    b.set_shapes(cand)
    singles = []
    for p in ps:
        f = ppf.Filter(p)
        P = ppf.patch_size(p)
        f.set_shape({0: 0, 1: 1, 2: 1 if P < 13 else 0}[cand])
        singles.append(f)
    for k in range(4):
        b.step(frames[k])
        for f in singles:
            f.step(frames[k])
        bst = b.stats()
        for t, f in enumerate(singles):
            for u, v in zip(b.particles(t), f.particles()):
                assert np.array_equal(u, v), (cand, k, t)
            assert bst[t]["delta"] == f.stats()["delta"]
    b.close()
    for f in singles:
        f.close()


def test_batch_autotune(ppf, frames):
    ps = [fparams(ppf, n, s, track_id=t) for t, (n, s) in enumerate(SIZES)]
    b = ppf.Batch(ps)
    b.step(frames[0])
    before = [b.particles(t) for t in range(len(ps))]
    ms, chosen = b.autotune(frames[1], reps=3)
    assert len(ms) == 3 and all(t > 0 for t in ms) and ms[chosen] == min(ms)
    for t in range(len(ps)):
        for u, v in zip(before[t], b.particles(t)):
            assert np.array_equal(u, v)
    twin = ppf.Batch(ps)
    twin.step(frames[0])
    twin.set_shapes(chosen)
    for k in (1, 2):
        b.step(frames[k])
        twin.step(frames[k])
        for t in range(len(ps)):
            for u, v in zip(b.particles(t), twin.particles(t)):
                assert np.array_equal(u, v)
    b.close()
    twin.close()
