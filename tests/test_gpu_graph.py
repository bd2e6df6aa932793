"""Graph mode: a step recorded once into a HIP graph and replayed, pointed at
each call's frame, gives bit for bit what the same step's launches give. Each
replay is checked against an eagerly stepped twin, with host work and
synchronisation between the replays, and the frames alternate between device
buffers so that the frame argument really changes."""
import math

import numpy as np
import pytest

from paper_1310_5045_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H = 128, 112
BASE = dict(width=W, height=H, psf_sigma=1.5, background=10.0, noise_sigma=3.0,
            init_a=(40, 36, -1, -1, 15), init_b=(88, 76, 1, 1, 45), seed=4)


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def frames():
    mv = synth.render_movie(W, H, 7, intensity=30.0, sigma=1.5, start_box=(48, 80, 44, 68), seed=9)
    # two copies in separate buffers: step k reads copy k % 2
    return [torch.from_numpy(mv.frames).cuda(), torch.from_numpy(mv.frames.copy()).cuda()]


def same_filter(a, b):
    for u, v in zip(a.particles(), b.particles()):
        assert np.array_equal(u, v)
    sa, sb = a.stats(), b.stats()
    for key in ("k", "resampled", "rolled_back", "ess", "delta", "cum"):
        assert sa[key] == sb[key] or (math.isnan(sa[key]) and math.isnan(sb[key])), key
    assert np.array_equal(sa["mean"], sb["mean"])


@pytest.mark.parametrize("extra", [
    dict(n_particles=5000),
    dict(n_particles=4096, ess_threshold=2000.0),
    dict(n_particles=2048, resample=1, rna_group=256, rna_exchange=0.1),
    dict(n_particles=4096, resample=2, rna_group=256, dlb=1),
    dict(n_particles=1 << 16, resample=2, rna_group=4, dlb=1, ess_threshold=float(1 << 15)),
    dict(n_particles=4096, resample=3, rna_group=256, rna_exchange=0.5, arna_min=0.05),
    dict(n_particles=3001, grad=1),
], ids=["systematic", "ess", "rna", "rpa", "rpa_many_groups_ess", "arna", "grad"])
def test_graph_replays_equal_launches(ppf, frames, extra):
    p = ppf.params(**BASE, **extra)
    eager, graphed = ppf.Filter(p), ppf.Filter(p)
    graphed.graph(True)
    with pytest.raises(ppf.PPFError):
        graphed.profile(True)  # timing and graph mode exclude each other
    for k in range(frames[0].shape[0]):
        f = frames[k % 2][k]
        eager.step(f)
        graphed.step(f)
        same_filter(eager, graphed)
        if extra.get("grad"):
            assert np.array_equal(eager.grad()[0], graphed.grad()[0])
    # switching off drops the graph; the filter goes on with plain launches
    graphed.graph(False)
    eager.step(frames[0][0])
    graphed.step(frames[0][0])
    same_filter(eager, graphed)
    eager.close()
    graphed.close()


def test_batch_graph_replays_equal_launches(ppf, frames):
    # patch sizes 7, 9, 13 (one fused step launch) and 15 (a launch of its own)
    ps = [ppf.params(n_particles=n, width=W, height=H, psf_sigma=s, seed=5, track_id=t,
                     init_a=(40, 36, -1, -1, 15), init_b=(88, 76, 1, 1, 45))
          for t, (n, s) in enumerate([(1000, 1.2), (2500, 1.5), (777, 2.0), (3000, 2.4),
                                      (64, 1.3)])]
    assert sorted({ppf.patch_size(p) for p in ps}) == [7, 9, 13, 15]
    eager, graphed = ppf.Batch(ps), ppf.Batch(ps)
    graphed.graph(True)
    for k in range(frames[0].shape[0]):
        f = frames[(k + 1) % 2][k]
        eager.step(f)
        graphed.step(f)
        se, sg = eager.stats(), graphed.stats()
        for t in range(len(ps)):
            for u, v in zip(eager.particles(t), graphed.particles(t)):
                assert np.array_equal(u, v), (k, t)
            assert se[t]["delta"] == sg[t]["delta"] and se[t]["cum"] == sg[t]["cum"]
    eager.close()
    graphed.close()
