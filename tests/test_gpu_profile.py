"""Kernel timing (ppf_profile_enable / ppf_profile_read): the timed units a
step reports for each resampling scheme, one launch of each per step, and
timing that changes nothing the filter computes (a timed filter equals an
untimed twin bit for bit)."""
import numpy as np
import pytest

from paper_1310_5045_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H = 128, 112
BASE = dict(width=W, height=H, psf_sigma=1.5, background=10.0, noise_sigma=3.0,
            init_a=(40, 36, -1, -1, 15), init_b=(88, 76, 1, 1, 45), seed=6)
STEPS = 5


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def frames():
    mv = synth.render_movie(W, H, STEPS, intensity=30.0, sigma=1.5, start_box=(48, 80, 44, 68),
                            seed=2)
    return torch.from_numpy(mv.frames).cuda()


@pytest.mark.parametrize("extra,units", [
    (dict(n_particles=5000), {"k_step", "k_merge", "k_resample"}),
    (dict(n_particles=4096, resample=1, rna_group=256, rna_exchange=0.1),
     {"k_step", "k_merge", "k_rna"}),
    (dict(n_particles=4096, resample=3, rna_group=256, rna_exchange=0.5, arna_min=0.05),
     {"k_step", "k_merge", "k_rna"}),
    (dict(n_particles=4096, resample=2, rna_group=256, dlb=1),
     {"k_step", "k_merge", "k_resample", "k_rpa"}),
], ids=["systematic", "rna", "arna", "rpa"])
def test_timed_units_and_no_effect(ppf, frames, extra, units):
    p = ppf.params(**BASE, **extra)
    timed, plain = ppf.Filter(p), ppf.Filter(p)
    timed.profile(True)
    for k in range(STEPS):
        timed.step(frames[k])
        plain.step(frames[k])
    kt = timed.kernel_times()
    assert set(kt) == units, kt
    for name, (launches, total_ms) in kt.items():
        assert launches == STEPS, (name, launches)
        assert total_ms > 0.0, name
    for u, v in zip(timed.particles(), plain.particles()):
        assert np.array_equal(u, v)
    assert timed.stats()["cum"] == plain.stats()["cum"]
    # enabling again clears the accumulated times
    timed.profile(True)
    assert timed.kernel_times() == {}
    timed.close()
    plain.close()
