"""The allocation-free systematic resampler (its scratch is the library's
static device array) through the C ABI against the entry point with caller
scratch: identical ancestors on two calls in a row, the second with fewer
weights, and a clear error beyond its limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


def logw(n, seed):
    rng = np.random.default_rng(seed)
    l = rng.normal(0, 3, n)
    l[rng.random(n) < 0.1] = -np.inf  # particles of zero weight
    l[n // 2: n // 2 + 100] += 25.0   # a heavy run for the long-run fill
    return torch.from_numpy(l.astype(np.float32)).cuda()


def test_static_matches_caller_scratch(ppf):
    for n, seed, u in ((ppf.STATIC_MAX_N, 1, 0.37), (300_001, 2, 0.9), (1, 3, 0.5)):
        lw = logw(n, seed)
        want = ppf.resample_systematic(lw, u).cpu().numpy()
        # poison the output so that every slot must be written
        anc = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        got = ppf.resample_systematic_static(lw, u, anc=anc).cpu().numpy()
        assert np.array_equal(got, want), (n, int((got != want).sum()))
        assert got.min() >= 0 and np.all(np.diff(got) >= 0)


def test_static_rejects_beyond_limit(ppf):
    n = ppf.STATIC_MAX_N + 1
    lw = torch.zeros(n, dtype=torch.float32, device="cuda")
    anc = torch.empty(n, dtype=torch.int32, device="cuda")
    rc = ppf.lib().ppf_resample_systematic_static(ctypes.c_void_p(lw.data_ptr()), n, 0.5,
                                                  ctypes.c_void_p(anc.data_ptr()), None)
    assert rc == ppf.PPF_EINVAL
    with pytest.raises(ValueError):
        ppf.resample_systematic_static(lw, 0.5)
