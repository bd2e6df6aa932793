"""GPU parity of resampling with proportional allocation (RPA, Section 3)
and the DLB schedules of Section 4 against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_5045_amd import synth

from parity import GpuState, check_propagate, check_systematic, check_weights, pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


def test_dlb_hand_example(ppf):
    counts = torch.tensor([9, 3, 7, 1, 4, 6, 2], dtype=torch.int32).cuda()
    assert ppf.dlb_schedule(ppf.DLB_GS, counts, 4).cpu().tolist() == [[0, 1, 1], [0, 3, 3],
                                                                      [0, 6, 1], [2, 6, 1]]
    assert ppf.dlb_schedule(ppf.DLB_SGS, counts, 4).cpu().tolist() == [[0, 3, 3], [0, 6, 2],
                                                                       [2, 1, 1]]
    assert ppf.dlb_schedule(ppf.DLB_LGS, counts, 4).cpu().tolist() == [[0, 3, 3], [2, 6, 2],
                                                                       [5, 1, 1]]


@pytest.mark.parametrize("G,n", [(1, 8), (37, 16), (1000, 64), (4096, 256)])
def test_dlb_schedules_match_oracle(ppf, G, n):
    rng = np.random.default_rng(G)
    for trial in range(3):
        if trial == 0:  # a real systematic allocation (balanced)
            w = rng.gamma(0.3, 1.0, G * n)
            w /= w.sum()
            counts = oracle.rpa_counts(oracle.resample_systematic(w, float(rng.uniform())), n)
        else:  # arbitrary counts, balanced or not
            counts = rng.integers(0, 3 * n, G).astype(np.int32)
        ct = torch.from_numpy(counts.astype(np.int32)).cuda()
        for kind in (ppf.DLB_GS, ppf.DLB_SGS, ppf.DLB_LGS):
            got = ppf.dlb_schedule(kind, ct, n).cpu().numpy()
            want = oracle.dlb_schedule(kind, counts, n)
            assert np.array_equal(got, want), (G, n, trial, kind)


@pytest.mark.parametrize("G,n", [(5000, 8), (152_000, 250)])
def test_dlb_schedules_many_groups_match_oracle(ppf, G, n):
    """Beyond one tile of the radix sort and of the scans: a systematic
    allocation at 152,000 groups (the 38M workload with groups of 250), and
    unbalanced counts."""
    rng = np.random.default_rng(G)
    w = rng.gamma(0.05, 1.0, G * n)
    w /= w.sum()
    balanced = oracle.rpa_counts(oracle.resample_systematic(w, float(rng.uniform())), n)
    for counts in (balanced, rng.integers(0, 3 * n, G).astype(np.int32)):
        ct = torch.from_numpy(counts.astype(np.int32)).cuda()
        for kind in (ppf.DLB_GS, ppf.DLB_SGS, ppf.DLB_LGS):
            got = ppf.dlb_schedule(kind, ct, n).cpu().numpy()
            want = oracle.dlb_schedule(kind, counts, n)
            assert np.array_equal(got, want), (G, n, kind, got.shape, want.shape)


def test_dlb_schedule_capacity(ppf):
    """Too small a capacity: the count reads -1 and no entry is written."""
    import ctypes
    counts = torch.tensor([9, 3, 7, 1, 4, 6, 2], dtype=torch.int32).cuda()
    sched = torch.full((3, 3), -7, dtype=torch.int32).cuda()
    m = torch.zeros(1, dtype=torch.int32).cuda()
    s = torch.cuda.current_stream()
    rc = ppf.lib().ppf_dlb_schedule(ppf.DLB_GS, ctypes.c_void_p(counts.data_ptr()), 7, 4,
                                    ctypes.c_void_p(sched.data_ptr()), 3,
                                    ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    assert rc == 0
    assert int(m.cpu()) == -1 and bool(torch.all(sched == -7))


@pytest.mark.parametrize("dlb", [0, 1])
@pytest.mark.parametrize("n,group", [(4096, 256), (8192, 64), (3000, 1000)])
def test_rpa_filter(ppf, dlb, n, group):
    mv = synth.render_movie(128, 128, 5, intensity=30.0, sigma=1.5, start_box=(40, 88, 40, 88),
                            seed=21)
    p, m = pair(ppf, n=n, width=128, height=128, s=1.5, b=10.0, sigma=3.0,
                init_a=(32, 32, -1, -1, 15), init_b=(96, 96, 1, 1, 45), resample=0, seed=4)
    p.resample = ppf.RESAMPLE_RPA
    p.rna_group = group
    p.dlb = dlb
    f = ppf.Filter(p)
    frames = torch.from_numpy(mv.frames).cuda()
    x, lw, anc = f.particles()
    prev = GpuState(x, lw, anc, False, np.full(n, -math.log(n)))
    for k in range(1, 5):
        f.step(frames[k - 1])
        x, lw, anc = f.particles()
        st = f.stats()
        cur = GpuState(x, lw, anc, bool(st["resampled"]), None)
        # the oracle's systematic filter step: propagation and weights
        check_propagate(m, k, prev, cur.x)
        check_weights(m, mv.frames[k - 1], prev.lw_next, cur.x, cur.lw, st)
        w_gpu = np.exp(cur.lw)
        # the resampled multiset is that of global systematic resampling
        sys_anc = np.sort(cur.anc)
        check_systematic(w_gpu, oracle.resample_uniform(m, k), sys_anc)
        # and the placement is the oracle's routing of that multiset
        assert np.array_equal(cur.anc, oracle.route_rpa(sys_anc, group, dlb)), k
        cur.lw_next = np.full(n, -math.log(n))
        prev = cur
    f.close()


@pytest.mark.parametrize("dlb", [0, 1])
@pytest.mark.parametrize("group", [64, 8])
def test_rpa_filter_many_groups(ppf, dlb, group):
    """2^20 particles in 16,384 or 131,072 groups (the sorted schedule's radix
    sort and the list scans over many tiles): the resampled multiset is the
    systematic one and the placement the oracle's routing."""
    n = 1 << 20
    mv = synth.render_movie(256, 256, 3, intensity=30.0, sigma=1.5, start_box=(96, 160, 96, 160),
                            seed=23)
    p, m = pair(ppf, n=n, width=256, height=256, s=1.5, b=10.0, sigma=3.0,
                init_a=(64, 64, -1, -1, 15), init_b=(192, 192, 1, 1, 45), resample=0, seed=6)
    p.resample = ppf.RESAMPLE_RPA
    p.rna_group = group
    p.dlb = dlb
    f = ppf.Filter(p)
    frames = torch.from_numpy(mv.frames).cuda()
    for k in range(1, 3):
        f.step(frames[k - 1])
        x, lw, anc = f.particles()
        assert f.stats()["resampled"]
        sys_anc = np.sort(anc)
        check_systematic(np.exp(lw), oracle.resample_uniform(m, k), sys_anc)
        routed = oracle.route_rpa(sys_anc, group, dlb)
        assert np.array_equal(anc, routed), (k, int(np.sum(anc != routed)))
    f.close()


@pytest.mark.parametrize("dlb", [0, 1])
def test_rpa_filter_ess_threshold_many_groups(ppf, dlb):
    """16,384 groups with an ESS threshold: steps that do not resample leave
    the ancestors and carried weights to the plain step (the routing kernels
    do nothing), steps that do are routed as the oracle routes them."""
    n, group = 1 << 16, 4
    mv = synth.render_movie(128, 128, 6, intensity=30.0, sigma=1.5, start_box=(40, 88, 40, 88),
                            seed=25)
    p, m = pair(ppf, n=n, width=128, height=128, s=1.5, b=10.0, sigma=3.0,
                init_a=(32, 32, -1, -1, 15), init_b=(96, 96, 1, 1, 45), resample=0, seed=8,
                ess_threshold=float(n // 100))  # the oracle's run resamples at steps 1, 2, 4, 5
    p.resample = ppf.RESAMPLE_RPA
    p.rna_group = group
    p.dlb = dlb
    f = ppf.Filter(p)
    frames = torch.from_numpy(mv.frames).cuda()
    x, lw, anc = f.particles()
    prev = GpuState(x, lw, anc, False, np.full(n, -math.log(n)))
    seen = set()
    for k in range(1, 7):
        f.step(frames[k - 1])
        x, lw, anc = f.particles()
        st = f.stats()
        cur = GpuState(x, lw, anc, bool(st["resampled"]), None)
        check_propagate(m, k, prev, cur.x)
        check_weights(m, mv.frames[k - 1], prev.lw_next, cur.x, cur.lw, st)
        seen.add(cur.resampled)
        if cur.resampled:
            sys_anc = np.sort(cur.anc)
            check_systematic(np.exp(cur.lw), oracle.resample_uniform(m, k), sys_anc)
            assert np.array_equal(cur.anc, oracle.route_rpa(sys_anc, group, dlb)), k
            cur.lw_next = np.full(n, -math.log(n))
        else:
            assert np.array_equal(cur.anc, np.arange(n))
            cur.lw_next = cur.lw
        prev = cur
    f.close()
    assert seen == {True, False}, seen
