"""Parity at the 2^20-particle workload, every particle, teacher-forced for
ten frames (tests/parity.py): 512 x 512 frames, s = 1.5 px, 9 x 9 patch,
uniform initial cloud over the frame (Section 6.3), resampling when ESS < N/2
(Algorithm 1), with global systematic resampling and with RNA over 4096
groups of 256 and a 10 % ring exchange (Section 3).

At this workload the ESS stays at 0.1-3 % of N (the oracle's own run of it),
so ESS < N/2 resamples at every frame. A third run lowers the threshold to
4096, where some frames keep their weights: the carried weights then go
through merges of many chunks (2^20 particles are 4096 block records, two
merge chunks of 2048) into the next step."""
import math

import numpy as np
import pytest

from paper_1310_5045_amd import synth

from parity import check_step, pair, snapshot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 1 << 20
W = H = 512
T = 10
C2 = dict(width=W, height=H, s=1.5, b=10.0, sigma=3.0, patch=9, init_kind=0,
          init_a=(0, 0, -1, -1, 15), init_b=(W, H, 1, 1, 45), seed=1)


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def movie():
    return synth.render_movie(W, H, T, intensity=30.0, sigma=1.5, background=10.0, noise_sd=3.0,
                              seed=1)


def teacher_forced(ppf, p, m, frames, rna=False):
    f = ppf.Filter(p)
    obs = torch.from_numpy(frames).cuda()
    prev, _ = snapshot(f, N, np.full(N, -math.log(N)))
    rep = []
    for k in range(1, T + 1):
        print(f"frame {k}", flush=True)
        f.step(obs[k - 1])
        cur, st = snapshot(f, N, None)
        rep.append(check_step(m, k, prev, cur, st, frames[k - 1], rna) + (st["resampled"],))
        prev = cur
    f.close()
    print(rep, flush=True)
    return rep


def test_c2_systematic_ess_half(ppf, movie):
    p, m = pair(ppf, n=N, ess_threshold=float(N // 2), **C2)
    rep = teacher_forced(ppf, p, m, movie.frames)
    assert all(r[-1] for r in rep)
    assert all(r[3] == 0 for r in rep), rep  # no ancestor mismatch beyond the 1e-10 band


def test_c2_systematic_carried_weights(ppf, movie):
    p, m = pair(ppf, n=N, ess_threshold=4096.0, **C2)
    rep = teacher_forced(ppf, p, m, movie.frames)
    kept = [r for r in rep if not r[-1]]
    assert kept and len(kept) < len(rep), rep  # both kinds of step occurred
    assert all(r[3] == 0 for r in rep if r[-1]), rep


def test_c2_rna_4096_groups(ppf, movie):
    p, m = pair(ppf, n=N, ess_threshold=float(N // 2), resample=1, rna_group=256,
                rna_exchange=0.1, **C2)
    assert m.rna_moved == 25 and N // m.rna_group == 4096
    rep = teacher_forced(ppf, p, m, movie.frames, rna=True)
    assert all(r[-1] for r in rep)
