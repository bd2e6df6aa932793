"""Pins of the oracle's RPA resampling and its DLB schedules (Section 4:
Greedy, Sorted Greedy and Largest Gradient schedulers) against hand-worked
schedules, the interval form of greedy matching, conservation and balance,
and the multiset of global systematic resampling."""
import numpy as np
import pytest

import oracle

GS, SGS, LGS = oracle.DLB_GS, oracle.DLB_SGS, oracle.DLB_LGS


def test_hand_worked_schedules():
    # counts of seven groups of n = 4: senders g0 (+5), g2 (+3), g5 (+2);
    # receivers g1 (-1), g3 (-3), g6 (-2)
    counts = np.array([9, 3, 7, 1, 4, 6, 2])
    # GS, both lists in group order: g0 fills g1 (1) and g3 (3), gives its
    # last particle to g6; g2 then fills g6's remaining slot; g2 and g5
    # keep the rest (the surplus exceeds the deficit here)
    assert oracle.dlb_schedule(GS, counts, 4).tolist() == [[0, 1, 1], [0, 3, 3], [0, 6, 1],
                                                           [2, 6, 1]]
    # SGS: senders g0 (5), g2 (3), g5 (2); receivers g3 (3), g6 (2), g1 (1):
    # g0 fills g3 and g6, g2 fills g1 -- one link fewer than GS
    assert oracle.dlb_schedule(SGS, counts, 4).tolist() == [[0, 3, 3], [0, 6, 2], [2, 1, 1]]
    # LGS: rank pairs (g0, g3), (g2, g6), (g5, g1), each moving the smaller
    # of surplus and deficit
    assert oracle.dlb_schedule(LGS, counts, 4).tolist() == [[0, 3, 3], [2, 6, 2], [5, 1, 1]]


def interval_matching(counts, n, order_s, order_r):
    """Greedy matching as overlaps of the senders' surplus intervals and the
    receivers' deficit intervals laid end to end (in the given orders)."""
    sur = np.array([counts[g] - n for g in order_s])
    dfc = np.array([n - counts[g] for g in order_r])
    cs = np.concatenate([[0], np.cumsum(sur)])
    cr = np.concatenate([[0], np.cumsum(dfc)])
    top = min(cs[-1], cr[-1])
    pts = np.unique(np.concatenate([cs[cs <= top], cr[cr <= top]]))
    out = []
    for a, b in zip(pts[:-1], pts[1:]):
        i = np.searchsorted(cs, a, side="right") - 1
        j = np.searchsorted(cr, a, side="right") - 1
        if out and out[-1][0] == order_s[i] and out[-1][1] == order_r[j]:
            out[-1][2] += int(b - a)
        else:
            out.append([int(order_s[i]), int(order_r[j]), int(b - a)])
    return out


def balanced_counts(rng, G, n):
    """Offspring counts of a real systematic allocation over G groups."""
    w = rng.gamma(0.3, 1.0, G * n)
    w /= w.sum()
    anc = oracle.resample_systematic(w, float(rng.uniform()))
    return oracle.rpa_counts(anc, n), w


@pytest.mark.parametrize("seed", range(6))
def test_greedy_schedules_are_interval_matchings_and_balance(seed):
    rng = np.random.default_rng(seed)
    G, n = int(rng.integers(2, 60)), int(rng.choice([4, 16, 64]))
    counts, _ = balanced_counts(rng, G, n)
    assert counts.sum() == G * n
    S = [g for g in range(G) if counts[g] > n]
    R = [g for g in range(G) if counts[g] < n]
    key_s = lambda g: (-(counts[g] - n), g)  # noqa: E731
    key_r = lambda g: (-(n - counts[g]), g)  # noqa: E731
    for kind, (os_, or_) in ((GS, (S, R)), (SGS, (sorted(S, key=key_s), sorted(R, key=key_r)))):
        sched = oracle.dlb_schedule(kind, counts, n)
        assert sched.tolist() == interval_matching(counts, n, os_, or_)
        moved_out = np.zeros(G, int)
        moved_in = np.zeros(G, int)
        for s, r, c in sched:
            assert c > 0
            moved_out[s] += c
            moved_in[r] += c
        # every group ends with n particles
        assert np.array_equal(counts - moved_out + moved_in, np.full(G, n))
        assert len(sched) <= len(S) + len(R) - 1 if S else len(sched) == 0


@pytest.mark.parametrize("seed", range(4))
def test_lgs_pairs_ranks(seed):
    rng = np.random.default_rng(10 + seed)
    G, n = 40, 16
    counts, _ = balanced_counts(rng, G, n)
    S = sorted([g for g in range(G) if counts[g] > n], key=lambda g: (-(counts[g] - n), g))
    R = sorted([g for g in range(G) if counts[g] < n], key=lambda g: (-(n - counts[g]), g))
    sched = oracle.dlb_schedule(LGS, counts, n)
    assert len(sched) == min(len(S), len(R))
    for i, (s, r, c) in enumerate(sched):
        assert s == S[i] and r == R[i]
        assert c == min(counts[s] - n, n - counts[r])


@pytest.mark.parametrize("kind", [GS, SGS])
@pytest.mark.parametrize("seed", range(4))
def test_rpa_resampling(kind, seed):
    rng = np.random.default_rng(20 + seed)
    G, n = int(rng.integers(3, 40)), 32
    w = rng.gamma(0.2, 1.0, G * n)
    w[rng.random(G * n) < 0.3] = 0.0
    w /= w.sum()
    u = float(rng.uniform())
    sys_anc = oracle.resample_systematic(w, u)
    anc = oracle.resample_rpa(w, u, n, kind)
    # the same offspring as global systematic resampling, only placed elsewhere
    assert np.array_equal(np.sort(anc), np.sort(sys_anc))
    counts = oracle.rpa_counts(sys_anc, n)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for g in range(G):
        keep = min(counts[g], n)
        # a group keeps its own first offspring, in order
        assert np.array_equal(anc[g * n:g * n + keep], sys_anc[first[g]:first[g] + keep])
        # and its remaining slots hold other groups' surplus
        assert np.all(anc[g * n + keep:(g + 1) * n] // n != g)
