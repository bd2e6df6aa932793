"""Teacher-forced comparison of one GPU filter step with the FP64 oracle.

Each check feeds the oracle the GPU's own fp32 inputs (widened exactly), so it
measures one step's arithmetic only:
  propagate   oracle propagates the GPU's previous states with the same
              Philox streams; the GPU state must match to fp32 rounding;
  weights     oracle evaluates Eq. 4 on the GPU's propagated states with the
              carried log weights the GPU used; normalised weights within
              1e-5 relative where l - m >= -40 (else GPU weight < 1e-17),
              MMSE estimate within 1e-3, log-likelihood increment within 1e-4;
  ancestors   oracle resamples the GPU's normalised weights with the same
              uniform; ancestors must be identical for every slot whose
              uniform is farther than `band` from a CDF step; mismatches
              inside the band are counted and returned.
"""
import math
from dataclasses import dataclass

import numpy as np

import oracle

WEIGHT_RTOL = 1e-5
MEAN_ATOL = 1e-3
DELTA_ATOL = 1e-4


def pair(ppf, **kw):
    """Matching library parameters and oracle model (library-only keys such
    as grad are not passed to the oracle)."""
    okw = {k: v for k, v in kw.items() if k not in ("grad",)}
    pkw = {}
    ren = dict(n="n_particles", s="psf_sigma", b="background", sigma="noise_sigma", track="track_id",
               rna_exchange="rna_exchange")
    for k, v in kw.items():
        pkw[ren.get(k, k)] = v
    return ppf.params(**pkw), oracle.Model(**okw)


@dataclass
class GpuState:
    x: np.ndarray       # (5, N) float32
    lw: np.ndarray      # (N,) float64 normalised log weights of the last step
    anc: np.ndarray     # (N,) int32
    resampled: bool
    lw_next: np.ndarray  # carried log weight the next step uses


def snapshot(f, n, lw_next):
    x, lw, anc = f.particles()
    st = f.stats()
    return GpuState(x, lw, anc, bool(st["resampled"]), lw_next), st


def check_propagate(m, k, prev: GpuState, x_gpu):
    parent = prev.anc if prev.resampled else None
    xo = oracle.propagate(m, k, prev.x.astype(np.float64), parent)
    tol = np.spacing(np.abs(xo).astype(np.float32)).astype(np.float64) + 1e-6
    err = np.abs(x_gpu.astype(np.float64) - xo)
    bad = err > tol
    assert not bad.any(), f"propagate: {bad.sum()} values off, worst {err.max():.3e}"
    return err.max()


def check_weights(m, obs, lw_in, x_gpu, lw_gpu, st):
    l = lw_in + oracle.loglik(m, obs, x_gpu.astype(np.float64))
    w, s = oracle.normalize(l)
    keep = l - s["m"] >= -40.0
    rel = np.abs(np.exp(lw_gpu[keep]) - w[keep]) / w[keep]
    assert rel.max() <= WEIGHT_RTOL, f"weights: worst relative error {rel.max():.3e}"
    assert np.all(np.exp(lw_gpu[~keep]) < 1e-17)
    mean = oracle.estimate(w, x_gpu.astype(np.float64))
    assert np.abs(mean - st["mean"]).max() <= MEAN_ATOL, (mean, st["mean"])
    assert abs(s["delta"] - st["delta"]) <= DELTA_ATOL, (s["delta"], st["delta"])
    assert math.isclose(s["ess"], st["ess"], rel_tol=1e-6)
    assert (st["ess"] < m.ess_threshold) == bool(st["resampled"])
    return rel.max(), s


def band_distance(u_slots, C):
    """Distance of each slot uniform to the nearest CDF step."""
    j = np.searchsorted(C, u_slots)
    lo = np.abs(u_slots - C[np.clip(j - 1, 0, C.size - 1)])
    hi = np.abs(C[np.clip(j, 0, C.size - 1)] - u_slots)
    return np.minimum(lo, hi)


def check_systematic(w_gpu, u, anc_gpu, band=1e-9):
    """Returns (mismatches inside band, inside 1e-10)."""
    n = w_gpu.size
    ao = oracle.resample_systematic(w_gpu, u)
    mism = ao != anc_gpu
    if not mism.any():
        return 0, 0
    C = np.cumsum(w_gpu)
    d = band_distance((np.arange(n) + u) / n, C[:-1])
    outside = mism & (d > band)
    assert not outside.any(), f"ancestors: {outside.sum()} mismatches outside band {band}"
    return int(mism.sum()), int((mism & (d > 1e-10)).sum())


def check_rna(w_gpu, group, moved, u_g, anc_gpu, band=1e-9):
    n = w_gpu.size
    ao, lwg, lws = oracle.resample_rna(w_gpu, group, moved, u_g)
    mism = ao != anc_gpu
    if mism.any():
        G = n // group
        d = np.full(n, np.inf)
        local = np.empty(n)
        for g in range(G):
            ws = w_gpu[g * group:(g + 1) * group]
            W = ws.sum()
            if W > 0:
                C = np.cumsum(ws) / W
                ul = (np.arange(group) + u_g[g]) / group
                local[g * group:(g + 1) * group] = band_distance(ul, C[:-1])
            else:
                local[g * group:(g + 1) * group] = np.inf
        for g in range(G):
            prev = (g - 1) % G
            for l in range(group):
                src = prev if l >= group - moved else g
                d[g * group + l] = local[src * group + l]
        outside = mism & (d > band)
        assert not outside.any(), f"RNA ancestors: {outside.sum()} mismatches outside band"
    return int(mism.sum()), lws


def local_band(w_gpu, group, u_g):
    """Per slot, the distance of its local uniform to the nearest step of its
    own group's local CDF (inf for a group without weight)."""
    n = w_gpu.size
    G = n // group
    local = np.empty(n)
    for g in range(G):
        ws = w_gpu[g * group:(g + 1) * group]
        W = ws.sum()
        if W > 0:
            C = np.cumsum(ws) / W
            ul = (np.arange(group) + u_g[g]) / group
            local[g * group:(g + 1) * group] = band_distance(ul, C[:-1])
        else:
            local[g * group:(g + 1) * group] = np.inf
    return local


def check_arna(m, k, w_gpu, anc_gpu, arna_gpu, ring_key, band=1e-9):
    """ARNA's resampling of the GPU's weights by the oracle with the ring of
    `ring_key`: the tracking count (up to groups within 1e-9 of the share
    theta / G), the slots exchanged, and the ancestors (identical outside the
    band, through each slot's source group). Returns (mismatches, slot log
    weights for the next step)."""
    n, group = w_gpu.size, m.rna_group
    G = n // group
    order = oracle.ring_order(m, ring_key, G)
    u_g = oracle.rna_uniforms(m, k)
    theta = float(np.float32(m.arna_track))
    _, _, _, t, _ = oracle.resample_arna(w_gpu, group, m.arna_mu_min, m.rna_moved, theta, u_g,
                                         order)
    W = w_gpu.reshape(G, group).sum(1)
    amb = int(np.sum(np.abs(W - theta / G) <= 1e-9 * theta / G))
    t_gpu = arna_gpu["tracking"]
    assert abs(t_gpu - t) <= amb, (arna_gpu, t, amb)
    mu = m.arna_mu_min + (m.rna_moved - m.arna_mu_min) * (G - t_gpu) // G
    assert arna_gpu["moved"] == mu, (arna_gpu, mu)
    # the oracle's resampling with the GPU's exchange size
    ao, lwg, lws, _, _ = oracle.resample_arna(w_gpu, group, mu, mu, theta, u_g, order)
    mism = ao != anc_gpu
    if mism.any():
        pos = np.empty(G, dtype=np.int64)
        pos[order] = np.arange(G)
        pred = order[(pos - 1) % G]
        local = local_band(w_gpu, group, u_g)
        g = np.arange(n) // group
        tail = (np.arange(n) % group) >= group - mu
        src = np.where(tail, pred[g], g)
        d = local[src * group + np.arange(n) % group]
        outside = mism & (d > band)
        assert not outside.any(), f"ARNA ancestors: {outside.sum()} mismatches outside band"
    return int(mism.sum()), lws


def check_step(m, k, prev: GpuState, cur: GpuState, st, obs, rna=False):
    """All checks of step k (propagate, weights, then the resampling or the
    carried weights); sets cur.lw_next and returns a report tuple."""
    n = m.n
    assert st["k"] == k
    check_propagate(m, k, prev, cur.x)
    rel, _ = check_weights(m, obs, prev.lw_next, cur.x, cur.lw, st)
    w_gpu = np.exp(cur.lw)
    if cur.resampled:
        if rna:
            ug = oracle.rna_uniforms(m, k)
            nm, lws = check_rna(w_gpu, m.rna_group, m.rna_moved, ug, cur.anc)
            cur.lw_next = lws
            return (k, rel, nm)
        nm, nm10 = check_systematic(w_gpu, oracle.resample_uniform(m, k), cur.anc)
        cur.lw_next = np.full(n, -math.log(n))
        return (k, rel, nm, nm10)
    assert np.array_equal(cur.anc, np.arange(n))
    cur.lw_next = cur.lw.copy()
    return (k, rel, 0)


# Workgroups of the step kernel take one of three ways to the patch moments,
# chosen by the bounding box of their 256 patch centres (acx x acy centres):
# "sum"  the box's tile fits the LDS copies and both row-sum tables (of D^2 and
#        of D) fit: nH = (acy + P - 1) acx <= 768 entries;
# "tab"  the tile fits (2 ceil((acx + P - 1) / 2) (acy + P - 1) <= 1008
#        doubles per copy) but only the D^2 table: 768 < nH;
# "glob" the tile does not fit: pixels are read from the frame.
# (A tile that fits always leaves room for the D^2 table, so there is no
# fourth way.) Each box below sits at the limit of its way.
PATH_BOXES = {
    9: {"sum": (5, 5), "tab": (30, 18), "glob": (31, 29)},
    11: {"sum": (5, 5), "tab": (40, 10), "glob": (41, 23)},
    13: {"sum": (5, 5), "tab": (44, 6), "glob": (45, 25)},
}
# where each layout's box starts: at the spot, over the left edge, over the
# bottom edge of a 96 x 80 frame
PATH_ORIGINS = {"sum": (44, 38), "tab": (-6, 30), "glob": (20, 60)}


def path_of(P, acx, acy):
    th = acy + P - 1
    if 2 * ((acx + P) // 2) * th > 1008:
        return "glob"
    return "sum" if th * acx <= 768 else "tab"


def box_layout(rng, n, acx, acy, x0, y0):
    """States whose patch centres fill an acx x acy box at (x0, y0) in every
    block of 256 (each block's first two particles sit at its corners),
    0.1 px off the centres so that the tiny process noise keeps the
    rounding; velocities 0."""
    cx = rng.integers(0, acx, n)
    cy = rng.integers(0, acy, n)
    for b0 in range(0, n, 256):
        cx[b0], cy[b0] = 0, 0
        if b0 + 1 < n:
            cx[b0 + 1], cy[b0 + 1] = acx - 1, acy - 1
    x = np.zeros((5, n))
    x[0] = x0 + cx + 0.1
    x[1] = y0 + cy - 0.1
    x[4] = rng.uniform(20, 40, n)
    return x.astype(np.float32)
