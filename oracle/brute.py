"""Exact rational enumeration of the resampling schemes — TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
anything under oracle/.

Systematic resampling draws one uniform u and gives slot i the particle
s(i) = min{ j : (i + u)/N < C_j } with C the CDF of the normalised weights
(the resampling step of Algorithm 1 with Pr[s(i) = l] = w^l realised by a
single stratified uniform). With rational weights the map u -> s is piecewise
constant with breakpoints u = N C_j - i; enumerating the pieces gives every
possible outcome and its exact probability. RNA (Section 3) applies the same
map inside each group, then moves the last slots of each group to the next.
"""
from fractions import Fraction
from itertools import product
from typing import List, Sequence, Tuple


def cdf(w: Sequence[Fraction]) -> List[Fraction]:
    out, acc = [], Fraction(0)
    for x in w:
        acc += x
        out.append(acc)
    return out


def systematic_at(w: Sequence[Fraction], u: Fraction) -> Tuple[int, ...]:
    """s(i) = min{ j : (i + u)/N < C_j }, with C_{N-1} taken as 1."""
    n = len(w)
    C = cdf(w)
    C[-1] = Fraction(1)
    anc = []
    for i in range(n):
        ui = (i + u) / n
        anc.append(next(j for j in range(n) if ui < C[j]))
    return tuple(anc)


def systematic_pieces(w: Sequence[Fraction]):
    """[(u_lo, u_hi, ancestors)] covering [0, 1): s is constant on each
    half-open piece [u_lo, u_hi)."""
    n = len(w)
    C = cdf(w)
    C[-1] = Fraction(1)
    cuts = {Fraction(0), Fraction(1)}
    for j in range(n):
        for i in range(n):
            u = n * C[j] - i
            if 0 < u < 1:
                cuts.add(u)
    cuts = sorted(cuts)
    pieces = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        pieces.append((lo, hi, systematic_at(w, lo)))  # constant on [lo, hi)
    return pieces


def expected_offspring(w: Sequence[Fraction]) -> List[Fraction]:
    """E_u[o_j], o_j = #{i : s(i) = j}, exactly."""
    n = len(w)
    e = [Fraction(0)] * n
    for lo, hi, anc in systematic_pieces(w):
        for j in anc:
            e[j] += hi - lo
    return e


def rna_at(w: Sequence[Fraction], group: int, moved: int, us: Sequence[Fraction]):
    """Ancestors and per-slot weights of RNA for one choice of group uniforms."""
    n = len(w)
    G = n // group
    local, Wg = [], []
    for g in range(G):
        ws = w[g * group:(g + 1) * group]
        W = sum(ws, Fraction(0))
        Wg.append(W)
        if W == 0:
            local.extend(range(g * group, (g + 1) * group))
        else:
            loc = systematic_at([x / W for x in ws], us[g])
            local.extend(g * group + j for j in loc)
    anc, wslot = [], []
    for g in range(G):
        prev = (g - 1) % G
        for l in range(group):
            if l >= group - moved:
                anc.append(local[prev * group + l])
                wslot.append(Wg[prev] / group)
            else:
                anc.append(local[g * group + l])
                wslot.append(Wg[g] / group)
    return tuple(anc), tuple(wslot)


def rna_pieces(w: Sequence[Fraction], group: int, moved: int):
    """Enumerate every combination of per-group pieces: [(prob, anc, wslot)]."""
    n = len(w)
    G = n // group
    per_group = []
    for g in range(G):
        ws = w[g * group:(g + 1) * group]
        W = sum(ws, Fraction(0))
        if W == 0:
            per_group.append([(Fraction(0), Fraction(1))])
        else:
            per_group.append([(lo, hi) for lo, hi, _ in systematic_pieces([x / W for x in ws])])
    out = []
    for combo in product(*per_group):
        prob = Fraction(1)
        for lo, hi in combo:
            prob *= hi - lo
        anc, wslot = rna_at(w, group, moved, [lo for lo, _ in combo])
        out.append((prob, anc, wslot))
    return out


def arna_at(w: Sequence[Fraction], group: int, mu_min: int, mu_max: int, theta: Fraction,
            us: Sequence[Fraction], order: Sequence[int]):
    """ARNA's resampling for one choice of group uniforms and a ring order
    (order[j]: the group at ring position j): RNA's local resampling, G_t =
    #{g : W_g >= theta / G}, mu = mu_min + floor((mu_max - mu_min)(G - G_t)/G),
    the last mu slots of each group from its ring predecessor. Returns
    (ancestors, slot weights, G_t, mu)."""
    n = len(w)
    G = n // group
    local, Wg = [], []
    for g in range(G):
        ws = w[g * group:(g + 1) * group]
        W = sum(ws, Fraction(0))
        Wg.append(W)
        if W == 0:
            local.extend(range(g * group, (g + 1) * group))
        else:
            loc = systematic_at([x / W for x in ws], us[g])
            local.extend(g * group + j for j in loc)
    t = sum(1 for W in Wg if W >= theta / G)
    mu = mu_min + ((mu_max - mu_min) * (G - t)) // G
    pos = {g: j for j, g in enumerate(order)}
    anc, wslot = [], []
    for g in range(G):
        pred = order[(pos[g] - 1) % G]
        for l in range(group):
            src = pred if l >= group - mu else g
            anc.append(local[src * group + l])
            wslot.append(Wg[src] / group)
    return tuple(anc), tuple(wslot), t, mu
