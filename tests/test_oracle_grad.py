"""Pins of the oracle's derivatives of log p^ (reparameterised: Philox noise
and resampling ancestors fixed) against central finite differences of the
oracle's own values, which the other oracle tests pin to the paper's model:
per particle (Eq. 4 in the state and in s, b, sigma_xi), for the tangents of
the dynamics in q, and for whole runs with the ancestors replayed. A wrong
sign, a dropped factor of I0 or 1/s^2, a missing in-frame mask in d/db, or a
tangent fed from the wrong parent or velocity fails one of these."""
import copy

import numpy as np
import pytest

import oracle
from paper_1310_5045_amd import synth

W, H = 40, 36


def perturbed(m, field, idx, delta):
    """C model with one fp64 field moved by delta (off the fp32 grid)."""
    c = m.c()
    if idx is None:
        setattr(c, field, getattr(c, field) + delta)
    else:
        getattr(c, field)[idx] += delta
    return c


@pytest.fixture(scope="module")
def frame():
    return synth.render_movie(W, H, 1, intensity=30.0, sigma=1.2, start_box=(10, 30, 10, 26),
                              seed=4).frames[0]


def states(n, rng):
    """Particles inside, across and outside the frame border, none within
    1e-3 of a half-pixel boundary (so small moves keep the patch centre)."""
    x = np.empty((5, n))
    x[0] = rng.uniform(-6, W + 6, n)
    x[1] = rng.uniform(-6, H + 6, n)
    x[2:4] = rng.uniform(-1, 1, (2, n))
    x[4] = rng.uniform(10, 50, n)
    for d in (0, 1):
        f = x[d] + 0.5 - np.floor(x[d] + 0.5)
        x[d] += np.where(f < 1e-3, 2e-3, 0.0) - np.where(f > 1 - 1e-3, 2e-3, 0.0)
    return x


def test_loglik_grad_state_components(frame):
    rng = np.random.default_rng(1)
    m = oracle.Model(n=400, width=W, height=H, s=1.2)
    x = states(m.n, rng)
    dll = oracle.loglik_grad(m, frame, x)
    for comp, row in ((0, 0), (1, 1), (4, 2)):
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[comp] += h
        xm[comp] -= h
        fd = (oracle.loglik(m, frame, xp) - oracle.loglik(m, frame, xm)) / (2 * h)
        assert np.allclose(dll[row], fd, rtol=1e-5, atol=1e-5), (comp, np.abs(dll[row] - fd).max())


@pytest.mark.parametrize("field,row,h", [("s", 3, 1e-6), ("b", 4, 1e-5), ("sigma", 5, 1e-6)])
def test_loglik_grad_model_components(frame, field, row, h):
    rng = np.random.default_rng(2)
    m = oracle.Model(n=400, width=W, height=H, s=1.2)
    x = states(m.n, rng)
    dll = oracle.loglik_grad(m, frame, x)
    lp = oracle.loglik(m, frame, x, c=perturbed(m, field, None, h))
    lm = oracle.loglik(m, frame, x, c=perturbed(m, field, None, -h))
    fd = (lp - lm) / (2 * h)
    assert np.allclose(dll[row], fd, rtol=1e-5, atol=1e-5), np.abs(dll[row] - fd).max()


def test_loglik_grad_b_only_counts_pixels_inside(frame):
    # a particle whose patch lies wholly outside the frame has dl/db = 0
    m = oracle.Model(n=2, width=W, height=H, s=1.2)
    x = np.array([[-30.0, 5.0], [-30.0, 5.0], [0, 0], [0, 0], [20.0, 20.0]])
    dll = oracle.loglik_grad(m, frame, x)
    assert dll[4, 0] == 0.0 and dll[4, 1] != 0.0


def test_tangents_match_finite_differences():
    rng = np.random.default_rng(3)
    m = oracle.Model(n=300, width=W, height=H, s=1.2, q=(0.5, 0.7, 0.2, 0.3, 1.5))
    x0 = states(m.n, rng)
    parents = [None, rng.integers(0, m.n, m.n).astype(np.int32),
               np.sort(rng.integers(0, m.n, m.n)).astype(np.int32)]
    t = np.zeros((7, m.n))
    for k in range(1, 4):
        t = oracle.propagate_tangent(m, k, t, parents[k - 1])
    # rows of the tangent and the state component they differentiate, per q_d
    cols = {0: [(0, 0)], 1: [(1, 1)], 2: [(2, 2), (3, 0)], 3: [(4, 3), (5, 1)], 4: [(6, 4)]}
    for d, pairs in cols.items():
        h = 1e-6
        xs = []
        for sgn in (1, -1):
            c = perturbed(m, "q", d, sgn * h)
            x = x0
            for k in range(1, 4):
                x = oracle.propagate(m, k, x, parents[k - 1], c=c)
            xs.append(x)
        for row, comp in pairs:
            fd = (xs[0][comp] - xs[1][comp]) / (2 * h)
            assert np.allclose(t[row], fd, rtol=1e-6, atol=1e-6), (d, row)
        # the other state components do not depend on q_d
        others = set(range(5)) - {comp for _, comp in pairs}
        for comp in others:
            assert np.array_equal(xs[0][comp], xs[1][comp])


def _fd_run(m, frames, T, anc, field, idx, h):
    """Central difference of cum with the ancestors replayed; h is reduced
    until no particle's patch centre differs between the two runs."""
    for _ in range(4):
        out = []
        for sgn in (1, -1):
            if field == "I0":
                c = m.c()
                c.init_a[4] += sgn * h
                c.init_b[4] += sgn * h
            else:
                c = perturbed(m, field, idx, sgn * h)
            out.append(oracle.run_grad(m, frames, T, anc_replay=anc, trace=True, c=c))
        cp = np.floor(out[0][3][:, :2] + 0.5)
        cm = np.floor(out[1][3][:, :2] + 0.5)
        if np.array_equal(cp, cm):
            return (out[0][0] - out[1][0]) / (2 * h)
        h /= 8
    pytest.fail(f"{field}: patch centres keep moving under the perturbation")


def test_run_grad_matches_finite_differences():
    mv = synth.render_movie(48, 48, 3, intensity=30.0, sigma=1.2, start_box=(18, 30, 18, 30),
                            seed=5)
    m = oracle.Model(n=150, width=48, height=48, s=1.2, init_a=(19, 19, -1, -1, 20),
                     init_b=(29, 29, 1, 1, 40), q=(0.5, 0.5, 0.2, 0.2, 1.0), seed=9)
    T = 3
    cum, g, anc = oracle.run_grad(m, mv.frames, T)
    # the ancestor replay reproduces the base run exactly
    cum2, g2, anc2 = oracle.run_grad(m, mv.frames, T, anc_replay=anc)
    assert cum2 == cum and np.array_equal(g2, g) and np.array_equal(anc2, anc)
    specs = [("s", None), ("b", None), ("sigma", None), ("q", 0), ("q", 1), ("q", 2), ("q", 3),
             ("q", 4), ("I0", None)]
    for j, (field, idx) in enumerate(specs):
        fd = _fd_run(m, mv.frames, T, anc, field, idx, 1e-6)
        assert abs(fd - g[j]) <= 1e-5 * max(1.0, abs(g[j])), (oracle.GRAD_NAMES[j], fd, g[j])
