"""GPU parity of the gradient mode: derivatives of log p^ in theta = (s, b,
sigma_xi, q_x, q_y, q_vx, q_vy, q_I, I0) with the Philox noise and the
resampling ancestors held fixed, against the FP64 oracle (whose derivatives
tests/test_oracle_grad.py pins to finite differences)."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_5045_amd import synth

from parity import PATH_BOXES, PATH_ORIGINS, box_layout, pair, path_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H = 96, 80
GKW = dict(width=W, height=H, s=1.5, b=10.0, sigma=3.0, init_a=(36, 30, -1, -1, 20),
           init_b=(56, 50, 1, 1, 40), q=(0.5, 0.5, 0.2, 0.2, 1.0), seed=3)


@pytest.fixture(scope="module")
def ppf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_5045_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def movie():
    return synth.render_movie(W, H, 6, intensity=30.0, sigma=1.5, start_box=(40, 52, 34, 46),
                              seed=8)


def step_terms(m, obs, x, tang, w_src_lw):
    """Oracle d delta/d theta on the GPU's states with the oracle's tangents,
    and the scale sum_i w_i |v_i| of each component (for cancellation)."""
    l = oracle.loglik(m, obs, x) + w_src_lw
    w, _ = oracle.normalize(l)
    dll = oracle.loglik_grad(m, obs, x)
    g = oracle.step_grad(w, dll, tang)
    v = np.stack([dll[3], dll[4], dll[5], dll[0] * tang[0], dll[1] * tang[1], dll[0] * tang[3],
                  dll[1] * tang[5], dll[2] * tang[6], dll[2]])
    scale = (w[None, :] * np.abs(v)).sum(axis=1)
    return g, scale


def test_grad_mode_leaves_the_filter_unchanged(ppf, movie):
    p0, _ = pair(ppf, n=5000, **GKW)
    p1, _ = pair(ppf, n=5000, grad=1, **GKW)
    f0, f1 = ppf.Filter(p0), ppf.Filter(p1)
    frames = torch.from_numpy(movie.frames).cuda()
    for k in range(5):
        f0.step(frames[k])
        f1.step(frames[k])
        a, b = f0.particles(), f1.particles()
        for u, v in zip(a, b):
            assert np.array_equal(u, v), k
        assert f0.stats()["cum"] == f1.stats()["cum"]
    f0.close()
    f1.close()


# (s, I): patches 9 x 9, 11 x 11 (the differentiable workload's spot) and 13 x 13
SPOTS = [(1.5, 30.0), (1.7, 25.0), (2.0, 30.0)]


@pytest.mark.parametrize("s,I", SPOTS)
@pytest.mark.parametrize("n", [4096, 3001])
def test_grad_teacher_forced_vs_oracle(ppf, n, s, I):
    mv = synth.render_movie(W, H, 6, intensity=I, sigma=s, start_box=(40, 52, 34, 46), seed=8)
    p, m = pair(ppf, n=n, grad=1, **dict(GKW, s=s))
    assert m.P == 2 * int(math.floor(3 * s)) + 1
    f = ppf.Filter(p)
    frames = torch.from_numpy(mv.frames).cuda()
    tang = np.zeros((7, n))
    prev_anc = None
    for k in range(1, 6):
        f.step(frames[k - 1])
        x, lw, anc = f.particles()
        st = f.stats()
        assert st["k"] == k and st["resampled"]
        # tangents follow the GPU's ancestors of the previous step
        tang = oracle.propagate_tangent(m, k, tang, prev_anc)
        g_o, scale = step_terms(m, mv.frames[k - 1], x.astype(np.float64), tang,
                                np.full(n, -math.log(n)))
        _, g_gpu = f.grad()
        err = np.abs(g_gpu - g_o)
        assert np.all(err <= 2e-5 * (np.abs(g_o) + scale) + 1e-9), (k, g_gpu, g_o, scale)
        prev_anc = anc
    f.close()


@pytest.mark.parametrize("P", [9, 11, 13])
@pytest.mark.parametrize("way", ["sum", "tab", "glob"])
def test_grad_every_moment_path_vs_oracle(ppf, P, way):
    """One step from placed particles whose blocks all take one way to the
    moments (and a ragged last block), with log weights that flatten the
    posterior so that every particle counts in sum_i w_i d l_i / d theta;
    two of the boxes reach over the frame's edge."""
    s = {9: 1.5, 11: 1.7, 13: 2.0}[P]
    acx, acy = PATH_BOXES[P][way]
    assert path_of(P, acx, acy) == way
    mv = synth.render_movie(W, H, 1, intensity=30.0, sigma=s, start_box=(40, 52, 34, 46), seed=8)
    n = 2 * 256 + 37
    kw = dict(GKW, s=s, q=(1e-3,) * 5)
    p, m = pair(ppf, n=n, grad=1, **kw)
    assert m.P == P
    rng = np.random.default_rng(P)
    x = box_layout(rng, n, acx, acy, *PATH_ORIGINS[way])
    ll = oracle.loglik(m, mv.frames[0], x.astype(np.float64))
    lw = -ll - np.log(np.exp(-ll - (-ll).max()).sum()) - (-ll).max()
    f = ppf.Filter(p)
    f.set_particles(x, lw)
    f.step(torch.from_numpy(mv.frames[0]).cuda())
    xg, _, _ = f.particles()
    centres = np.floor(xg[:2].astype(np.float64) + 0.5)
    for b0 in range(0, n, 256):
        c = centres[:, b0:b0 + 256]
        assert (c[0].max() - c[0].min() + 1, c[1].max() - c[1].min() + 1) == (acx, acy)
    tang = oracle.propagate_tangent(m, 1, np.zeros((7, n)), None)
    g_o, scale = step_terms(m, mv.frames[0], xg.astype(np.float64), tang, lw)
    _, g_gpu = f.grad()
    err = np.abs(g_gpu - g_o)
    print(way, P, g_gpu, g_o, flush=True)
    assert np.all(err <= 2e-5 * (np.abs(g_o) + scale) + 1e-9), (g_gpu, g_o, scale)
    f.close()


def test_grad_full_run_vs_oracle_replay(ppf, movie):
    n, T = 3000, 6
    p, m = pair(ppf, n=n, grad=1, **GKW)
    f = ppf.Filter(p)
    frames = torch.from_numpy(movie.frames).cuda()
    ancs = []
    for k in range(T):
        f.step(frames[k])
        ancs.append(f.particles()[2])
    cum_gpu, _ = f.loglik()
    g_gpu, _ = f.grad()
    f.close()
    cum_o, g_o, anc_o = oracle.run_grad(m, movie.frames, T, anc_replay=np.stack(ancs))
    assert abs(cum_gpu - cum_o) <= 1e-6 * abs(cum_o)
    # scale: the oracle's gradient over the same run with |per-step terms|
    assert np.all(np.abs(g_gpu - g_o) <= 1e-4 * np.maximum(np.abs(g_o), 1.0)), (g_gpu, g_o)


def test_autograd_function_and_ascent(ppf):
    mv = synth.render_movie(128, 128, 8, intensity=25.0, sigma=1.7, start_box=(56, 72, 56, 72),
                            seed=12)
    frames = torch.from_numpy(mv.frames).cuda()
    # a too-wide spot model (s = 2.0, the generator's is 1.7) that still
    # tracks the spot; the patch stays 11 x 11 while s moves
    base = ppf.params(n_particles=1 << 16, width=128, height=128, psf_sigma=2.0, patch=11,
                      background=10.0, noise_sigma=3.0, init_a=(54, 54, -1, -1, 15),
                      init_b=(74, 74, 1, 1, 35), seed=2)
    theta = torch.tensor(ppf.theta_of(base), dtype=torch.float64, requires_grad=True)
    L = ppf.loglik(theta, frames, base)
    L.backward()
    f = ppf.Filter(ppf.params_at(base, theta.detach().tolist()))
    for k in range(frames.shape[0]):
        f.step(frames[k])
    g_ref, _ = f.grad()
    assert np.array_equal(theta.grad.numpy(), g_ref)
    assert float(L.detach()) == f.loglik()[0]
    f.close()
    # sign-gradient ascent on the spot width from 2.0 towards the generator's 1.7
    th = theta.detach().clone()
    start = float(L.detach())
    for _ in range(12):
        t = th.clone().requires_grad_(True)
        Lk = ppf.loglik(t, frames, base)
        Lk.backward()
        th[0] += 0.05 * float(torch.sign(t.grad[0]))
    assert abs(float(th[0]) - 1.7) < 0.15, float(th[0])
    assert float(ppf.loglik(th, frames, base)) > start
