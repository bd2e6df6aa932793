"""Seeded synthetic inputs shaped like the paper's tracking movies.

The paper evaluates on synthetic fluorescence-microscopy movies: bright
Gaussian spots (Eq. 3) moving under near-constant-velocity dynamics
(Section 6.1) on a constant background with additive noise (Section 6.3,
512 x 512 frames, 50 frames). Those movies are not published, so this module
renders stand-ins from a seed. It is input generation only: the filter's
arithmetic lives in the HIP kernels (product) and in the oracle (tests), and
neither imports the other; this module is shared by both only as a source of
inputs.

Recipe (numpy float64, stored as float32):
  truth   p_1 ~ U(start box); v_1 ~ U[-vmax, vmax]^2 per spot; I_1 = I;
          p_k = p_{k-1} + v_{k-1} + eta_k, eta_k ~ N(0, jitter^2 I_2);
          v_k = v_{k-1} + zeta_k, zeta_k ~ N(0, vel_jitter^2 I_2);
          I_k = I_{k-1} + iota_k, iota_k ~ N(0, int_jitter^2)
          (vel_jitter = int_jitter = 0 by default: constant velocity and
          intensity; with all three set, the truth follows the filter's own
          near-constant-velocity model with q = (jitter, jitter, vel_jitter,
          vel_jitter, int_jitter)).
  frame   Z_k[y][x] = b + sum_spots I_k exp(-((x - px)^2 + (y - py)^2) / (2 s^2))
          + noise_sd * N(0, 1), pixel (x, y) at integer coordinates.
"""
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


@dataclass
class Movie:
    frames: np.ndarray      # (T, H, W) float32
    truth: np.ndarray       # (T, n_spots, 2) float64 spot centres per frame
    intensity: np.ndarray   # (n_spots,) float64
    sigma: np.ndarray       # (n_spots,) float64 PSF widths
    velocity: np.ndarray    # (n_spots, 2) float64 initial velocities
    intensity_track: Optional[np.ndarray] = None  # (T, n_spots) per-frame intensities


def render_movie(width: int, height: int, T: int, *, n_spots: int = 1,
                 intensity=30.0, sigma=1.5, background: float = 10.0,
                 noise_sd: float = 3.0, vmax: float = 1.0, jitter: float = 0.3,
                 vel_jitter: float = 0.0, int_jitter: float = 0.0,
                 start_box: Optional[Sequence[float]] = None, seed: int = 1) -> Movie:
    """Render T frames. intensity/sigma: a number or a (lo, hi) range drawn
    uniformly per spot. start_box: (x0, x1, y0, y1); default the central half
    [W/4, 3W/4] x [H/4, 3H/4] of the frame."""
    rng = np.random.default_rng(seed)
    if start_box is None:
        start_box = (width / 4, 3 * width / 4, height / 4, 3 * height / 4)

    def per_spot(v):
        if np.ndim(v) == 0:
            return np.full(n_spots, float(v))
        return rng.uniform(float(v[0]), float(v[1]), n_spots)

    I = per_spot(intensity)
    s = per_spot(sigma)
    p = np.stack([rng.uniform(start_box[0], start_box[1], n_spots),
                  rng.uniform(start_box[2], start_box[3], n_spots)], axis=1)
    vel = rng.uniform(-vmax, vmax, (n_spots, 2))
    vel0 = vel.copy()
    Ik = I.copy()
    truth = np.zeros((T, n_spots, 2))
    itrack = np.zeros((T, n_spots))
    frames = np.empty((T, height, width), dtype=np.float32)
    for k in range(T):
        if k > 0:
            p = p + vel + rng.normal(0.0, jitter, (n_spots, 2))
            # (no draws when the walks are off, so default movies are unchanged)
            if vel_jitter > 0.0:
                vel = vel + rng.normal(0.0, vel_jitter, (n_spots, 2))
            if int_jitter > 0.0:
                Ik = Ik + rng.normal(0.0, int_jitter, n_spots)
        truth[k] = p
        itrack[k] = Ik
        img = np.full((height, width), float(background))
        for j in range(n_spots):
            r = int(np.ceil(8.0 * s[j]))
            cx, cy = int(np.floor(p[j, 0])), int(np.floor(p[j, 1]))
            x0, x1 = max(cx - r, 0), min(cx + r + 1, width)
            y0, y1 = max(cy - r, 0), min(cy + r + 1, height)
            if x0 >= x1 or y0 >= y1:
                continue
            xs = np.arange(x0, x1, dtype=np.float64)
            ys = np.arange(y0, y1, dtype=np.float64)
            gx = np.exp(-((xs - p[j, 0]) ** 2) / (2.0 * s[j] ** 2))
            gy = np.exp(-((ys - p[j, 1]) ** 2) / (2.0 * s[j] ** 2))
            img[y0:y1, x0:x1] += Ik[j] * gy[:, None] * gx[None, :]
        img += noise_sd * rng.standard_normal((height, width))
        frames[k] = img.astype(np.float32)
    return Movie(frames, truth, I, s, vel0, itrack)


@dataclass
class LinearGaussianTrack:
    obs: np.ndarray    # (T, 3) float32 observations of (x, y, I0)
    states: np.ndarray  # (T, 5) float64 true states


def linear_gaussian_track(T: int, mean0: Sequence[float], sd0: Sequence[float],
                          q: Sequence[float], r: Sequence[float], seed: int = 1
                          ) -> LinearGaussianTrack:
    """States from the near-constant-velocity model with Gaussian noise (unit
    frame interval), observed as (x, y, I0) plus Gaussian noise of sds r."""
    rng = np.random.default_rng(seed)
    x = np.asarray(mean0, float) + np.asarray(sd0, float) * rng.standard_normal(5)
    q = np.asarray(q, float)
    r = np.asarray(r, float)
    states = np.zeros((T, 5))
    obs = np.zeros((T, 3), dtype=np.float32)
    for k in range(T):
        x = x.copy()
        x[0] += x[2]
        x[1] += x[3]
        x = x + q * rng.standard_normal(5)
        states[k] = x
        obs[k] = (x[[0, 1, 4]] + r * rng.standard_normal(3)).astype(np.float32)
    return LinearGaussianTrack(obs, states)


# Workloads of the benchmark configurations (frame size, frames, particles).
CONFIGS = {
    "sir_128_n4096": dict(width=128, height=128, T=10, n=4096, s=1.5, I=30.0, P=9,
                          ess_threshold=float("inf")),
    "sir_512_n1m": dict(width=512, height=512, T=50, n=1 << 20, s=1.5, I=30.0, P=9,
                        ess_threshold=float(1 << 19)),
    "sir_1024_n38m": dict(width=1024, height=1024, T=20, n=38_000_000, s=2.0, I=30.0, P=13,
                          ess_threshold=float("inf")),
}
