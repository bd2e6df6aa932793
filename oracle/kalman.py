"""Kalman filter of the linear-Gaussian variant — TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
anything under oracle/.

For a linear state-space model with Gaussian noise the Bayes recursion of
Eqs. 1-2 (Section 2) is closed: prior and posterior stay Gaussian, and the
normaliser p(z_k | Z^{k-1}) of Eq. 1 is a Gaussian density. The particle
filter's MMSE estimate (Section 2) and its log-likelihood estimate must
converge to these as N grows. The model is the near-constant-velocity
dynamics of Section 6.1 (unit frame interval) observed as (x, y, I0) plus
independent Gaussian noise.
"""
import numpy as np

from . import Model


def matrices(m: Model):
    """F, Q, H, R, prior mean and covariance, all float64 from the fp32
    parameter values."""
    f32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)  # noqa: E731
    F = np.eye(5)
    F[0, 2] = 1.0
    F[1, 3] = 1.0
    Q = np.diag(f32(m.q) ** 2)
    H = np.zeros((3, 5))
    H[0, 0] = H[1, 1] = H[2, 4] = 1.0
    R = np.diag(f32(m.lg_r) ** 2)
    mu0 = f32(m.init_a)
    P0 = np.diag(f32(m.init_b) ** 2)
    return F, Q, H, R, mu0, P0


def run(m: Model, obs: np.ndarray):
    """Kalman filter over obs (T, 3). Returns (means (T, 5), covariances
    (T, 5, 5), log p(z_k | z_1:k-1) per step (T,))."""
    F, Q, H, R, x, P = matrices(m)
    z_all = np.asarray(obs, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    T = z_all.shape[0]
    means = np.zeros((T, 5))
    covs = np.zeros((T, 5, 5))
    ll = np.zeros(T)
    for k in range(T):
        x = F @ x                       # prior mean, Eq. 2
        P = F @ P @ F.T + Q
        S = H @ P @ H.T + R             # covariance of p(z_k | Z^{k-1})
        e = z_all[k] - H @ x
        sign, logdet = np.linalg.slogdet(2.0 * np.pi * S)
        ll[k] = -0.5 * (e @ np.linalg.solve(S, e) + logdet)
        K = np.linalg.solve(S, H @ P).T  # gain P H^T S^-1 (S symmetric)
        x = x + K @ e                   # posterior, Eq. 1
        P = (np.eye(5) - K @ H) @ P
        P = 0.5 * (P + P.T)
        means[k], covs[k] = x, P
    return means, covs, ll
