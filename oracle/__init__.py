"""FP64 CPU oracle of the SIR filter step — TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import, call, link or execute anything under oracle/. The product package
never imports this module, and the two share no code.

This module only marshals numpy arrays into the plain C oracle
(ppf_oracle.c); all arithmetic of the method is in that file, in double
precision, following Algorithm 1 (Section 2), the models of Sections 6.1-6.2
and RNA (Section 3). The Kalman filter (kalman.py) and the exact rational
enumerations (brute.py) are further oracle pieces.
"""
import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_liboracle.so")
_lib = None


class _Model(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("obs_model", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("patch", ctypes.c_int32),
        ("s", ctypes.c_double),
        ("b", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("q", ctypes.c_double * 5),
        ("init_kind", ctypes.c_int32),
        ("resample", ctypes.c_int32),
        ("init_a", ctypes.c_double * 5),
        ("init_b", ctypes.c_double * 5),
        ("lg_r", ctypes.c_double * 3),
        ("ess_threshold", ctypes.c_double),
        ("rna_group", ctypes.c_int32),
        ("rna_moved", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("track", ctypes.c_uint32),
        ("arna_mu_min", ctypes.c_int32),
        ("arna_track", ctypes.c_double),
        ("arna_lost", ctypes.c_double),
    ]


def lib():
    """Load oracle/_liboracle.so, building it with gcc if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d, i32, u32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
        vp = ctypes.c_void_p
        L.orc_philox_many.argtypes = [ctypes.c_uint64, i64, vp, vp]
        L.orc_u24_open_hi.argtypes = [u32]
        L.orc_u24_open_hi.restype = d
        L.orc_u24_open_lo.argtypes = [u32]
        L.orc_u24_open_lo.restype = d
        L.orc_u53.argtypes = [u32, u32]
        L.orc_u53.restype = d
        L.orc_box_muller.argtypes = [u32, u32, P(d), P(d)]
        L.orc_normal_fields.argtypes = [vp, vp, vp]
        L.orc_resample_uniform.argtypes = [P(_Model), i64]
        L.orc_resample_uniform.restype = d
        L.orc_rna_uniform.argtypes = [P(_Model), i64, i64]
        L.orc_rna_uniform.restype = d
        L.orc_init.argtypes = [P(_Model), vp, vp]
        L.orc_init.restype = ctypes.c_int
        L.orc_init_indexed.restype = ctypes.c_int
        L.orc_zorder_key.argtypes = [u32, u32]
        L.orc_zorder_key.restype = u32
        L.orc_zorder_perm.argtypes = [P(_Model), i64, vp]
        L.orc_zorder_perm.restype = ctypes.c_int
        L.orc_propagate.argtypes = [P(_Model), i64, vp, vp, vp]
        L.orc_init_indexed.argtypes = [P(_Model), i64, vp, vp]
        L.orc_propagate_indexed.argtypes = [P(_Model), i64, vp, vp, vp]
        L.orc_loglik_spot.argtypes = [P(_Model), vp, vp, vp]
        L.orc_loglik_lg.argtypes = [P(_Model), vp, vp, vp]
        L.orc_normalize.argtypes = [i64, vp, vp, vp]
        L.orc_normalize.restype = ctypes.c_int
        L.orc_estimate.argtypes = [i64, vp, vp, vp]
        L.orc_resample_systematic.argtypes = [i64, vp, d, vp]
        L.orc_resample_rna.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp]
        L.orc_run.argtypes = [P(_Model), i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_run.restype = ctypes.c_int
        L.orc_propagate_tangent.argtypes = [P(_Model), i64, vp, vp, vp]
        L.orc_loglik_spot_grad.argtypes = [P(_Model), vp, vp, vp]
        L.orc_step_grad.argtypes = [i64, vp, vp, vp, vp]
        L.orc_run_grad.argtypes = [P(_Model), i32, vp, vp, vp, vp, P(d), vp]
        L.orc_run_grad.restype = ctypes.c_int
        L.orc_rpa_counts.argtypes = [i64, i32, vp, vp]
        L.orc_dlb_schedule.argtypes = [ctypes.c_int, i64, i32, vp, i64, vp]
        L.orc_dlb_schedule.restype = i64
        L.orc_resample_rpa.argtypes = [i64, i32, ctypes.c_int, vp, vp]
        L.orc_resample_rpa.restype = ctypes.c_int
        L.orc_ring_order.argtypes = [P(_Model), i64, i64, vp]
        L.orc_arna_lost.argtypes = [P(_Model), d, d]
        L.orc_arna_lost.restype = ctypes.c_int
        L.orc_resample_arna.argtypes = [i64, i32, i32, i32, d, vp, vp, vp, vp, vp, vp, P(i32),
                                        P(i32)]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Host threads of the per-particle loops (propagation, Eq. 4); returns
    the count in effect. The results do not depend on it."""
    return lib().orc_set_threads(int(n))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Model:
    """Filter parameters in the paper's notation; floats are taken as the
    float32 values the GPU library receives, widened exactly to float64."""
    n: int = 4096
    obs_model: int = 0            # 0 spot (Eqs. 3-4), 1 linear-Gaussian
    width: int = 128
    height: int = 128
    s: float = 1.5                # sigma_PSF
    b: float = 10.0               # I_bg
    sigma: float = 3.0            # sigma_xi
    patch: int = 0                # 0: 2 floor(3 s) + 1
    q: Sequence[float] = (0.5, 0.5, 0.1, 0.1, 1.0)
    init_kind: int = 0            # 0 uniform [a, b), 1 Gaussian N(a, b^2), 2 stratified,
                                  # 3 uniform in Z order
    init_a: Sequence[float] = (0.0, 0.0, -1.0, -1.0, 15.0)
    init_b: Sequence[float] = (128.0, 128.0, 1.0, 1.0, 45.0)
    lg_r: Sequence[float] = (1.0, 1.0, 1.0)
    resample: int = 0             # 0 systematic, 1 RNA, 2 ARNA
    ess_threshold: float = math.inf
    rna_group: int = 256
    rna_exchange: float = 0.1     # RNA: rho; ARNA: the largest exchange ratio
    seed: int = 1
    track: int = 0
    arna_min: float = 0.0         # ARNA: the smallest exchange ratio
    arna_track: float = 0.5       # ARNA: a group tracks when W_g >= arna_track / G
    arna_lost: float = 3.0        # ARNA: kappa of the lost test

    @property
    def P(self) -> int:
        return self.patch if self.patch else 2 * int(math.floor(3.0 * float(np.float32(self.s)))) + 1

    @property
    def rna_moved(self) -> int:
        return int(math.floor(float(np.float32(self.rna_exchange)) * self.rna_group))

    @property
    def arna_mu_min(self) -> int:
        return int(math.floor(float(np.float32(self.arna_min)) * self.rna_group))

    def c(self) -> _Model:
        f = lambda v: float(np.float32(v))  # noqa: E731  (exact widening of the fp32 value)
        m = _Model()
        m.n = self.n
        m.obs_model = self.obs_model
        m.width, m.height = self.width, self.height
        m.patch = self.P
        m.s, m.b, m.sigma = f(self.s), f(self.b), f(self.sigma)
        for d in range(5):
            m.q[d] = f(self.q[d])
            m.init_a[d] = f(self.init_a[d])
            m.init_b[d] = f(self.init_b[d])
        for d in range(3):
            m.lg_r[d] = f(self.lg_r[d])
        m.init_kind = self.init_kind
        m.resample = self.resample
        m.ess_threshold = float(self.ess_threshold)
        m.rna_group = self.rna_group
        m.rna_moved = self.rna_moved
        m.seed = self.seed
        m.track = self.track
        m.arna_mu_min = self.arna_mu_min
        m.arna_track = f(self.arna_track)
        m.arna_lost = f(self.arna_lost)
        return m


# ------------------------------------------------------------- RNG pieces
def philox(seed: int, ctr: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_many(seed, ctr.shape[0], _ptr(ctr), _ptr(out))
    return out


def u24_open_hi(a: int) -> float:
    return lib().orc_u24_open_hi(a)


def u24_open_lo(a: int) -> float:
    return lib().orc_u24_open_lo(a)


def u53(a: int, b: int) -> float:
    return lib().orc_u53(a, b)


def normal_fields(r) -> tuple:
    """(radius fields, angle fields) of one Philox block of 4 words."""
    w = np.ascontiguousarray(r, dtype=np.uint32).reshape(4)
    rad = np.empty(3, dtype=np.uint32)
    ang = np.empty(3, dtype=np.uint32)
    lib().orc_normal_fields(_ptr(w), _ptr(rad), _ptr(ang))
    return [int(v) for v in rad], [int(v) for v in ang]


def box_muller(rad: int, ang: int):
    """Box-Muller pair from a 24-bit radius field and an 18-bit angle field."""
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().orc_box_muller(rad, ang, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def resample_uniform(m: Model, k: int) -> float:
    c = m.c()
    return lib().orc_resample_uniform(ctypes.byref(c), k)


def rna_uniforms(m: Model, k: int) -> np.ndarray:
    c = m.c()
    G = m.n // m.rna_group
    return np.array([lib().orc_rna_uniform(ctypes.byref(c), g, k) for g in range(G)])


# ---------------------------------------------------------- filter pieces
def init(m: Model):
    c = m.c()
    x = np.empty(5 * m.n)
    lw = np.empty(m.n)
    if lib().orc_init(ctypes.byref(c), _ptr(x), _ptr(lw)) != 0:
        raise MemoryError("orc_init")
    return x.reshape(5, m.n), lw


def zorder_key(wx: int, wy: int) -> int:
    """Init kind 3's key: the Morton code of the top 16 bits of two words."""
    return int(lib().orc_zorder_key(wx, wy))


def zorder_perm(m: Model, n: int) -> np.ndarray:
    """Init kind 3: the draw index of the particle at each position."""
    c = m.c()
    out = np.empty(n, dtype=np.int64)
    if lib().orc_zorder_perm(ctypes.byref(c), n, _ptr(out)) != 0:
        raise MemoryError("orc_zorder_perm")
    return out


def propagate(m: Model, k: int, x_prev: np.ndarray, parent: Optional[np.ndarray] = None, c=None):
    c = m.c() if c is None else c
    xp = np.ascontiguousarray(x_prev, dtype=np.float64).reshape(5, m.n)
    par = None if parent is None else np.ascontiguousarray(parent, dtype=np.int32)
    xn = np.empty((5, m.n))
    lib().orc_propagate(ctypes.byref(c), k, _ptr(xp), _ptr(par), _ptr(xn))
    return xn


def init_indexed(m: Model, n_total: int, index: np.ndarray) -> np.ndarray:
    """Initial states of particles `index` of a run with n_total particles;
    m.n must equal len(index)."""
    c = m.c()
    idx = np.ascontiguousarray(index, dtype=np.int64)
    assert idx.size == m.n
    x = np.empty((5, m.n))
    if lib().orc_init_indexed(ctypes.byref(c), n_total, _ptr(idx), _ptr(x)) != 0:
        raise MemoryError("orc_init_indexed")
    return x


def propagate_indexed(m: Model, k: int, index: np.ndarray, parents: np.ndarray) -> np.ndarray:
    """Propagate particles `index` (their random numbers) from the given
    parent states (5, len(index)); m.n must equal len(index)."""
    c = m.c()
    idx = np.ascontiguousarray(index, dtype=np.int64)
    xp = np.ascontiguousarray(parents, dtype=np.float64).reshape(5, m.n)
    xn = np.empty((5, m.n))
    lib().orc_propagate_indexed(ctypes.byref(c), k, _ptr(idx), _ptr(xp), _ptr(xn))
    return xn


def loglik(m: Model, obs: np.ndarray, x: np.ndarray, c=None) -> np.ndarray:
    c = m.c() if c is None else c
    z = np.ascontiguousarray(obs, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(5, m.n)
    ll = np.empty(m.n)
    fn = lib().orc_loglik_spot if m.obs_model == 0 else lib().orc_loglik_lg
    fn(ctypes.byref(c), _ptr(z), _ptr(xx), _ptr(ll))
    return ll


def normalize(lwt: np.ndarray):
    """Returns (w, {m, log_sum, ess, delta}) or raises FloatingPointError."""
    l = np.ascontiguousarray(lwt, dtype=np.float64)
    w = np.empty_like(l)
    st = np.empty(4)
    if lib().orc_normalize(l.size, _ptr(l), _ptr(w), _ptr(st)) != 0:
        raise FloatingPointError("no finite normaliser")
    return w, dict(m=st[0], log_sum=st[1], ess=st[2], delta=st[3])


def estimate(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    ww = np.ascontiguousarray(w, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(5)
    lib().orc_estimate(ww.size, _ptr(ww), _ptr(xx), _ptr(out))
    return out


def resample_systematic(w: np.ndarray, u: float) -> np.ndarray:
    ww = np.ascontiguousarray(w, dtype=np.float64)
    anc = np.empty(ww.size, dtype=np.int32)
    lib().orc_resample_systematic(ww.size, _ptr(ww), float(u), _ptr(anc))
    return anc


def resample_rna(w: np.ndarray, group: int, moved: int, u_g: np.ndarray):
    """Returns (anc, lwg per group, lw per slot)."""
    ww = np.ascontiguousarray(w, dtype=np.float64)
    n = ww.size
    ug = np.ascontiguousarray(u_g, dtype=np.float64)
    anc = np.empty(n, dtype=np.int32)
    lwg = np.empty(n // group)
    lws = np.empty(n)
    lib().orc_resample_rna(n, group, moved, _ptr(ww), _ptr(ug), _ptr(anc), _ptr(lwg), _ptr(lws))
    return anc, lwg, lws


# ------------------------------------------------------------ ARNA
def ring_order(m: Model, key: int, G: int) -> np.ndarray:
    """ARNA's ring: the group at each ring position (key 0: index order)."""
    out = np.empty(G, dtype=np.int64)
    lib().orc_ring_order(ctypes.byref(m.c()), int(key), int(G), _ptr(out))
    return out


def arna_lost(m: Model, delta: float, ref: float) -> bool:
    """ARNA's lost test of a frame's log-likelihood increment against that of
    the last frame that was not lost."""
    return bool(lib().orc_arna_lost(ctypes.byref(m.c()), float(delta), float(ref)))


def resample_arna(w: np.ndarray, group: int, mu_min: int, mu_max: int, theta: float,
                  u_g: np.ndarray, order: np.ndarray):
    """(ancestors, log(W_g / n), per-slot log weights, tracking groups, slots
    exchanged) of ARNA's resampling with ring `order`."""
    n = w.size
    ww = np.ascontiguousarray(w, dtype=np.float64)
    ug = np.ascontiguousarray(u_g, dtype=np.float64)
    od = np.ascontiguousarray(order, dtype=np.int64)
    anc = np.empty(n, dtype=np.int32)
    lwg = np.empty(n // group)
    lws = np.empty(n)
    t, mu = ctypes.c_int32(), ctypes.c_int32()
    with np.errstate(divide="ignore"):
        lib().orc_resample_arna(n, group, mu_min, mu_max, float(theta), _ptr(ww), _ptr(ug),
                                _ptr(od), _ptr(anc), _ptr(lwg), _ptr(lws), ctypes.byref(t),
                                ctypes.byref(mu))
    return anc, lwg, lws, t.value, mu.value


@dataclass
class RunResult:
    mean: np.ndarray
    ess: np.ndarray
    delta: np.ndarray
    resampled: np.ndarray
    x: np.ndarray
    lw: np.ndarray
    anc: np.ndarray
    status: int = 0
    extra: dict = field(default_factory=dict)


def run(m: Model, obs: np.ndarray, T: Optional[int] = None) -> RunResult:
    """A whole filter run (Algorithm 1) over T observations."""
    z = np.ascontiguousarray(obs, dtype=np.float32)
    if T is None:
        T = z.shape[0]
    c = m.c()
    mean = np.zeros((T, 5))
    ess = np.zeros(T)
    delta = np.zeros(T)
    res = np.zeros(T, dtype=np.int32)
    x = np.zeros((5, m.n))
    lw = np.zeros(m.n)
    anc = np.zeros(m.n, dtype=np.int32)
    arna = np.zeros((T, 3), dtype=np.int64)
    st = lib().orc_run(ctypes.byref(c), T, _ptr(z), _ptr(mean), _ptr(ess), _ptr(delta), _ptr(res),
                       _ptr(x), _ptr(lw), _ptr(anc), _ptr(arna))
    extra = {"arna": arna} if m.resample == 2 else {}
    return RunResult(mean, ess, delta, res, x, lw, anc, st, extra)


# ------------------------------------------------------------ derivatives
GRAD_NAMES = ("s", "b", "sigma", "q_x", "q_y", "q_vx", "q_vy", "q_I", "I0")


def propagate_tangent(m: Model, k: int, t_prev: np.ndarray, parent: Optional[np.ndarray] = None):
    """Tangents (7, n) of frame k's states in q from the parents' (see
    orc_propagate_tangent)."""
    c = m.c()
    tp = np.ascontiguousarray(t_prev, dtype=np.float64).reshape(7, m.n)
    par = None if parent is None else np.ascontiguousarray(parent, dtype=np.int32)
    out = np.empty((7, m.n))
    lib().orc_propagate_tangent(ctypes.byref(c), k, _ptr(tp), _ptr(par), _ptr(out))
    return out


def loglik_grad(m: Model, obs: np.ndarray, x: np.ndarray, c=None) -> np.ndarray:
    """dl/d(x, y, I0, s, b, sigma) per particle, (6, n). `c` may give the
    C model directly (fp64 fields, e.g. perturbed off the fp32 grid)."""
    c = m.c() if c is None else c
    fr = np.ascontiguousarray(obs, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(5, m.n)
    out = np.empty((6, m.n))
    lib().orc_loglik_spot_grad(ctypes.byref(c), _ptr(fr), _ptr(xx), _ptr(out))
    return out


def step_grad(w: np.ndarray, dll: np.ndarray, tang: np.ndarray) -> np.ndarray:
    """sum_i w_i dl_i/dtheta, theta as GRAD_NAMES."""
    n = w.size
    ww = np.ascontiguousarray(w, dtype=np.float64)
    dd = np.ascontiguousarray(dll, dtype=np.float64).reshape(6, n)
    tt = np.ascontiguousarray(tang, dtype=np.float64).reshape(7, n)
    g = np.empty(9)
    lib().orc_step_grad(n, _ptr(ww), _ptr(dd), _ptr(tt), _ptr(g))
    return g


def run_grad(m: Model, frames: np.ndarray, T: int, anc_replay: Optional[np.ndarray] = None,
             trace: bool = False, c=None):
    """(cum, grad (9,), ancestors (T, n)[, states (T, 5, n)]) of a whole run
    with systematic resampling at every step; anc_replay fixes the ancestors.
    `c` may give the C model directly."""
    c = m.c() if c is None else c
    fr = np.ascontiguousarray(frames[:T], dtype=np.float32)
    rep_ = None if anc_replay is None else np.ascontiguousarray(anc_replay, dtype=np.int32)
    anc = np.empty((T, m.n), dtype=np.int32)
    xt = np.empty((T, 5, m.n)) if trace else None
    cum = ctypes.c_double()
    g = np.empty(9)
    st = lib().orc_run_grad(ctypes.byref(c), T, _ptr(fr), _ptr(rep_), _ptr(anc), _ptr(xt),
                            ctypes.byref(cum), _ptr(g))
    if st != 0:
        raise FloatingPointError(f"orc_run_grad returned {st}")
    return (cum.value, g, anc, xt) if trace else (cum.value, g, anc)


# ------------------------------------------------------ RPA and DLB (Section 4)
DLB_GS, DLB_SGS, DLB_LGS = 0, 1, 2


def rpa_counts(anc_sys: np.ndarray, group: int) -> np.ndarray:
    a = np.ascontiguousarray(anc_sys, dtype=np.int32)
    out = np.empty(a.size // group, dtype=np.int32)
    lib().orc_rpa_counts(a.size, group, _ptr(a), _ptr(out))
    return out


def dlb_schedule(kind: int, counts: np.ndarray, n: int) -> np.ndarray:
    """(m, 3) int32 entries (sender group, receiver group, particles)."""
    c = np.ascontiguousarray(counts, dtype=np.int32)
    cap = 2 * c.size + 1
    out = np.empty((cap, 3), dtype=np.int32)
    m = lib().orc_dlb_schedule(kind, c.size, n, _ptr(c), cap, _ptr(out))
    if m < 0:
        raise RuntimeError("schedule capacity exceeded")
    return out[:m].copy()


def route_rpa(anc_sys: np.ndarray, group: int, kind: int) -> np.ndarray:
    """RPA ancestors (kind GS or SGS) from the global systematic ancestors."""
    a = np.ascontiguousarray(anc_sys, dtype=np.int32)
    out = np.empty(a.size, dtype=np.int32)
    st = lib().orc_resample_rpa(a.size, group, kind, _ptr(a), _ptr(out))
    if st != 0:
        raise RuntimeError("RPA left a group unbalanced")
    return out


def resample_rpa(w: np.ndarray, u: float, group: int, kind: int) -> np.ndarray:
    """RPA ancestors (kind GS or SGS) for normalised weights w with the
    systematic uniform u."""
    return route_rpa(resample_systematic(w, u), group, kind)
