"""MI355X (gfx950) SIR particle filter — Python binding of libppf.so.

A thin ctypes layer over the C ABI in include/ppf.h: it marshals arguments
and lets PyTorch provide device memory and the HIP stream. Every step of the
filter (Algorithm 1 of the PPF paper with the models of its Section 6) runs
in the library's HIP kernels; nothing here computes the method, and there is
no CPU fallback: without the built library every entry point raises.

    import torch, paper_1310_5045_amd as ppf
    p = ppf.params(n_particles=1 << 20, width=512, height=512)
    f = ppf.Filter(p)
    f.step(frame_tensor)          # async on the current stream
    mean, ess = f.estimate()      # syncs
"""
import ctypes
import math
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppf.so")

PPF_OK, PPF_EINVAL, PPF_ENOMEM, PPF_EDEVICE, PPF_ESTATE, PPF_ENUMERIC, PPF_ENOTIMPL = (
    0, -1, -2, -3, -4, -5, -6)
RESAMPLE_SYSTEMATIC, RESAMPLE_RNA, RESAMPLE_RPA, RESAMPLE_ARNA = 0, 1, 2, 3
DLB_GS, DLB_SGS, DLB_LGS = 0, 1, 2
STATIC_MAX_N = 1 << 22  # weights the allocation-free resampler takes
OBS_SPOT, OBS_LINEAR_GAUSSIAN = 0, 1
INIT_UNIFORM, INIT_GAUSSIAN, INIT_STRATIFIED, INIT_UNIFORM_ZORDER = 0, 1, 2, 3
MAX_PATCH = 25
NUM_SHAPES, TUNE_MAX = 2, 3  # step-kernel workgroup shapes; tuning candidates at most
# theta of ppf_grad, in order
GRAD_NAMES = ("psf_sigma", "background", "noise_sigma", "q_x", "q_y", "q_vx", "q_vy", "q_I", "I0")


class Params(ctypes.Structure):
    """Mirror of ppf_params (include/ppf.h)."""
    _fields_ = [
        ("state_dim", ctypes.c_int32),
        ("obs_model", ctypes.c_int32),
        ("n_particles", ctypes.c_int64),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("psf_sigma", ctypes.c_float),
        ("background", ctypes.c_float),
        ("noise_sigma", ctypes.c_float),
        ("patch", ctypes.c_int32),
        ("q", ctypes.c_float * 5),
        ("init_kind", ctypes.c_int32),
        ("init_a", ctypes.c_float * 5),
        ("init_b", ctypes.c_float * 5),
        ("lg_r", ctypes.c_float * 3),
        ("resample", ctypes.c_int32),
        ("ess_threshold", ctypes.c_double),
        ("rna_group", ctypes.c_int32),
        ("rna_exchange", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("track_id", ctypes.c_uint32),
        ("grad", ctypes.c_int32),
        ("dlb", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("arna_min", ctypes.c_float),
        ("arna_track", ctypes.c_float),
        ("arna_lost", ctypes.c_float),
        ("arna_pad", ctypes.c_int32),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class Stats(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("resampled", ctypes.c_int32),
        ("rolled_back", ctypes.c_int32),
        ("ess", ctypes.c_double),
        ("max_logw", ctypes.c_double),
        ("log_sum", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("cum", ctypes.c_double),
        ("mean", ctypes.c_double * 5),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class PPFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ppf error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "ppf_version": (ctypes.c_char_p, []),
    "ppf_params_size": (ctypes.c_size_t, []),
    "ppf_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "ppf_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "ppf_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ppf_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "ppf_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ppf_set_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ppf_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "ppf_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "ppf_estimate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "ppf_loglik": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    "ppf_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ppf_arna_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "ppf_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_get_particles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "ppf_set_particles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ppf_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelTime), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "ppf_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ppf_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ppf_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "ppf_philox4x32_10": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p]),
    "ppf_resample_scratch_bytes": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "ppf_resample_systematic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p]),
    "ppf_resample_systematic_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                                      ctypes.c_double, ctypes.c_void_p,
                                                      ctypes.c_void_p]),
    "ppf_resample_rna": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "ppf_dlb_schedule": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "ppf_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "ppf_batch_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "ppf_step_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ppf_batch_set_shapes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ppf_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "ppf_batch_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats), ctypes.c_int32]),
    "ppf_batch_get_particles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "ppf_batch_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ppf_batch_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelTime),
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "ppf_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ppf_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}


def lib():
    """The loaded libppf.so. Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.ppf_params_size() != ctypes.sizeof(Params):
            raise RuntimeError("ppf_params layout mismatch between libppf.so and the binding")
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().ppf_error_string(code).decode()


def _check(rc: int, handle=None, last_error=None):
    if rc != PPF_OK:
        msg = error_string(rc)
        if handle is not None:
            detail = (last_error or lib().ppf_last_error)(handle)
            if detail:
                msg += f" ({detail.decode()})"
        raise PPFError(rc, msg)


def params(**kw) -> Params:
    """ppf_params with the library defaults, overridden by keyword arguments
    (array fields accept sequences)."""
    p = Params()
    _check(lib().ppf_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        cur = getattr(p, k)
        if isinstance(cur, ctypes.Array):
            if len(v) != len(cur):
                raise ValueError(f"{k} needs {len(cur)} values")
            for j, x in enumerate(v):
                cur[j] = x
        else:
            setattr(p, k, v)
    return p


def workspace_bytes(p: Params) -> int:
    n = ctypes.c_size_t()
    _check(lib().ppf_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def patch_size(p: Params) -> int:
    return p.patch if p.patch else 2 * int(math.floor(3.0 * float(np.float32(p.psf_sigma)))) + 1


def _stream_ptr(stream) -> int:
    return stream.cuda_stream if stream is not None else 0


class Filter:
    """One SIR filter whose state lives in a torch-allocated device
    workspace; all launches go to `stream` (default: the current stream)."""

    def __init__(self, p: Params, device=None, stream=None):
        import torch
        self.torch = torch
        self.p = p
        self.n = int(p.n_particles)
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = workspace_bytes(p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = lib().ppf_create(ctypes.byref(p), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                              ctypes.c_void_p(_stream_ptr(self.stream)), ctypes.byref(h))
        _check(rc)
        self._h = h

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().ppf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        if not self._h:
            raise PPFError(PPF_ESTATE, "filter closed")
        return self._h

    # -- the step
    def _obs_ptr(self, obs):
        t = self.torch
        if not isinstance(obs, t.Tensor) or obs.device.type != "cuda":
            raise TypeError("observation must be a CUDA tensor")
        if obs.dtype != t.float32 or not obs.is_contiguous():
            raise TypeError("observation must be contiguous float32")
        need = 3 if self.p.obs_model == OBS_LINEAR_GAUSSIAN else self.p.width * self.p.height
        if obs.numel() != need:
            raise ValueError(f"observation must have {need} elements")
        return ctypes.c_void_p(obs.data_ptr())

    def step(self, obs):
        """One filter step on a device observation; async."""
        _check(lib().ppf_step(self.handle, self._obs_ptr(obs)), self.handle)

    def reset(self):
        _check(lib().ppf_reset(self.handle), self.handle)

    def sync(self):
        _check(lib().ppf_sync(self.handle), self.handle)

    def estimate(self) -> Tuple[np.ndarray, float]:
        mean = (ctypes.c_double * 5)()
        ess = ctypes.c_double()
        _check(lib().ppf_estimate(self.handle, mean, ctypes.byref(ess)), self.handle)
        return np.array(mean[:]), ess.value

    def loglik(self) -> Tuple[float, float]:
        cum, last = ctypes.c_double(), ctypes.c_double()
        _check(lib().ppf_loglik(self.handle, ctypes.byref(cum), ctypes.byref(last)), self.handle)
        return cum.value, last.value

    def stats(self) -> dict:
        s = Stats()
        _check(lib().ppf_stats(self.handle, ctypes.byref(s)), self.handle)
        return _stats_dict(s)

    def arna_state(self) -> dict:
        """ARNA after the last committed step: ring_key (the frame of the
        latest loss, 0 before any), lost, tracking groups and slots exchanged
        of its resampling. Syncs."""
        key, lost, t, mu = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ppf_arna_state(self.handle, ctypes.byref(key), ctypes.byref(lost),
                                    ctypes.byref(t), ctypes.byref(mu)), self.handle)
        return dict(ring_key=key.value, lost=bool(lost.value), tracking=t.value, moved=mu.value)

    def grad(self) -> Tuple[np.ndarray, np.ndarray]:
        """(d cum / d theta, the last step's term), theta as GRAD_NAMES; the
        filter must have been created with grad=1. Syncs."""
        cum = np.empty(len(GRAD_NAMES))
        last = np.empty(len(GRAD_NAMES))
        _check(lib().ppf_grad(self.handle, cum.ctypes.data_as(ctypes.c_void_p),
                              last.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return cum, last

    def particles(self):
        """(state (5, N) float32, normalised log weights (N,) float64,
        ancestors (N,) int32) of the last committed step, on the host."""
        x = np.empty((5, self.n), dtype=np.float32)
        lw = np.empty(self.n, dtype=np.float64)
        anc = np.empty(self.n, dtype=np.int32)
        _check(lib().ppf_get_particles(self.handle, x.ctypes.data_as(ctypes.c_void_p),
                                       lw.ctypes.data_as(ctypes.c_void_p),
                                       anc.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return x, lw, anc

    def set_particles(self, state: np.ndarray, logw: np.ndarray):
        x = np.ascontiguousarray(state, dtype=np.float32).reshape(5, self.n)
        lw = np.ascontiguousarray(logw, dtype=np.float64).reshape(self.n)
        _check(lib().ppf_set_particles(self.handle, x.ctypes.data_as(ctypes.c_void_p),
                                       lw.ctypes.data_as(ctypes.c_void_p)), self.handle)

    def gather(self, out=None):
        """Resampled states x_k^i = x~_k^{s(i)} as a (5, N) float32 device
        tensor; async."""
        t = self.torch
        if out is None:
            out = t.empty((5, self.n), dtype=t.float32, device=self.device)
        if out.dtype != t.float32 or not out.is_contiguous() or out.numel() != 5 * self.n:
            raise ValueError("out must be a contiguous float32 tensor of 5*N elements")
        _check(lib().ppf_gather(self.handle, ctypes.c_void_p(out.data_ptr())), self.handle)
        return out

    def graph(self, on: bool = True):
        """Graph mode: steps replay one recorded HIP graph of their launches."""
        _check(lib().ppf_set_graph(self.handle, 1 if on else 0), self.handle)

    def set_shape(self, shape: int):
        """Workgroup shape of the step kernel (see PPF_NUM_SHAPES)."""
        _check(lib().ppf_set_shape(self.handle, int(shape)), self.handle)

    def autotune(self, obs, reps: int = 5):
        """Times each step-kernel shape on the current particles and frame
        `obs`, keeps the fastest; returns (ms per launch by candidate, chosen)."""
        ms = (ctypes.c_double * TUNE_MAX)()
        n, ch = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ppf_autotune(self.handle, self._obs_ptr(obs), int(reps), ms,
                                  ctypes.byref(n), ctypes.byref(ch)), self.handle)
        return list(ms[:n.value]), ch.value

    # -- timing
    def profile(self, on: bool = True):
        _check(lib().ppf_profile_enable(self.handle, 1 if on else 0), self.handle)

    def kernel_times(self) -> dict:
        buf = (KernelTime * 16)()
        n = ctypes.c_int()
        _check(lib().ppf_profile_read(self.handle, buf, 16, ctypes.byref(n)), self.handle)
        return {buf[j].name.decode(): (buf[j].launches, buf[j].total_ms) for j in range(n.value)}


def _stats_dict(s: Stats) -> dict:
    return dict(k=s.k, resampled=bool(s.resampled), rolled_back=s.rolled_back, ess=s.ess,
                max_logw=s.max_logw, log_sum=s.log_sum, delta=s.delta, cum=s.cum,
                mean=np.array(s.mean[:]))


def batch_workspace_bytes(ps) -> int:
    arr = (Params * len(ps))(*ps)
    n = ctypes.c_size_t()
    _check(lib().ppf_batch_workspace_bytes(arr, len(ps), ctypes.byref(n)))
    return n.value


class Batch:
    """Independent filters (tracks), one per Params, stepped together on one
    shared frame stream by the library's batched launches. Track t behaves
    exactly as Filter(ps[t]) would."""

    def __init__(self, ps, device=None, stream=None):
        import torch
        self.torch = torch
        self.ps = list(ps)
        self.count = len(self.ps)
        self.n = [int(p.n_particles) for p in self.ps]
        self.device = torch.device(device if device is not None else "cuda")
        arr = (Params * self.count)(*self.ps)
        nbytes = batch_workspace_bytes(self.ps)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().ppf_batch_create(arr, self.count, ctypes.c_void_p(self.workspace.data_ptr()),
                                      nbytes, ctypes.c_void_p(_stream_ptr(self.stream)),
                                      ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ppf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise PPFError(PPF_ESTATE, "batch closed")
        return self._h

    def _chk(self, rc):
        _check(rc, self.handle, lib().ppf_batch_last_error)

    def _obs_ptr(self, obs):
        t = self.torch
        if not isinstance(obs, t.Tensor) or obs.device.type != "cuda":
            raise TypeError("observation must be a CUDA tensor")
        if obs.dtype != t.float32 or not obs.is_contiguous():
            raise TypeError("observation must be contiguous float32")
        if obs.numel() != self.ps[0].width * self.ps[0].height:
            raise ValueError("observation must be one H x W frame")
        return ctypes.c_void_p(obs.data_ptr())

    def step(self, obs):
        """One step of every track on a device frame; async."""
        self._chk(lib().ppf_step_batched(self.handle, self._obs_ptr(obs)))

    def reset(self):
        self._chk(lib().ppf_batch_reset(self.handle))

    def stats(self):
        buf = (Stats * self.count)()
        self._chk(lib().ppf_batch_stats(self.handle, buf, self.count))
        return [_stats_dict(buf[j]) for j in range(self.count)]

    def particles(self, track: int):
        n = self.n[track]
        x = np.empty((5, n), dtype=np.float32)
        lw = np.empty(n, dtype=np.float64)
        anc = np.empty(n, dtype=np.int32)
        self._chk(lib().ppf_batch_get_particles(self.handle, track,
                                                x.ctypes.data_as(ctypes.c_void_p),
                                                lw.ctypes.data_as(ctypes.c_void_p),
                                                anc.ctypes.data_as(ctypes.c_void_p)))
        return x, lw, anc

    def graph(self, on: bool = True):
        """Graph mode: batched steps replay one recorded HIP graph."""
        self._chk(lib().ppf_batch_set_graph(self.handle, 1 if on else 0))

    def set_shapes(self, candidate: int):
        """Workgroup shapes of the fused step launches (candidates 0-2)."""
        self._chk(lib().ppf_batch_set_shapes(self.handle, int(candidate)))

    def autotune(self, obs, reps: int = 5):
        """Times the shape candidates on the current particles and frame
        `obs`, keeps the fastest; returns (ms per step launches, chosen)."""
        ms = (ctypes.c_double * TUNE_MAX)()
        n, ch = ctypes.c_int32(), ctypes.c_int32()
        self._chk(lib().ppf_batch_autotune(self.handle, self._obs_ptr(obs), int(reps), ms,
                                           ctypes.byref(n), ctypes.byref(ch)))
        return list(ms[:n.value]), ch.value

    def profile(self, on: bool = True):
        self._chk(lib().ppf_batch_profile_enable(self.handle, 1 if on else 0))

    def kernel_times(self) -> dict:
        buf = (KernelTime * 16)()
        n = ctypes.c_int()
        self._chk(lib().ppf_batch_profile_read(self.handle, buf, 16, ctypes.byref(n)))
        return {buf[j].name.decode(): (buf[j].launches, buf[j].total_ms) for j in range(n.value)}

    def sync(self):
        self.stream.synchronize()


# --------------------------------------------------- differentiable log p^
def params_at(base: Params, theta) -> Params:
    """A copy of `base` with theta = (psf_sigma, background, noise_sigma,
    q[0..4], I0) applied: I0 moves init_a[4] and init_b[4] together, and the
    patch is pinned to base's so that it does not jump as psf_sigma moves."""
    p = Params.from_buffer_copy(base)
    th = [float(v) for v in theta]
    p.patch = patch_size(base)
    p.psf_sigma, p.background, p.noise_sigma = th[0], th[1], th[2]
    for d in range(5):
        p.q[d] = th[3 + d]
    p.init_a[4] = base.init_a[4] + th[8]
    p.init_b[4] = base.init_b[4] + th[8]
    p.grad = 1
    return p


def theta_of(base: Params):
    """theta of `base` itself (I0 offset 0)."""
    return [base.psf_sigma, base.background, base.noise_sigma] + list(base.q) + [0.0]


def _make_loglik_function():
    import torch

    class LogLikelihood(torch.autograd.Function):
        """log p^(z_1:T) of one filter run over `frames` as a function of
        theta (see params_at): the forward pass runs the filter in gradient
        mode, which carries the derivatives alongside the particles, and the
        backward pass scales them by the incoming gradient."""

        @staticmethod
        def forward(ctx, theta, frames, base):
            p = params_at(base, theta.detach().cpu().tolist())
            f = Filter(p, device=frames.device)
            for k in range(frames.shape[0]):
                f.step(frames[k])
            cum, _ = f.loglik()
            g, _ = f.grad()
            f.close()
            ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
            return torch.tensor(cum, dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None

    return LogLikelihood


_LogLikelihood = None


def loglik(theta, frames, base: Params):
    """Differentiable log p^(z_1:T): theta a 9-element float64 tensor (see
    GRAD_NAMES), frames a (T, H, W) float32 CUDA tensor, base the filter's
    other parameters (systematic resampling at every step, spot model). The
    Philox noise and the resampling ancestors are held fixed in the
    derivative."""
    global _LogLikelihood
    if _LogLikelihood is None:
        _LogLikelihood = _make_loglik_function()
    return _LogLikelihood.apply(theta, frames, base)


# ------------------------------------------------------ standalone primitives
def philox(seed: int, ctr, stream=None):
    """Philox4x32-10 of a (n, 4) uint32-valued CUDA tensor (int32 storage)."""
    import torch
    if ctr.dtype != torch.int32 or not ctr.is_contiguous() or ctr.dim() != 2 or ctr.shape[1] != 4:
        raise TypeError("ctr must be a contiguous (n, 4) int32 CUDA tensor")
    out = torch.empty_like(ctr)
    s = stream if stream is not None else torch.cuda.current_stream(ctr.device)
    _check(lib().ppf_philox4x32_10(seed, ctypes.c_void_p(ctr.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctr.shape[0],
                                   ctypes.c_void_p(_stream_ptr(s))))
    return out


def _scratch(n: int, device):
    import torch
    nb = ctypes.c_size_t()
    _check(lib().ppf_resample_scratch_bytes(n, ctypes.byref(nb)))
    return torch.empty(nb.value, dtype=torch.uint8, device=device), nb.value


def resample_systematic(logw, u: float, stream=None):
    """Systematic resampling of fp32 log weights (CUDA tensor); returns the
    int32 ancestors (async)."""
    import torch
    if logw.dtype != torch.float32 or not logw.is_contiguous() or logw.dim() != 1:
        raise TypeError("logw must be a contiguous 1-D float32 CUDA tensor")
    n = logw.numel()
    anc = torch.empty(n, dtype=torch.int32, device=logw.device)
    scr, nbytes = _scratch(n, logw.device)
    s = stream if stream is not None else torch.cuda.current_stream(logw.device)
    _check(lib().ppf_resample_systematic(ctypes.c_void_p(logw.data_ptr()), n, float(u),
                                         ctypes.c_void_p(anc.data_ptr()),
                                         ctypes.c_void_p(scr.data_ptr()), nbytes,
                                         ctypes.c_void_p(_stream_ptr(s))))
    anc._ppf_scratch = scr  # keep the scratch alive until the caller syncs
    return anc


def resample_systematic_static(logw, u: float, anc=None, stream=None):
    """Systematic resampling like resample_systematic, through the entry
    point that allocates nothing (its scratch is the library's own device
    array; at most STATIC_MAX_N weights). `anc`: an optional int32 output
    tensor (else one is made here). Calls on one device must not overlap."""
    import torch
    if logw.dtype != torch.float32 or not logw.is_contiguous() or logw.dim() != 1:
        raise TypeError("logw must be a contiguous 1-D float32 CUDA tensor")
    n = logw.numel()
    if n > STATIC_MAX_N:
        raise ValueError(f"at most {STATIC_MAX_N} weights (the static scratch's limit)")
    if anc is None:
        anc = torch.empty(n, dtype=torch.int32, device=logw.device)
    if anc.dtype != torch.int32 or not anc.is_contiguous() or anc.numel() != n:
        raise TypeError("anc must be a contiguous int32 tensor of n elements")
    s = stream if stream is not None else torch.cuda.current_stream(logw.device)
    _check(lib().ppf_resample_systematic_static(ctypes.c_void_p(logw.data_ptr()), n, float(u),
                                                ctypes.c_void_p(anc.data_ptr()),
                                                ctypes.c_void_p(_stream_ptr(s))))
    return anc


def dlb_schedule(kind: int, counts, n: int, stream=None):
    """DLB schedule (DLB_GS, DLB_SGS or DLB_LGS) of int32 group counts (CUDA
    tensor) towards n each: an (m, 3) int32 tensor of (sender group,
    receiver group, particles). Syncs to read the entry count."""
    import torch
    if counts.dtype != torch.int32 or not counts.is_contiguous() or counts.dim() != 1:
        raise TypeError("counts must be a contiguous 1-D int32 CUDA tensor")
    G = counts.numel()
    cap = 2 * G + 1
    sched = torch.empty((cap, 3), dtype=torch.int32, device=counts.device)
    m = torch.empty(1, dtype=torch.int32, device=counts.device)
    s = stream if stream is not None else torch.cuda.current_stream(counts.device)
    _check(lib().ppf_dlb_schedule(kind, ctypes.c_void_p(counts.data_ptr()), G, n,
                                  ctypes.c_void_p(sched.data_ptr()), cap,
                                  ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(_stream_ptr(s))))
    k = int(m.cpu())
    if k < 0:
        raise PPFError(PPF_EINVAL, "schedule capacity exceeded")
    return sched[:k]


def resample_rna(logw, group: int, moved: int, u, stream=None):
    """RNA resampling of fp32 log weights with per-group uniforms u (float64
    CUDA tensor); returns (int32 ancestors, float64 log(W_g / group))."""
    import torch
    if logw.dtype != torch.float32 or not logw.is_contiguous() or logw.dim() != 1:
        raise TypeError("logw must be a contiguous 1-D float32 CUDA tensor")
    n = logw.numel()
    if group < 1 or n % group:
        raise ValueError("n must be a multiple of group")
    if u.dtype != torch.float64 or u.numel() != n // group or not u.is_contiguous():
        raise TypeError("u must be n/group contiguous float64 values")
    anc = torch.empty(n, dtype=torch.int32, device=logw.device)
    lwg = torch.empty(n // group, dtype=torch.float64, device=logw.device)
    scr, nbytes = _scratch(n, logw.device)
    s = stream if stream is not None else torch.cuda.current_stream(logw.device)
    _check(lib().ppf_resample_rna(ctypes.c_void_p(logw.data_ptr()), n, group, moved,
                                  ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(anc.data_ptr()),
                                  ctypes.c_void_p(lwg.data_ptr()), ctypes.c_void_p(scr.data_ptr()),
                                  nbytes, ctypes.c_void_p(_stream_ptr(s))))
    anc._ppf_scratch = scr
    return anc, lwg
