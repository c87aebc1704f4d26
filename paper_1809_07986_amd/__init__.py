"""Reduced-space SGM fused by a per-pixel Kalman filter on MI355X (gfx950).

Python face of libsgm.so.  Every stage runs in the library's HIP kernels;
this module only marshals arguments: torch supplies device memory and the
current HIP stream.  Names follow the C ABI (include/sgm.h).

    sgm = ReducedSGM(width, height, max_disp, f=720.0, baseline=0.54)
    sgm.full_frame(left, right)            # uint8 [H, W] tensors on the GPU
    sgm.reduced_frame(left, right, T)      # T: 4x4 ego-motion k-1 -> k
    d = sgm.disparity(); m = sgm.motion_mask()
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _native as N

__all__ = ["ReducedSGM", "SgmBatch", "SgmError", "default_params", "as_matrix"]


class SgmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsgm error {code}: {msg}")
        self.code = code


def _lib():
    return N.load()


def _check(rc: int):
    if rc != N.SGM_OK:
        raise SgmError(rc, _lib().sgm_last_error().decode(errors="replace"))


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _dev_image(img, device) -> torch.Tensor:
    if not isinstance(img, torch.Tensor):
        img = torch.from_numpy(np.ascontiguousarray(img, dtype=np.uint8))
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("images must be uint8 [H, W]")
    return img.to(device, non_blocking=True).contiguous()


def default_params(width: int, height: int, max_disp: int, **over) -> N.SgmParams:
    p = N.SgmParams()
    _check(_lib().sgm_default_params(ctypes.byref(p), width, height, max_disp))
    for k, v in over.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    if "cx" not in over:
        p.cx = (width - 1) / 2.0
    if "cy" not in over:
        p.cy = (height - 1) / 2.0
    return p


def as_matrix(T) -> ctypes.Array:
    """4x4 row-major ego-motion as the double[16] the C ABI takes."""
    return (ctypes.c_double * 16)(*np.asarray(T, dtype=np.float64).reshape(16).tolist())


class ReducedSGM:
    """One stereo stream: owns a library context on the current device."""

    def __init__(self, width: int, height: int, max_disp: int, device: Optional[torch.device] = None, **params):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.params = default_params(width, height, max_disp, **params)
            h = ctypes.c_void_p()
            _check(_lib().sgm_create(ctypes.byref(self.params), ctypes.byref(h)))
        self._h = h
        self.W, self.H, self.D = width, height, max_disp

    @classmethod
    def _view(cls, handle, width: int, height: int, max_disp: int, device) -> "ReducedSGM":
        """A non-owning view of a context that belongs to a batch."""
        obj = cls.__new__(cls)
        obj._h = ctypes.c_void_p(handle)
        obj._owner = False
        obj.device = device
        obj.W, obj.H, obj.D = width, height, max_disp
        return obj

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owner", True):
            with torch.cuda.device(self.device):
                _lib().sgm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- frames --------------------------------------------------------------
    def full_frame(self, left, right):
        l, r = _dev_image(left, self.device), _dev_image(right, self.device)
        _check(_lib().sgm_full_frame(self._h, _ptr(l), _ptr(r), l.shape[1], _stream()))
        self._keep = (l, r)

    def reduced_frame(self, left, right, T):
        l, r = _dev_image(left, self.device), _dev_image(right, self.device)
        t = T if isinstance(T, ctypes.Array) else as_matrix(T)
        _check(_lib().sgm_reduced_frame(self._h, _ptr(l), _ptr(r), l.shape[1], t, _stream()))
        self._keep = (l, r)

    def match_windows(self, left, right, lo, hi):
        l, r = _dev_image(left, self.device), _dev_image(right, self.device)
        lo_t = torch.as_tensor(np.ascontiguousarray(lo, np.int32)).to(self.device)
        hi_t = torch.as_tensor(np.ascontiguousarray(hi, np.int32)).to(self.device)
        dstar = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device)
        dz = torch.empty((self.H, self.W), dtype=torch.float64, device=self.device)
        _check(_lib().sgm_match_windows(self._h, _ptr(l), _ptr(r), l.shape[1], _ptr(lo_t), _ptr(hi_t),
                                        _ptr(dstar), _ptr(dz), _stream()))
        self._keep = (l, r, lo_t, hi_t)
        return dstar, dz

    # -- outputs -------------------------------------------------------------
    def disparity(self) -> torch.Tensor:
        out = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        _check(_lib().sgm_get_disparity(self._h, _ptr(out), self.W, _stream()))
        return out

    def variance(self) -> torch.Tensor:
        out = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        _check(_lib().sgm_get_variance(self._h, _ptr(out), self.W, _stream()))
        return out

    def motion_mask(self) -> torch.Tensor:
        out = torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device)
        _check(_lib().sgm_get_motion_mask(self._h, _ptr(out), self.W, _stream()))
        return out

    def get_state(self):
        d = torch.empty((self.H, self.W), dtype=torch.float64, device=self.device)
        p = torch.empty_like(d)
        f = torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device)
        _check(_lib().sgm_get_state(self._h, _ptr(d), _ptr(p), _ptr(f), _stream()))
        return d, p, f

    def set_state(self, d, p, sflags):
        d = torch.as_tensor(np.ascontiguousarray(d, np.float64)).to(self.device)
        p = torch.as_tensor(np.ascontiguousarray(p, np.float64)).to(self.device)
        f = torch.as_tensor(np.ascontiguousarray(sflags, np.uint8)).to(self.device)
        _check(_lib().sgm_set_state(self._h, _ptr(d), _ptr(p), _ptr(f), _stream()))
        self._keep = (d, p, f)

    def set_debug(self, on: bool = True):
        _check(_lib().sgm_set_debug(self._h, 1 if on else 0))

    def set_profiling(self, on: bool = True):
        _check(_lib().sgm_set_profiling(self._h, 1 if on else 0))

    def read_profile(self):
        """{stage: accumulated ms}, frames measured (synchronises the stream)."""
        ms = (ctypes.c_double * len(N.PROF_STAGES))()
        n = ctypes.c_int64()
        _check(_lib().sgm_read_profile(self._h, ms, ctypes.byref(n), _stream()))
        return dict(zip(N.PROF_STAGES, list(ms))), n.value

    def cost_cells(self) -> int:
        m = ctypes.c_int64()
        _check(_lib().sgm_cost_cells(self._h, ctypes.byref(m), _stream()))
        return m.value

    _STAGE_DT = {N.STAGE_CENSUS_L: torch.int64, N.STAGE_CENSUS_R: torch.int64, N.STAGE_LO: torch.int32,
                 N.STAGE_HI: torch.int32, N.STAGE_OFFSETS: torch.int32, N.STAGE_COST: torch.uint8,
                 N.STAGE_SUM: torch.int16, N.STAGE_DHAT: torch.float64, N.STAGE_PM: torch.float64,
                 N.STAGE_FLAGS: torch.uint8, N.STAGE_DSTAR: torch.int32, N.STAGE_DZ: torch.float64,
                 N.STAGE_STATUS: torch.int32}

    def stage(self, stage: int) -> torch.Tensor:
        """Intermediate result of the last frame (see include/sgm.h)."""
        npx = self.H * self.W
        if stage in (N.STAGE_COST, N.STAGE_SUM) or stage >= N.STAGE_PATH0:
            count = self.cost_cells()
        elif stage == N.STAGE_OFFSETS:
            count = npx + 1
        elif stage == N.STAGE_STATUS:
            count = 1
        else:
            count = npx
        dt = self._STAGE_DT.get(stage, torch.uint8)
        out = torch.empty(count, dtype=dt, device=self.device)
        _check(_lib().sgm_get_stage(self._h, stage, _ptr(out), out.numel() * out.element_size(), _stream()))
        if count == npx:
            out = out.view(self.H, self.W)
        return out


class SgmBatch:
    """Many independent stereo streams stepped together over concurrent lanes.

    `streams` is a list of dicts with width, height, max_disp and any other
    sgm_params field.  The batch owns one uint8 [H, W] input tensor pair per
    stream (`left[i]`, `right[i]`); load each frame into them with `load`.
    """

    def __init__(self, streams, device: Optional[torch.device] = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        n = len(streams)
        self.n = n
        self.left, self.right, self.shapes = [], [], []
        prm = (N.SgmParams * n)()
        with torch.cuda.device(self.device):
            for i, st in enumerate(streams):
                st = dict(st)
                w, h, dmax = st.pop("width"), st.pop("height"), st.pop("max_disp")
                prm[i] = default_params(w, h, dmax, **st)
                self.left.append(torch.zeros((h, w), dtype=torch.uint8, device=self.device))
                self.right.append(torch.zeros((h, w), dtype=torch.uint8, device=self.device))
                self.shapes.append((w, h, dmax))
            lp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.left])
            rp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.right])
            pitch = (ctypes.c_int32 * n)(*[s[0] for s in self.shapes])
            h = ctypes.c_void_p()
            torch.cuda.synchronize()
            _check(_lib().sgm_batch_create(n, prm, lp, rp, pitch, ctypes.byref(h)))
        self._h = h
        self.contexts = []
        for i, (w, hh, dmax) in enumerate(self.shapes):
            ch = _lib().sgm_batch_context(self._h, i)
            if not ch:
                raise SgmError(N.SGM_EINVAL, _lib().sgm_last_error().decode())
            self.contexts.append(ReducedSGM._view(ch, w, hh, dmax, self.device))

    def close(self):
        if getattr(self, "_h", None):
            with torch.cuda.device(self.device):
                _lib().sgm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, i: int, left, right):
        self.left[i].copy_(_dev_image(left, self.device))
        self.right[i].copy_(_dev_image(right, self.device))

    @staticmethod
    def _Ts(Ts) -> ctypes.Array:
        if isinstance(Ts, ctypes.Array):
            return Ts
        a = np.ascontiguousarray(np.asarray(Ts, dtype=np.float64).reshape(-1))
        return (ctypes.c_double * a.size)(*a.tolist())

    def full(self):
        _check(_lib().sgm_batch_full(self._h, _stream()))

    def step(self, Ts):
        _check(_lib().sgm_batch_step(self._h, self._Ts(Ts), _stream()))

    def step_graph(self, Ts):
        """Captured-graph stepping (currently disabled in the library: raises)."""
        _check(_lib().sgm_batch_step_graph(self._h, self._Ts(Ts), _stream()))

    def set_schedule(self, lanes: int, order: int):
        _check(_lib().sgm_batch_set_schedule(self._h, lanes, order))

    def autotune(self, Ts, reps: int = 3):
        chosen = (ctypes.c_int32 * 2)()
        _check(_lib().sgm_batch_autotune(self._h, self._Ts(Ts), reps, chosen, _stream()))
        return int(chosen[0]), int(chosen[1])
