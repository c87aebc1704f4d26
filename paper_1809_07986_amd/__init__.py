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

__all__ = ["ReducedSGM", "SgmBatch", "CnnTrainer", "Detector", "SgmError", "default_params", "detect_params",
           "as_matrix", "load_window_model"]


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


def default_params(width: int, height: int, max_disp: int, preset: str = "default", **over) -> N.SgmParams:
    """Library defaults (preset "default") or the paper's Table 1 settings
    (preset "paper": census 5x5, P1=6, P2=65), then the overrides."""
    p = N.SgmParams()
    if preset == "default":
        _check(_lib().sgm_default_params(ctypes.byref(p), width, height, max_disp))
    elif preset == "paper":
        _check(_lib().sgm_paper_params(ctypes.byref(p), width, height, max_disp))
    else:
        raise ValueError(f"unknown preset {preset!r}")
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

    def disparity_median(self) -> torch.Tensor:
        """3x3 block median of the filtered disparity (Section 2.3 post-processing)."""
        out = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        _check(_lib().sgm_get_disparity_median(self._h, _ptr(out), self.W, _stream()))
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

    def set_debug(self, on=True):
        """True/False: record the cost and sum stages; an int: the SGM_DEBUG_* bit mask."""
        flags = int(on) if not isinstance(on, bool) else (N.DEBUG_STAGES if on else 0)
        _check(_lib().sgm_set_debug(self._h, flags))

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
                 N.STAGE_STATUS: torch.int32, N.STAGE_NU: torch.float64, N.STAGE_NU_W: torch.float64,
                 N.STAGE_FEATURES: torch.int16, N.STAGE_CNN_OUT: torch.float32, N.STAGE_HALFWIDTH: torch.float32,
                 N.STAGE_RPIX: torch.float32, N.STAGE_KAPPA: torch.int32, N.STAGE_RERUN: torch.int32}

    def stage(self, stage: int) -> torch.Tensor:
        """Intermediate result of the last frame (see include/sgm.h)."""
        npx = self.H * self.W
        if stage in (N.STAGE_COST, N.STAGE_SUM) or N.STAGE_PATH0 <= stage < N.STAGE_PATH0 + 8:
            count = self.cost_cells()
        elif stage == N.STAGE_OFFSETS:
            count = npx + 1
        elif stage == N.STAGE_STATUS:
            count = 1
        elif stage == N.STAGE_RERUN:
            count = 3
        elif stage == N.STAGE_FEATURES:
            count = npx * 4
        elif stage == N.STAGE_CNN_OUT:
            count = npx * 2
        else:
            count = npx
        dt = self._STAGE_DT.get(stage, torch.uint8)
        out = torch.empty(count, dtype=dt, device=self.device)
        _check(_lib().sgm_get_stage(self._h, stage, _ptr(out), out.numel() * out.element_size(), _stream()))
        if count == npx:
            out = out.view(self.H, self.W)
        elif stage in (N.STAGE_FEATURES, N.STAGE_CNN_OUT):
            out = out.view(self.H, self.W, -1)
        return out

    # -- learned search window --------------------------------------------------
    def set_window_model(self, params):
        """Network parameters (CNN_NPARAMS floats, layout of include/sgm.h)."""
        arr = np.ascontiguousarray(params, np.float32).reshape(-1)
        with torch.cuda.device(self.device):
            _check(_lib().sgm_set_window_model(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               arr.size))

    def features(self, left) -> torch.Tensor:
        """bfloat16 network input [H, W, 4] (as int16 bit patterns) of the last predicted frame."""
        l = _dev_image(left, self.device)
        out = torch.empty((self.H, self.W, 4), dtype=torch.int16, device=self.device)
        _check(_lib().sgm_get_features(self._h, _ptr(l), l.shape[1], _ptr(out), _stream()))
        self._keep = (l,)
        return out

    def learned_targets(self, dz_full: torch.Tensor, gt: torch.Tensor) -> torch.Tensor:
        """float [H, W, 4] (e, m, we, wm) of the last predicted frame."""
        dz = dz_full.to(self.device, torch.float64).contiguous()
        g = gt.to(self.device, torch.float32).contiguous()
        out = torch.empty((self.H, self.W, 4), dtype=torch.float32, device=self.device)
        _check(_lib().sgm_learned_targets(self._h, _ptr(dz), _ptr(g), _ptr(out), _stream()))
        self._keep = (dz, g)
        return out


def load_window_model(path: Optional[str] = None) -> np.ndarray:
    """Parameters of the trained window network shipped with the package."""
    import os
    if path is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "window_cnn.f32")
    arr = np.fromfile(path, dtype="<f4")
    if arr.size != N.CNN_NPARAMS:
        raise ValueError(f"{path}: {arr.size} floats, expected {N.CNN_NPARAMS}")
    return arr


def detect_params(width: int, height: int, sizes=None, **over) -> N.SgmDetectParams:
    """Library detection defaults, then the overrides (sizes: list of (w, h))."""
    p = N.SgmDetectParams()
    _check(_lib().sgm_detect_default_params(ctypes.byref(p), width, height))
    if sizes is not None:
        if not 1 <= len(sizes) <= 8:
            raise ValueError("1..8 window sizes")
        p.n_sizes = len(sizes)
        for k, (w, h) in enumerate(sizes):
            p.sizes[k][0], p.sizes[k][1] = int(w), int(h)
    for k, v in over.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Detector:
    """Moving-object boxes from the disagreement of predicted and measured
    disparity (Section 4); owns a library detector on the current device."""

    def __init__(self, width: int, height: int, sizes=None, device: Optional[torch.device] = None, **params):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.W, self.H = width, height
        with torch.cuda.device(self.device):
            self.params = detect_params(width, height, sizes, **params)
            h = ctypes.c_void_p()
            _check(_lib().sgm_detector_create(width, height, ctypes.byref(self.params), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(_lib().sgm_detector_windows(self._h, ctypes.byref(n)))
        self.windows = n.value
        self.boxes_buf = torch.empty((self.params.max_detections, 4), dtype=torch.int32, device=self.device)
        self.count_buf = torch.empty(2, dtype=torch.int32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            with torch.cuda.device(self.device):
                _lib().sgm_detector_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _result(self):
        n, fired = (int(v) for v in self.count_buf.cpu())
        return self.boxes_buf[:n].clone(), fired

    def detect(self, dhat, dz, flags):
        """Boxes [k, 4] int32 (x0, y0, x1, y1 half-open) and the fired-window count."""
        dh = torch.as_tensor(dhat).to(self.device, torch.float64).contiguous()
        z = torch.as_tensor(dz).to(self.device, torch.float64).contiguous()
        f = torch.as_tensor(flags).to(self.device, torch.uint8).contiguous()
        _check(_lib().sgm_detect(self._h, _ptr(dh), _ptr(z), _ptr(f), _ptr(self.boxes_buf), _ptr(self.count_buf),
                                 _stream()))
        return self._result()

    def detect_frame(self, sgm: "ReducedSGM"):
        """Boxes of the last frame of a stream."""
        _check(_lib().sgm_detect_frame(self._h, sgm._h, _ptr(self.boxes_buf), _ptr(self.count_buf), _stream()))
        return self._result()

    def stage(self, which: int) -> torch.Tensor:
        top = self.params.top
        if which == N.DSTAGE_SAT:
            out = torch.empty((self.H - top + 1, self.W + 1), dtype=torch.int32, device=self.device)
        elif which == N.DSTAGE_FIRED:
            out = torch.empty(max(self.windows, 1), dtype=torch.uint8, device=self.device)
        else:
            raise ValueError(which)
        _check(_lib().sgm_detector_stage(self._h, which, _ptr(out), out.numel() * out.element_size(), _stream()))
        return out[:self.windows] if which == N.DSTAGE_FIRED else out


class CnnTrainer:
    """Trainer of the window network (library kernels for every step)."""

    def __init__(self, max_images: int, height: int, width: int, device: Optional[torch.device] = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.H, self.W, self.maxn = height, width, max_images
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _check(_lib().sgm_cnn_create(max_images, height, width, ctypes.byref(h)))
        self._h = h
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            with torch.cuda.device(self.device):
                _lib().sgm_cnn_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        arr = np.ascontiguousarray(params, np.float32).reshape(-1)
        _check(_lib().sgm_cnn_set_params(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), arr.size))

    def get_params(self) -> np.ndarray:
        arr = np.zeros(N.CNN_NPARAMS, np.float32)
        _check(_lib().sgm_cnn_get_params(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), arr.size))
        return arr

    def _x(self, x: torch.Tensor) -> torch.Tensor:
        if x.dtype != torch.int16 or x.dim() != 4 or x.shape[1:] != (self.H, self.W, 4):
            raise ValueError("x must be int16 (bfloat16 bits) [n, H, W, 4]")
        return x.contiguous()

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = self._x(x)
        out = torch.empty((x.shape[0], self.H, self.W, 2), dtype=torch.float32, device=self.device)
        _check(_lib().sgm_cnn_forward(self._h, _ptr(x), x.shape[0], _ptr(out), _stream()))
        self._keep = (x,)
        return out

    def loss_grad(self, targets: torch.Tensor) -> torch.Tensor:
        """Loss of the last forward (device scalar) and its parameter gradient."""
        t = targets.to(self.device, torch.float32).contiguous()
        _check(_lib().sgm_cnn_loss(self._h, _ptr(t), _ptr(self.loss), _stream()))
        _check(_lib().sgm_cnn_backward(self._h, _stream()))
        self._keep_t = t
        return self.loss

    def grads(self) -> np.ndarray:
        arr = np.zeros(N.CNN_NPARAMS, np.float32)
        _check(_lib().sgm_cnn_get_grads(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), arr.size))
        return arr

    def adam(self, lr: float):
        _check(_lib().sgm_cnn_adam(self._h, float(lr), _stream()))

    def train_step(self, x: torch.Tensor, targets: torch.Tensor, lr: float) -> torch.Tensor:
        x = self._x(x)
        t = targets.contiguous()
        _check(_lib().sgm_cnn_train_step(self._h, _ptr(x), _ptr(t), x.shape[0], float(lr), _ptr(self.loss),
                                         _stream()))
        self._keep = (x, t)
        return self.loss


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

    def step(self, Ts, images=None):
        """One frame of every stream.  Ts: n ego-motions (a row whose [3, 3]
        entry is 0 runs a full-range frame), or None for all full range.
        images: optional list of (left, right) device uint8 tensors for this
        step (default: the batch's own buffers)."""
        l = r = p = None
        if images is not None:
            ims = [(_dev_image(a, self.device), _dev_image(b, self.device)) for a, b in images]
            l = (ctypes.c_void_p * self.n)(*[a.data_ptr() for a, _ in ims])
            r = (ctypes.c_void_p * self.n)(*[b.data_ptr() for _, b in ims])
            p = (ctypes.c_int32 * self.n)(*[a.stride(0) for a, _ in ims])
            self._keep = ims
        T = None if Ts is None else self._Ts(Ts)
        _check(_lib().sgm_batch_step(self._h, l, r, p, T, _stream()))

    def step_graph(self, Ts):
        """Captured-graph stepping (disabled in the library: raises SgmError)."""
        _check(_lib().sgm_batch_step_graph(self._h, self._Ts(Ts), _stream()))

    def set_schedule(self, lanes: int, order: int):
        _check(_lib().sgm_batch_set_schedule(self._h, lanes, order))

    def autotune(self, Ts, reps: int = 3):
        """-> (lanes, order, horizontal segment length, horizontal kernel family)."""
        chosen = (ctypes.c_int32 * 4)()
        _check(_lib().sgm_batch_autotune(self._h, self._Ts(Ts), reps, chosen, _stream()))
        return tuple(int(v) for v in chosen)

    def autotune_budget(self, budget_ms: int):
        _check(_lib().sgm_autotune(self._h, int(budget_ms)))
