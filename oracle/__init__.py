"""Plain CPU oracle (test infrastructure only).

A thin ctypes binding over ``sgm_oracle.c``: dense numpy arrays in, dense
numpy arrays out, double precision for every floating-point quantity.  Only
the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
use it; the GPU library never does.

Flags returned by :func:`predict` (per pixel of a predicted frame):
``PRED`` a prediction exists, ``RESET`` the previous frame forced a full
search, ``FULLWIN`` the window is [0, D-1].
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading
from typing import Optional

import numpy as np

__all__ = ["Params", "build", "use_threads", "census", "cost", "aggregate", "wta", "match", "predict", "predict_aux", "median3x3",
           "DetectParams", "motion_values", "integral", "detect_windows", "merge_boxes", "detect",
           "learned_windows", "correct", "correct_ex", "OracleFilter", "PRED", "RESET", "FULLWIN", "GATEFAIL",
           "PATH_DX", "PATH_DY"]

PRED, RESET, FULLWIN, GATEFAIL = 1, 2, 4, 8
# path k has direction r = (PATH_DX[k], PATH_DY[k]); the predecessor of p is p - r
PATH_DX = (+1, -1, 0, 0, +1, -1, -1, +1)
PATH_DY = (0, 0, +1, -1, +1, -1, +1, -1)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source with -fopenmp: its parallel loops on several threads, same results (CPU baseline)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lock = threading.Lock()
_libs = {}
_threaded = False


def _build_one(lib: str, extra, force: bool):
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
        return lib
    tmp = lib + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off",
                    "-fno-fast-math", "-shared", "-fPIC"] + extra + [_SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction): oracle/liboracle.so
    (one thread, the parity reference) and oracle/liboracle_omp.so (-fopenmp)."""
    _build_one(_LIB_OMP, ["-fopenmp"], force)
    return _build_one(_LIB, [], force)


def use_threads(on: bool) -> int:
    """Route every oracle call through the OpenMP build (True) or the
    one-thread build (False, the default).  Returns the thread count the
    selected build uses."""
    global _threaded
    _threaded = bool(on)
    return int(_load().orc_threads())


class _CParams(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_disp", ctypes.c_int32),
                ("census_w", ctypes.c_int32), ("census_h", ctypes.c_int32), ("path_mask", ctypes.c_uint32),
                ("p1", ctypes.c_int32), ("p2", ctypes.c_int32),
                ("k_sigma", ctypes.c_double), ("q", ctypes.c_double), ("r", ctypes.c_double),
                ("chi2_gate", ctypes.c_double), ("disc_thresh", ctypes.c_double),
                ("f", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("baseline", ctypes.c_double)]


@dataclasses.dataclass
class Params:
    """Method parameters (same fields and meaning as the GPU library's)."""
    width: int
    height: int
    max_disp: int
    census_w: int = 9
    census_h: int = 7
    path_mask: int = 0xFF
    p1: int = 7
    p2: int = 86
    k_sigma: float = 3.0
    q: float = 0.5
    r: float = 1.0
    chi2_gate: float = 6.634896601021214   # chi^2 with 1 dof, 99 %
    disc_thresh: float = 2.0
    f: float = 350.0
    cx: Optional[float] = None
    cy: Optional[float] = None
    baseline: float = 0.54
    r_curv: float = 0.0     # > 0: per-pixel measurement variance r_curv / kappa (curvature_r); not in the C struct

    def __post_init__(self):
        if self.cx is None:
            self.cx = (self.width - 1) / 2.0
        if self.cy is None:
            self.cy = (self.height - 1) / 2.0

    @property
    def nbits(self) -> int:
        return self.census_w * self.census_h - 1

    def c(self) -> _CParams:
        return _CParams(self.width, self.height, self.max_disp, self.census_w, self.census_h,
                        self.path_mask, self.p1, self.p2, self.k_sigma, self.q, self.r, self.chi2_gate,
                        self.disc_thresh, self.f, self.cx, self.cy, self.baseline)


def _load():
    with _lock:
        key = "omp" if _threaded else "1t"
        if key not in _libs:
            build(force=False)
            lib = ctypes.CDLL(_LIB_OMP if _threaded else _LIB)
            P = ctypes.c_void_p
            i = ctypes.c_int
            lib.orc_census.argtypes = [P, i, i, i, i, P]
            lib.orc_cost.argtypes = [P, P, i, i, i, i, P, P, P]
            lib.orc_aggregate.argtypes = [P, i, i, i, P, P, i, i, ctypes.c_uint, P, P]
            lib.orc_wta.argtypes = [P, i, i, i, P, P, P, P]
            lib.orc_match.argtypes = [P, P, P, P, P, P, P, P, P]
            lib.orc_predict.argtypes = [P, P, P, P, P, P, P, P, P, P]
            lib.orc_correct.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
            lib.orc_full_frame.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
            lib.orc_reduced_frame.argtypes = [P] + [P] * 14
            lib.orc_predict_aux.argtypes = [P] * 12
            lib.orc_learned_windows.argtypes = [P] * 6
            lib.orc_correct_ex.argtypes = [P] * 14
            lib.orc_curvature_r.argtypes = [P, i, i, i, P, P, P, ctypes.c_double, ctypes.c_double, P, P]
            lib.orc_median3x3.argtypes = [P, i, i, P]
            lib.orc_motion_values.argtypes = [P, P, P, i, i, i, i, P]
            lib.orc_integral.argtypes = [P, i, i, P]
            lib.orc_detect_windows.argtypes = [P, P, i, i, P, P]
            lib.orc_merge_boxes.argtypes = [P, i, ctypes.c_double, ctypes.c_int64]
            lib.orc_detect.argtypes = [P, P, P, P, i, i, P, P]
            for name in ("orc_census", "orc_cost", "orc_aggregate", "orc_wta", "orc_match", "orc_predict",
                         "orc_correct", "orc_full_frame", "orc_reduced_frame", "orc_predict_aux",
                         "orc_learned_windows", "orc_correct_ex", "orc_median3x3", "orc_motion_values",
                         "orc_integral", "orc_detect_windows", "orc_merge_boxes", "orc_detect", "orc_threads"):
                getattr(lib, name).restype = ctypes.c_int
            lib.orc_threads.argtypes = []
            _libs[key] = lib
        return _libs[key]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def census(img: np.ndarray, cw: int = 9, ch: int = 7) -> np.ndarray:
    img = _c(img, np.uint8)
    H, W = img.shape
    out = np.zeros((H, W), np.uint64)
    _check(_load().orc_census(_p(img), W, H, cw, ch, _p(out)), "census")
    return out


def cost(cl: np.ndarray, cr: np.ndarray, D: int, nbits: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Dense [H, W, D] int32 costs; cells outside [lo, hi] are -1."""
    cl, cr = _c(cl, np.uint64), _c(cr, np.uint64)
    lo, hi = _c(lo, np.int32), _c(hi, np.int32)
    H, W = cl.shape
    C = np.full((H, W, D), -1, np.int32)
    _check(_load().orc_cost(_p(cl), _p(cr), W, H, D, nbits, _p(lo), _p(hi), _p(C)), "cost")
    return C


def aggregate(C: np.ndarray, lo: np.ndarray, hi: np.ndarray, p1: int, p2: int, path_mask: int = 0xFF,
              want_lr: bool = False):
    """S [H, W, D] int32 (and per-path L_r [8, H, W, D] if want_lr); -1 outside windows."""
    C = _c(C, np.int32)
    lo, hi = _c(lo, np.int32), _c(hi, np.int32)
    H, W, D = C.shape
    S = np.full((H, W, D), -1, np.int32)
    Lr = np.full((8, H, W, D), -1, np.int32) if want_lr else None
    _check(_load().orc_aggregate(_p(C), W, H, D, _p(lo), _p(hi), p1, p2, path_mask, _p(S), _p(Lr)),
           "aggregate")
    return (S, Lr) if want_lr else S


def wta(S: np.ndarray, lo: np.ndarray, hi: np.ndarray):
    S = _c(S, np.int32)
    lo, hi = _c(lo, np.int32), _c(hi, np.int32)
    H, W, D = S.shape
    dstar = np.zeros((H, W), np.int32)
    dz = np.zeros((H, W), np.float64)
    _check(_load().orc_wta(_p(S), W, H, D, _p(lo), _p(hi), _p(dstar), _p(dz)), "wta")
    return dstar, dz


def match(prm: Params, left: np.ndarray, right: np.ndarray, lo: np.ndarray, hi: np.ndarray,
          want_cs: bool = False):
    """Census, cost, aggregation and WTA on the given windows -> (dstar, dz[, C, S])."""
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    lo, hi = _c(lo, np.int32), _c(hi, np.int32)
    H, W = left.shape
    dstar = np.zeros((H, W), np.int32)
    dz = np.zeros((H, W), np.float64)
    C = np.full((H, W, prm.max_disp), -1, np.int32) if want_cs else None
    S = np.full((H, W, prm.max_disp), -1, np.int32) if want_cs else None
    cp = prm.c()
    _check(_load().orc_match(ctypes.byref(cp), _p(left), _p(right), _p(lo), _p(hi), _p(dstar), _p(dz),
                             _p(C), _p(S)), "match")
    return (dstar, dz, C, S) if want_cs else (dstar, dz)


def predict(prm: Params, d: np.ndarray, p: np.ndarray, sflags: np.ndarray, T: np.ndarray):
    """Warp + hole fill + discontinuity rejection + windows -> (dhat, pm, flags, lo, hi)."""
    d, p = _c(d, np.float64), _c(p, np.float64)
    sflags = _c(sflags, np.uint8)
    T = _c(T, np.float64).reshape(16)
    H, W = d.shape
    dhat = np.zeros((H, W), np.float64)
    pm = np.zeros((H, W), np.float64)
    flags = np.zeros((H, W), np.uint8)
    lo = np.zeros((H, W), np.int32)
    hi = np.zeros((H, W), np.int32)
    cp = prm.c()
    _check(_load().orc_predict(ctypes.byref(cp), _p(d), _p(p), _p(sflags), _p(T), _p(dhat), _p(pm),
                               _p(flags), _p(lo), _p(hi)), "predict")
    return dhat, pm, flags, lo, hi


def predict_aux(prm: Params, d, p, sflags, T, aux):
    """predict() that also carries a per-source value with the warp winner
    -> (dhat, pm, flags, lo, hi, aux_out); aux_out is 0 for filled holes and
    pixels without prediction."""
    d, p = _c(d, np.float64), _c(p, np.float64)
    sflags = _c(sflags, np.uint8)
    aux = _c(aux, np.float64)
    T = _c(T, np.float64).reshape(16)
    H, W = d.shape
    dhat = np.zeros((H, W), np.float64)
    pm = np.zeros((H, W), np.float64)
    flags = np.zeros((H, W), np.uint8)
    lo = np.zeros((H, W), np.int32)
    hi = np.zeros((H, W), np.int32)
    aux_out = np.zeros((H, W), np.float64)
    cp = prm.c()
    _check(_load().orc_predict_aux(ctypes.byref(cp), _p(d), _p(p), _p(sflags), _p(aux), _p(T), _p(dhat),
                                   _p(pm), _p(flags), _p(lo), _p(hi), _p(aux_out)), "predict_aux")
    return dhat, pm, flags, lo, hi, aux_out


def learned_windows(prm: Params, dhat, hw, flags, lo, hi):
    """Windows [floor(dhat - hw), ceil(dhat + hw)] for pixels not already at
    the full range; hw >= 32 sends a pixel to the full range.  Returns new
    (flags, lo, hi)."""
    dhat, hw = _c(dhat, np.float64), _c(hw, np.float64)
    flags = np.array(flags, np.uint8, copy=True, order="C")
    lo = np.array(lo, np.int32, copy=True, order="C")
    hi = np.array(hi, np.int32, copy=True, order="C")
    cp = prm.c()
    _check(_load().orc_learned_windows(ctypes.byref(cp), _p(dhat), _p(hw), _p(flags), _p(lo), _p(hi)),
           "learned_windows")
    return flags, lo, hi


def correct_ex(prm: Params, dhat, pm, flags, lo, hi, dstar, dz, rpix=None):
    """correct() with an optional per-pixel measurement variance; GATEFAIL
    pixels restart from the measurement and stay marked moving.
    -> (d, p, mask, sflags, nu)."""
    dhat, pm, dz = _c(dhat, np.float64), _c(pm, np.float64), _c(dz, np.float64)
    flags = _c(flags, np.uint8)
    lo, hi, dstar = _c(lo, np.int32), _c(hi, np.int32), _c(dstar, np.int32)
    rp = None if rpix is None else _c(rpix, np.float64)
    H, W = dhat.shape
    d = np.zeros((H, W), np.float64)
    p = np.zeros((H, W), np.float64)
    mask = np.zeros((H, W), np.uint8)
    sflags = np.zeros((H, W), np.uint8)
    nu = np.zeros((H, W), np.float64)
    cp = prm.c()
    _check(_load().orc_correct_ex(ctypes.byref(cp), _p(dhat), _p(pm), _p(flags), _p(lo), _p(hi), _p(dstar),
                                  _p(dz), _p(rp), _p(d), _p(p), _p(mask), _p(sflags), _p(nu)), "correct_ex")
    return d, p, mask, sflags, nu


def curvature_r(S, lo, hi, dstar, r_curv: float, r_const: float):
    """Per-pixel measurement variance from the cost curvature kappa = a + b
    of the sub-pixel parabola: r = clamp(r_curv / kappa, 1/256, 64), r_const
    where d* lies on a window edge (kappa = 0).  S dense [H, W, D].
    -> (rpix float64, kappa int32)."""
    S = _c(S, np.int32)
    lo, hi, dstar = _c(lo, np.int32), _c(hi, np.int32), _c(dstar, np.int32)
    H, W, D = S.shape
    rpix = np.zeros((H, W), np.float64)
    kappa = np.zeros((H, W), np.int32)
    _check(_load().orc_curvature_r(_p(S), W, H, D, _p(lo), _p(hi), _p(dstar), float(r_curv), float(r_const),
                                   _p(rpix), _p(kappa)), "curvature_r")
    return rpix, kappa


def median3x3(d) -> np.ndarray:
    """3x3 block median with clamped borders (Section 2.3 post-processing)."""
    d = _c(d, np.float64)
    H, W = d.shape
    out = np.zeros((H, W), np.float64)
    _check(_load().orc_median3x3(_p(d), W, H, _p(out)), "median3x3")
    return out


class _CDetect(ctypes.Structure):
    _fields_ = [("top", ctypes.c_int32), ("n_sizes", ctypes.c_int32), ("sizes", (ctypes.c_int32 * 2) * 8),
                ("scale", ctypes.c_int32), ("cap", ctypes.c_int32), ("thresh", ctypes.c_int32),
                ("max_detections", ctypes.c_int32), ("min_area", ctypes.c_int64), ("merge_iou", ctypes.c_double)]


@dataclasses.dataclass
class DetectParams:
    """Moving-object detection settings (Section 4); `top` None = height // 3."""
    sizes: tuple = ((20, 20), (30, 30), (40, 40), (50, 50), (50, 75))
    top: Optional[int] = None
    scale: int = 16
    cap: int = 256
    thresh: int = 16
    max_detections: int = 2048
    min_area: int = 1600
    merge_iou: float = 0.0

    def c(self, height: int) -> _CDetect:
        out = _CDetect()
        out.top = height // 3 if self.top is None else self.top
        out.n_sizes = len(self.sizes)
        for k, (w, h) in enumerate(self.sizes):
            out.sizes[k][0], out.sizes[k][1] = w, h
        out.scale, out.cap, out.thresh = self.scale, self.cap, self.thresh
        out.max_detections, out.min_area, out.merge_iou = self.max_detections, self.min_area, self.merge_iou
        return out


def motion_values(dhat, dz, flags, scale: int = 16, cap: int = 256) -> np.ndarray:
    """Fixed-point |d^ - d_z| where a prediction exists, else 0 (Section 4)."""
    dhat, dz, flags = _c(dhat, np.float64), _c(dz, np.float64), _c(flags, np.uint8)
    H, W = dhat.shape
    v = np.zeros((H, W), np.int32)
    _check(_load().orc_motion_values(_p(dhat), _p(dz), _p(flags), W, H, scale, cap, _p(v)), "motion_values")
    return v


def integral(v) -> np.ndarray:
    """(H+1) x (W+1) summed-area table of an int32 map."""
    v = _c(v, np.int32)
    H, W = v.shape
    S = np.zeros((H + 1, W + 1), np.int64)
    _check(_load().orc_integral(_p(v), W, H, _p(S)), "integral")
    return S


def detect_windows(S, dp: DetectParams):
    """Sliding-window detections (k x 4 half-open boxes) and the number that fired."""
    S = _c(S, np.int64)
    H, W = S.shape[0] - 1, S.shape[1] - 1
    c = dp.c(H)
    boxes = np.zeros((max(dp.max_detections, 1), 4), np.int32)
    fired = ctypes.c_int32(0)
    n = _load().orc_detect_windows(ctypes.byref(c), _p(S), W, H, _p(boxes), ctypes.byref(fired))
    return boxes[:n].copy(), fired.value


def merge_boxes(boxes, merge_iou: float = 0.0, min_area: int = 0) -> np.ndarray:
    """Greedy IoU grouping followed by the small-box discard."""
    b = _c(np.asarray(boxes).reshape(-1, 4), np.int32).copy()
    n = _load().orc_merge_boxes(_p(b), b.shape[0], float(merge_iou), int(min_area))
    return b[:n].copy()


def detect(dhat, dz, flags, dp: Optional[DetectParams] = None):
    """Moving-object boxes of one frame and the number of windows that fired."""
    dp = dp or DetectParams()
    dhat, dz, flags = _c(dhat, np.float64), _c(dz, np.float64), _c(flags, np.uint8)
    H, W = dhat.shape
    c = dp.c(H)
    boxes = np.zeros((max(dp.max_detections, 1), 4), np.int32)
    fired = ctypes.c_int32(0)
    n = _load().orc_detect(ctypes.byref(c), _p(dhat), _p(dz), _p(flags), W, H, _p(boxes), ctypes.byref(fired))
    _check(0 if n >= 0 else n, "detect")
    return boxes[:n].copy(), fired.value


def correct(prm: Params, dhat, pm, flags, lo, hi, dstar, dz):
    """Kalman correction + innovation test -> (d, p, mask, sflags)."""
    dhat, pm, dz = _c(dhat, np.float64), _c(pm, np.float64), _c(dz, np.float64)
    flags = _c(flags, np.uint8)
    lo, hi, dstar = _c(lo, np.int32), _c(hi, np.int32), _c(dstar, np.int32)
    H, W = dhat.shape
    d = np.zeros((H, W), np.float64)
    p = np.zeros((H, W), np.float64)
    mask = np.zeros((H, W), np.uint8)
    sflags = np.zeros((H, W), np.uint8)
    cp = prm.c()
    _check(_load().orc_correct(ctypes.byref(cp), _p(dhat), _p(pm), _p(flags), _p(lo), _p(hi), _p(dstar),
                               _p(dz), _p(d), _p(p), _p(mask), _p(sflags)), "correct")
    return d, p, mask, sflags


class OracleFilter:
    """Frame-level driver: full_frame() once, then reduced_frame(T) per frame.

    After each call the attributes hold the frame's results: d, p (state),
    sflags (RESET for the next frame), mask (moving), lo, hi, dstar, dz and,
    for reduced frames, dhat, pm, flags.
    """

    def __init__(self, prm: Params):
        self.prm = prm
        H, W = prm.height, prm.width
        self.d = np.zeros((H, W), np.float64)
        self.p = np.zeros((H, W), np.float64)
        self.sflags = np.zeros((H, W), np.uint8)
        self.mask = np.zeros((H, W), np.uint8)
        self.lo = np.zeros((H, W), np.int32)
        self.hi = np.zeros((H, W), np.int32)
        self.dstar = np.zeros((H, W), np.int32)
        self.dz = np.zeros((H, W), np.float64)
        self.dhat = np.zeros((H, W), np.float64)
        self.pm = np.zeros((H, W), np.float64)
        self.flags = np.zeros((H, W), np.uint8)
        self.nu = np.zeros((H, W), np.float64)      # innovation of the last frame
        self.nu_w = np.zeros((H, W), np.float64)    # previous innovation carried by the warp
        self.hw = None
        self.rpix = None
        self.started = False

    def full_frame(self, left, right):
        left, right = _c(left, np.uint8), _c(right, np.uint8)
        if self.prm.r_curv > 0:
            # as orc_full_frame, keeping the sums for the curvature of each pixel
            D = self.prm.max_disp
            self.lo[:] = 0
            self.hi[:] = D - 1
            self.dstar, self.dz, _, S = match(self.prm, left, right, self.lo, self.hi, want_cs=True)
            self.rpix, self.kappa = curvature_r(S, self.lo, self.hi, self.dstar, self.prm.r_curv, self.prm.r)
            self.d[:] = self.dz
            self.p[:] = self.prm.r
            self.sflags[:] = 0
            self.mask[:] = 0
            self.flags[:] = FULLWIN
            self.nu[:] = 0.0
            self.started = True
            return
        cp = self.prm.c()
        _check(_load().orc_full_frame(ctypes.byref(cp), _p(left), _p(right), _p(self.d), _p(self.p),
                                      _p(self.sflags), _p(self.mask), _p(self.lo), _p(self.hi),
                                      _p(self.dstar), _p(self.dz)), "full_frame")
        self.flags[:] = FULLWIN
        self.nu[:] = 0.0
        self.started = True

    def reduced_frame(self, left, right, T):
        if not self.started:
            raise RuntimeError("reduced_frame before full_frame")
        left, right = _c(left, np.uint8), _c(right, np.uint8)
        T = _c(T, np.float64).reshape(16)
        if self.prm.r_curv > 0:
            # predict, match keeping the sums, correct with the curvature variance
            self.dhat, self.pm, self.flags, self.lo, self.hi = predict(self.prm, self.d, self.p, self.sflags, T)
            self.dstar, self.dz, _, S = match(self.prm, left, right, self.lo, self.hi, want_cs=True)
            self.rpix, self.kappa = curvature_r(S, self.lo, self.hi, self.dstar, self.prm.r_curv, self.prm.r)
            self.d, self.p, self.mask, self.sflags, self.nu = correct_ex(
                self.prm, self.dhat, self.pm, self.flags, self.lo, self.hi, self.dstar, self.dz, self.rpix)
            return
        cp = self.prm.c()
        _check(_load().orc_reduced_frame(ctypes.byref(cp), _p(left), _p(right), _p(T), _p(self.d),
                                         _p(self.p), _p(self.sflags), _p(self.mask), _p(self.dhat),
                                         _p(self.pm), _p(self.flags), _p(self.lo), _p(self.hi),
                                         _p(self.dstar), _p(self.dz)), "reduced_frame")
        self.nu = np.where((self.flags & PRED) != 0, self.dz - self.dhat, 0.0)

    def predict_learned(self, left, T):
        """Prediction step of a learned-window frame -> the network input
        (float64 [H, W, 4], before rounding to bfloat16)."""
        from . import cnn
        if not self.started:
            raise RuntimeError("reduced_frame before full_frame")
        (self.dhat, self.pm, self.flags, self.lo, self.hi,
         self.nu_w) = predict_aux(self.prm, self.d, self.p, self.sflags, T, self.nu)
        return cnn.features(left, self.dhat, self.pm, self.flags, self.nu_w)

    def finish_learned(self, left, right, hw, rpix, gate_rerun: bool):
        """Rest of a learned-window frame after predict_learned(): windows
        from the half-widths hw, matching, correction with the per-pixel
        measurement variance rpix and, with gate_rerun, one more matching
        pass in which the pixels that failed the innovation test search the
        full range and restart from that measurement."""
        self.hw, self.rpix = np.asarray(hw, np.float64), np.asarray(rpix, np.float64)
        self.flags, self.lo, self.hi = learned_windows(self.prm, self.dhat, self.hw, self.flags, self.lo,
                                                       self.hi)
        self.dstar, self.dz = match(self.prm, left, right, self.lo, self.hi)
        d, p, mask, sflags, nu = correct_ex(self.prm, self.dhat, self.pm, self.flags, self.lo, self.hi,
                                            self.dstar, self.dz, self.rpix)
        self.gatefail = mask.astype(bool)
        if gate_rerun and self.gatefail.any():
            D = self.prm.max_disp
            self.flags = np.where(self.gatefail, self.flags | FULLWIN | GATEFAIL, self.flags).astype(np.uint8)
            self.lo = np.where(self.gatefail, 0, self.lo).astype(np.int32)
            self.hi = np.where(self.gatefail, D - 1, self.hi).astype(np.int32)
            self.dstar, self.dz = match(self.prm, left, right, self.lo, self.hi)
            d, p, mask, sflags, nu = correct_ex(self.prm, self.dhat, self.pm, self.flags, self.lo, self.hi,
                                                self.dstar, self.dz, self.rpix)
        self.d, self.p, self.mask, self.sflags, self.nu = d, p, mask, sflags, nu

    def learned_frame(self, left, right, T, theta, gate_rerun: bool = True):
        """A whole learned-window frame with the fp64 network of oracle.cnn
        applied to the bfloat16-rounded input."""
        from . import cnn
        f = self.predict_learned(left, T)
        o, _ = cnn.forward(theta, cnn.bf16_round(f)[None])
        hw, rpix = cnn.head(o[0], self.prm.k_sigma)
        self.finish_learned(left, right, hw, rpix, gate_rerun)

    def set_state(self, d, p, sflags):
        self.d[:] = d
        self.p[:] = p
        self.sflags[:] = sflags
        self.nu[:] = 0.0
        self.started = True
