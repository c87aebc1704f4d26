"""Seeded synthetic stereo sequences (input generator shared by the tests, the
oracle harness and the benchmark).

This module renders scenes; it holds none of the matching / filtering
arithmetic of the method.  It stands in for the KITTI raw sequences the paper
evaluates on (Section 5): every item is built procedurally from a seed.

Camera conventions: rectified pinhole pair, x right, y down, z forward, the
right camera displaced by +baseline along x, principal point at the image
centre ((W-1)/2, (H-1)/2).  Disparity d = x_left - x_right >= 0, d = f*B/Z.
The ego-motion T_k_km1 (4x4, row-major) maps camera coordinates of frame k-1
into camera coordinates of frame k: X_k = R X_{k-1} + t.

Rendering:
  * each left pixel is ray-cast against planes and (oriented) boxes; the ray
    direction has unit z so the hit parameter is the camera depth Z;
  * texture is world-anchored value noise (hashed lattice, bilinear, two
    octaves) so a surface keeps its texture as the camera moves;
  * ground-truth disparity is round(f*B/Z); the right image is the left image
    forward-warped by that integer disparity (larger disparity wins), with
    fresh random texture where nothing lands;
  * independent Gaussian noise is added to both images, rounded half-to-even
    and clipped to [0, 255].
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from typing import List, Optional

import numpy as np

__all__ = ["Camera", "Sequence", "make_sequence", "CONFIGS", "synthetic_cost_volume",
           "random_windows", "random_state"]


@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    f: float
    baseline: float

    @property
    def cx(self) -> float:
        return (self.width - 1) / 2.0

    @property
    def cy(self) -> float:
        return (self.height - 1) / 2.0

    @property
    def fB(self) -> float:
        return self.f * self.baseline


@dataclasses.dataclass
class Sequence:
    name: str
    cam: Camera
    max_disp: int
    left: np.ndarray      # [K, H, W] uint8
    right: np.ndarray     # [K, H, W] uint8
    disp_gt: np.ndarray   # [K, H, W] int16, -1 where invalid
    valid: np.ndarray     # [K, H, W] bool (visible in both views, 0 <= d <= D-1, x-d >= 0)
    mover: np.ndarray     # [K, H, W] bool (pixel shows an independently moving object)
    T: np.ndarray         # [K, 4, 4] float64; T[k] maps frame k-1 camera coords to frame k (T[0] = I)

    @property
    def frames(self) -> int:
        return self.left.shape[0]

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.left, self.right, self.disp_gt, self.valid, self.mover, self.T):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


# ----------------------------------------------------------------------------
# texture
# ----------------------------------------------------------------------------

_M1 = np.uint64(0x9E3779B97F4A7C15)
_M2 = np.uint64(0xBF58476D1CE4E5B9)
_M3 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele et al.), vectorised on uint64."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M2
        z = (z ^ (z >> np.uint64(27))) * _M3
        return z ^ (z >> np.uint64(31))


def _lattice(i: np.ndarray, j: np.ndarray, key: int) -> np.ndarray:
    """Uniform [0, 255] value per integer lattice point (i, j) of surface `key`."""
    with np.errstate(over="ignore"):
        z = (i.astype(np.int64).astype(np.uint64) * _M1) ^ (
            j.astype(np.int64).astype(np.uint64) * _M2) ^ (np.uint64(key & 0xFFFFFFFFFFFF) * _M3)
        return (_mix(z) >> np.uint64(56)).astype(np.float64)


def _value_noise(u: np.ndarray, v: np.ndarray, key: int, cell: float) -> np.ndarray:
    fu, fv = u / cell, v / cell
    i0, j0 = np.floor(fu), np.floor(fv)
    a, b = fu - i0, fv - j0
    i0 = i0.astype(np.int64)
    j0 = j0.astype(np.int64)
    v00 = _lattice(i0, j0, key)
    v10 = _lattice(i0 + 1, j0, key)
    v01 = _lattice(i0, j0 + 1, key)
    v11 = _lattice(i0 + 1, j0 + 1, key)
    return (v00 * (1 - a) + v10 * a) * (1 - b) + (v01 * (1 - a) + v11 * a) * b


def _texture(u: np.ndarray, v: np.ndarray, key: int) -> np.ndarray:
    t = 0.55 * _value_noise(u, v, key * 2 + 1, 0.05) + 0.45 * _value_noise(u, v, key * 2 + 2, 0.21)
    return np.clip(128.0 + 1.6 * (t - 127.5), 0.0, 255.0)


# ----------------------------------------------------------------------------
# scene primitives (world frame = camera frame of frame 0)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class _Plane:
    n: np.ndarray          # unit normal
    h: float               # n . X = h
    u_axis: np.ndarray
    v_axis: np.ndarray
    key: int
    bounds: Optional[tuple] = None   # (umin, umax, vmin, vmax) in plane coords, None = infinite
    mover: bool = False


@dataclasses.dataclass
class _Box:
    half: np.ndarray       # half extents in object coords (x, y, z)
    key: int
    mover: bool = False
    # per-frame pose: world <- object: X_w = Rz(yaw about y) X_o + c
    centers: Optional[np.ndarray] = None   # [K, 3]
    yaws: Optional[np.ndarray] = None      # [K]


def _rot_y(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _hit_plane(pl: _Plane, o: np.ndarray, dw: np.ndarray):
    denom = dw @ pl.n
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (pl.h - o @ pl.n) / denom
    t = np.where(np.abs(denom) > 1e-12, t, np.inf)
    # rays parallel to the plane (t = inf) take t = 0 here; they are rejected below
    P = o[None, :] + np.where(np.isfinite(t), t, 0.0)[:, None] * dw
    u = P @ pl.u_axis
    v = P @ pl.v_axis
    ok = (t > 0.05) & np.isfinite(t)
    if pl.bounds is not None:
        ok &= (u >= pl.bounds[0]) & (u <= pl.bounds[1]) & (v >= pl.bounds[2]) & (v <= pl.bounds[3])
    t = np.where(ok, t, np.inf)
    return t, u, v


def _hit_box(bx: _Box, k: int, o: np.ndarray, dw: np.ndarray):
    R = _rot_y(float(bx.yaws[k]))
    c = bx.centers[k]
    oo = R.T @ (o - c)
    dd = dw @ R                      # rows: R^T d
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dd
        t1 = (-bx.half[None, :] - oo[None, :]) * inv
        t2 = (bx.half[None, :] - oo[None, :]) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    tmin = np.where(np.isnan(tmin), -np.inf, tmin)
    tmax = np.where(np.isnan(tmax), np.inf, tmax)
    tn = tmin.max(axis=1)
    tf = tmax.min(axis=1)
    face = tmin.argmax(axis=1)
    ok = (tn <= tf) & (tn > 0.05)
    t = np.where(ok, tn, np.inf)
    P = oo[None, :] + np.where(np.isfinite(t), t, 0.0)[:, None] * dd
    # texture coords: the two coordinates of the hit face's plane
    u = np.where(face == 0, P[:, 2], P[:, 0])
    v = np.where(face == 1, P[:, 2], P[:, 1])
    return t, u, v, face


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def _ego_poses(K: int, speed: float, yaw_step_deg: float, rng: np.random.Generator):
    """Camera centres c_k and world->camera rotations R_k; heading random-walks."""
    heading = 0.0
    cs = [np.zeros(3)]
    Rs = [np.eye(3)]
    for _ in range(1, K):
        heading += math.radians(rng.uniform(-yaw_step_deg, yaw_step_deg)) if yaw_step_deg > 0 else 0.0
        fwd = np.array([math.sin(heading), 0.0, math.cos(heading)])
        cs.append(cs[-1] + speed * fwd)
        Rs.append(_rot_y(heading).T)
    return cs, Rs


def _relative_T(cs, Rs) -> np.ndarray:
    K = len(cs)
    T = np.zeros((K, 4, 4))
    T[0] = np.eye(4)
    for k in range(1, K):
        R = Rs[k] @ Rs[k - 1].T
        t = Rs[k] @ (cs[k - 1] - cs[k])
        T[k, :3, :3] = R
        T[k, :3, 3] = t
        T[k, 3, 3] = 1.0
    return T


def _scene_tiny(K: int, rng: np.random.Generator):
    prims = []
    ez = np.array([0.0, 0.0, 1.0])
    ex = np.array([1.0, 0.0, 0.0])
    ey = np.array([0.0, 1.0, 0.0])
    prims.append(_Plane(-ez, -30.0, ex, ey, key=int(rng.integers(1 << 40))))
    prims.append(_Plane(-ez, -10.0, ex, ey, key=int(rng.integers(1 << 40)), bounds=(-4.2, -0.8, -1.3, 1.1)))
    prims.append(_Plane(-ez, -5.0, ex, ey, key=int(rng.integers(1 << 40)), bounds=(0.25, 1.7, -0.55, 0.62)))
    box = _Box(np.array([0.5, 0.4, 0.5]), key=int(rng.integers(1 << 40)), mover=True)
    box.centers = np.array([[-0.9 + 0.3 * k, 0.15, 7.0] for k in range(K)])
    box.yaws = np.zeros(K)
    prims.append(box)
    return prims


def _scene_driving(K: int, speed: float, rng: np.random.Generator, n_cars: int = 4, cam_h: float = 1.65,
                   depth: float = 120.0, cs=None, near: Optional[float] = None):
    prims = []
    ex = np.array([1.0, 0.0, 0.0])
    ey = np.array([0.0, 1.0, 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    # ground plane y = cam_h (y points down), textured in (x, z)
    prims.append(_Plane(ey, cam_h, ex, ez, key=int(rng.integers(1 << 40))))
    # backdrop far away
    prims.append(_Plane(-ez, -500.0, ex, ey, key=int(rng.integers(1 << 40))))
    # buildings on both sides
    for side in (-1.0, 1.0):
        z = -5.0
        while z < depth:
            length = rng.uniform(10.0, 30.0)
            height = rng.uniform(5.0, 15.0)
            lat = rng.uniform(6.0, 12.0)
            dep = 10.0
            bx = _Box(np.array([dep / 2, height / 2, length / 2]), key=int(rng.integers(1 << 40)))
            bx.centers = np.tile(np.array([side * (lat + dep / 2), cam_h - height / 2, z + length / 2]), (K, 1))
            bx.yaws = np.zeros(K)
            prims.append(bx)
            z += length + rng.uniform(2.0, 8.0)
    # cars: independent (x, z, yaw) motion, kept >= 6 m from the ego centre
    # (with `near`, the nearest car surface may come to about `near` metres)
    min_dist = 6.0 if near is None else near + 2.1
    lanes = [-3.5, 0.0, 3.5, -3.5, 3.5, 0.0, -7.0, 7.0]
    placed = 0
    tries = 0
    while placed < n_cars and tries < 1000:
        tries += 1
        lane = lanes[placed % len(lanes)] + rng.uniform(-0.4, 0.4)
        if near is None:
            z0 = rng.uniform(12.0, 45.0) + 6.0 * placed
        else:
            z0 = rng.uniform(min_dist, 25.0) + 4.0 * placed
        v = rng.uniform(0.5, 2.0) * (1.0 if lane >= 0 else -1.0)
        yaw = rng.uniform(-0.1, 0.1)
        centers, yaws = [], []
        x, zc = lane, z0
        for k in range(K):
            centers.append([x, cam_h - 0.75, zc])
            yaws.append(yaw)
            dyaw = math.radians(rng.uniform(-3.0, 3.0))
            yaw += dyaw
            step = min(abs(v), 2.0) * math.copysign(1.0, v)
            x += step * math.sin(yaw) * 0.3
            zc += step * math.cos(yaw)
        centers = np.array(centers)
        ok = True
        for k in range(K):
            if np.linalg.norm(centers[k] - cs[k] - np.array([0, cam_h - 0.75, 0])) < min_dist:
                ok = False
        for other in prims:
            if isinstance(other, _Box) and other.mover:
                if np.min(np.linalg.norm(other.centers - centers, axis=1)) < 5.0:
                    ok = False
        if not ok:
            continue
        car = _Box(np.array([0.9, 0.75, 2.1]), key=int(rng.integers(1 << 40)), mover=True)
        car.centers = centers
        car.yaws = np.array(yaws)
        prims.append(car)
        placed += 1
    return prims


def _scene_movers(K: int, speed: float, rng: np.random.Generator, n_movers: int, cam_h: float, cs,
                  near: Optional[float] = None):
    prims = _scene_driving(K, speed, rng, n_cars=n_movers, cam_h=cam_h, depth=40.0 + speed * K, cs=cs, near=near)
    return prims


# ----------------------------------------------------------------------------
# rendering
# ----------------------------------------------------------------------------

def _box_screen_rect(bx: _Box, k: int, cam: Camera, c: np.ndarray, Rwc: np.ndarray):
    """Pixel rectangle covering the box's projection, or None when the box
    reaches behind the camera (then every pixel is tested)."""
    R = _rot_y(float(bx.yaws[k]))
    sx, sy, sz = bx.half
    corners = np.array([[i * sx, j * sy, l * sz] for i in (-1, 1) for j in (-1, 1) for l in (-1, 1)])
    Xw = corners @ R.T + bx.centers[k]
    Xc = (Xw - c) @ Rwc.T
    if np.any(Xc[:, 2] <= 0.1):
        return None
    u = cam.f * Xc[:, 0] / Xc[:, 2] + cam.cx
    v = cam.f * Xc[:, 1] / Xc[:, 2] + cam.cy
    x0, x1 = int(max(np.floor(u.min()) - 1, 0)), int(min(np.ceil(u.max()) + 1, cam.width - 1))
    y0, y1 = int(max(np.floor(v.min()) - 1, 0)), int(min(np.ceil(v.max()) + 1, cam.height - 1))
    if x0 > x1 or y0 > y1:
        return (0, -1, 0, -1)
    return (x0, x1, y0, y1)


def _render(prims, cam: Camera, c: np.ndarray, Rwc: np.ndarray, k: int):
    H, W = cam.height, cam.width
    xs = (np.arange(W) - cam.cx) / cam.f
    ys = (np.arange(H) - cam.cy) / cam.f
    dcx = np.broadcast_to(xs[None, :], (H, W)).reshape(-1)
    dcy = np.broadcast_to(ys[:, None], (H, W)).reshape(-1)
    dc = np.stack([dcx, dcy, np.ones_like(dcx)], axis=1)      # camera-frame ray, z = 1
    dw = dc @ Rwc                                             # world-frame ray: R^T d (rows)
    best = np.full(H * W, np.inf)
    val = np.zeros(H * W)
    mov = np.zeros(H * W, dtype=bool)
    for pr in prims:
        if isinstance(pr, _Plane):
            sub = None
            t, u, v = _hit_plane(pr, c, dw)
        else:
            rect = _box_screen_rect(pr, k, cam, c, Rwc)
            if rect is None:
                sub = None
                t, u, v, face = _hit_box(pr, k, c, dw)
            else:
                x0, x1, y0, y1 = rect
                if x0 > x1:
                    continue
                yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
                sub = (yy * W + xx).reshape(-1)
                t, u, v, face = _hit_box(pr, k, c, dw[sub])
        if sub is None:
            sub = np.arange(H * W)
        closer = t < best[sub]
        if not np.any(closer):
            continue
        loc = np.nonzero(closer)[0]
        idx = sub[loc]
        best[idx] = t[loc]
        if isinstance(pr, _Box):
            # different faces of a box get independent texture
            for fc in range(3):
                m = face[loc] == fc
                if np.any(m):
                    val[idx[m]] = _texture(u[loc][m], v[loc][m], pr.key * 8 + fc)
        else:
            val[idx] = _texture(u[loc], v[loc], pr.key)
        mov[idx] = pr.mover
    return best.reshape(H, W), val.reshape(H, W), mov.reshape(H, W)


def _stereo_pair(Z: np.ndarray, tex: np.ndarray, cam: Camera, D: int, rng: np.random.Generator, noise: float):
    H, W = Z.shape
    with np.errstate(divide="ignore"):
        dfloat = cam.fB / Z
    dgt = np.where(np.isfinite(dfloat), np.rint(dfloat), -1).astype(np.int64)
    xs = np.broadcast_to(np.arange(W)[None, :], (H, W))
    ys = np.broadcast_to(np.arange(H)[:, None], (H, W))
    left_clean = np.rint(tex).astype(np.int64)
    inrange = (dgt >= 0) & (dgt <= D - 1)
    xr = xs - dgt
    lands = inrange & (xr >= 0)
    # z-buffer in the right view: key = d * 256 + value, max wins (larger disparity is nearer)
    zb = np.full(H * W, -1, dtype=np.int64)
    tgt = (ys * W + xr)[lands]
    keyv = (dgt * 256 + left_clean)[lands]
    np.maximum.at(zb, tgt, keyv)
    right_clean = np.where(zb >= 0, zb & 255, rng.integers(0, 256, H * W)).reshape(H, W)
    # visible in both views: the pixel won the z-buffer at its target
    won = np.zeros((H, W), dtype=bool)
    won[lands] = (zb[tgt] // 256) == dgt[lands]
    valid = won & inrange
    noisy_l = np.clip(np.rint(left_clean + rng.normal(0.0, noise, (H, W))), 0, 255).astype(np.uint8)
    noisy_r = np.clip(np.rint(right_clean + rng.normal(0.0, noise, (H, W))), 0, 255).astype(np.uint8)
    d16 = np.where(valid, dgt, -1).astype(np.int16)
    return noisy_l, noisy_r, d16, valid


# ----------------------------------------------------------------------------
# public API
# ----------------------------------------------------------------------------

CONFIGS = {
    # 320x96, D=64, f=350, B=0.54, 3 frames, 0.5 m/frame forward, fronto-parallel planes + one moving box
    "tiny": dict(width=320, height=96, max_disp=64, f=350.0, baseline=0.54, frames=3, speed=0.5,
                 yaw=0.0, noise=2.0, scene="tiny", seed=1),
    # 1242x375, D=128, f=720, B=0.54, 20 frames, 1 m/frame + yaw <= 2 deg, ground, buildings, 4 cars
    "driving": dict(width=1242, height=375, max_disp=128, f=720.0, baseline=0.54, frames=20, speed=1.0,
                    yaw=2.0, noise=2.0, scene="driving", seed=2, cars=4),
    # learned-window sequences: 1242x375, D=256, 50 frames, 6 cars that may come as near as 1.6 m
    # (training seeds 4000-4039, held out 4100-4104)
    "learned": dict(width=1242, height=375, max_disp=256, f=720.0, baseline=0.54, frames=50, speed=1.0,
                    yaw=2.0, noise=2.0, scene="driving", seed=4000, cars=6, near=1.6),
}


def make_sequence(name: str = "tiny", frames: Optional[int] = None, seed: Optional[int] = None,
                  cache_dir: Optional[str] = None, cache: bool = True, **over) -> Sequence:
    """Render a seeded synthetic stereo sequence.

    `name` selects a preset in CONFIGS; keyword overrides change any preset
    field (width, height, max_disp, f, baseline, frames, speed, yaw, noise,
    cars).  Results are cached as .npz under `cache_dir` (default: the
    SGMK_DATA directory or `<repo>/_data`) keyed by all parameters.
    """
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    if frames is not None:
        cfg["frames"] = frames
    if seed is not None:
        cfg["seed"] = seed
    tag = hashlib.sha1(repr(sorted(cfg.items())).encode()).hexdigest()[:16]
    if cache_dir is None:
        cache_dir = os.environ.get("SGMK_DATA", os.path.join(os.path.dirname(os.path.dirname(
            os.path.abspath(__file__))), "_data"))
    path = os.path.join(cache_dir, f"{name}_{tag}.npz")
    cam = Camera(cfg["width"], cfg["height"], cfg["f"], cfg["baseline"])
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Sequence(name, cam, cfg["max_disp"], z["left"], z["right"], z["disp_gt"], z["valid"],
                        z["mover"], z["T"])
    rng = np.random.default_rng(cfg["seed"])
    K = cfg["frames"]
    cs, Rs = _ego_poses(K, cfg["speed"], cfg["yaw"], rng)
    if cfg["scene"] == "tiny":
        prims = _scene_tiny(K, rng)
    else:
        prims = _scene_movers(K, cfg["speed"], rng, cfg.get("cars", 4), 1.65, cs, cfg.get("near"))
    T = _relative_T(cs, Rs)
    D = cfg["max_disp"]
    L, R, G, V, M = [], [], [], [], []
    for k in range(K):
        Z, tex, mov = _render(prims, cam, cs[k], Rs[k], k)
        l, r, d, v = _stereo_pair(Z, tex, cam, D, rng, cfg["noise"])
        L.append(l), R.append(r), G.append(d), V.append(v), M.append(mov)
    seq = Sequence(name, cam, D, np.stack(L), np.stack(R), np.stack(G), np.stack(V), np.stack(M), T)
    if not cache:
        return seq
    try:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, left=seq.left, right=seq.right, disp_gt=seq.disp_gt, valid=seq.valid,
                 mover=seq.mover, T=seq.T)
        os.replace(tmp, path)
    except OSError:
        pass
    return seq


# ----------------------------------------------------------------------------
# small random inputs for unit-level parity cases
# ----------------------------------------------------------------------------

def random_windows(rng: np.random.Generator, H: int, W: int, D: int, max_width: int = 12,
                   full_frac: float = 0.1, smooth: bool = True):
    """Random per-pixel inclusive windows [lo, hi] inside [0, D-1].

    With `smooth`, window centres follow a random smooth surface (as a real
    prediction would) with occasional jumps; `full_frac` of the pixels get the
    full range.  Returns (lo, hi) as int32 [H, W].
    """
    if smooth:
        yy, xx = np.mgrid[0:H, 0:W]
        cen = (D / 2 + (D / 3) * np.sin(xx / max(W, 1) * rng.uniform(1, 6) + rng.uniform(0, 6))
               * np.cos(yy / max(H, 1) * rng.uniform(1, 4)))
        jumps = rng.random((H, W)) < 0.03
        cen = np.where(jumps, rng.uniform(0, D - 1, (H, W)), cen)
    else:
        cen = rng.uniform(0, D - 1, (H, W))
    half = rng.integers(0, max(1, max_width // 2) + 1, (H, W))
    lo = np.clip(np.floor(cen) - half, 0, D - 1).astype(np.int32)
    hi = np.clip(np.floor(cen) + half + rng.integers(0, 2, (H, W)), 0, D - 1).astype(np.int32)
    hi = np.maximum(hi, lo)
    full = rng.random((H, W)) < full_frac
    lo = np.where(full, 0, lo).astype(np.int32)
    hi = np.where(full, D - 1, hi).astype(np.int32)
    return lo, hi


def synthetic_cost_volume(rng: np.random.Generator, H: int, W: int, D: int, cmax: int = 62):
    """Dense random integer costs in [0, cmax] with a planted minimum per pixel."""
    C = rng.integers(0, cmax + 1, (H, W, D)).astype(np.int32)
    return C


def random_state(rng: np.random.Generator, H: int, W: int, D: int, base: Optional[np.ndarray] = None):
    """Random filter state (d, p, flags) for prediction-stage parity cases."""
    if base is None:
        yy, xx = np.mgrid[0:H, 0:W]
        base = 8.0 + (D * 0.4) * (yy / max(H - 1, 1)) + 3.0 * np.sin(xx / 7.0)
    d = np.clip(base + rng.normal(0, 0.3, (H, W)), 0, D - 1).astype(np.float64)
    p = rng.uniform(0.4, 1.0, (H, W)).astype(np.float64)
    flags = np.zeros((H, W), dtype=np.uint8)
    return d, p, flags
