"""Seeded synthetic LiDAR scenes and sequences (test and benchmark *input* only).

This module produces point clouds; it holds none of the compression method's
arithmetic.  It ray-casts a spinning multi-beam sensor against a procedural
scene (ground plane, axis-aligned boxes, vertical cylinders) along the pixel
centre directions of the sensor grid, adds Gaussian range noise along the ray
and drops returns at random.  Sequences move the sensor forward with a small
yaw change per frame and move a few car-sized boxes, so that the predicted
frames of Section III-D (temporal encoding) see rigid ego-motion plus
independently moving objects.

Random numbers come from ``numpy.random.Generator(PCG64)`` seeded by
``SeedSequence([seed, stream])``, so every array is a pure function of the
seed.  The paper's experiments use KITTI (HDL-64E) scans; these scenes stand
in for them and reproduce no dataset content.

Conventions shared with the sensor model of the encoder (a fact about the
sensor, not an implementation detail): row 0 is the top beam, elevations are
strictly descending, column ``u`` covers the clockwise azimuth interval
``(az0 - (u+1)*2pi/W, az0 - u*2pi/W]`` and its centre is at
``az0 - (u + 1/2)*2pi/W``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEG = math.pi / 180.0
GROUND_Z = -1.7


# --------------------------------------------------------------------------
# sensors
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Sensor:
    """A spinning sensor with ``H`` beams at uniform elevations and ``W`` azimuth bins."""

    H: int
    W: int
    top_deg: float
    bot_deg: float
    az0: float = math.pi

    def elevations(self) -> np.ndarray:
        """Beam elevations in radians, FP32, strictly descending (row 0 = top)."""
        e = np.linspace(self.top_deg, self.bot_deg, self.H, dtype=np.float64) * DEG
        return e.astype(np.float32)

    @property
    def pixels(self) -> int:
        return self.H * self.W


SENSORS = {
    # 16 beams, +-15 deg, 512 bins (small single-frame case)
    "c1": Sensor(16, 512, 15.0, -15.0),
    # HDL-64E-like: 64 beams from +2 to -24.8 deg, 2048 bins
    "c2": Sensor(64, 2048, 2.0, -24.8),
    # the seed network's sensor: 128 beams from +15 to -25 deg, 2048 bins
    # (config-2 style scenes)
    "c5": Sensor(128, 2048, 15.0, -25.0),
}


# The five workloads the encoder is measured and tested on, by name: the
# sensors, the scene kind, tile shape, error bounds, frames per sequence
# with the key frame's index, sequences, and the first seed.
WORKLOADS = {
    "single-16": dict(sensors=("c1",), scene="c1", tile=(4, 4), eps=(0.02,), frames=1, key=0, sequences=1, seed=1000),
    "single-64": dict(sensors=("c2",), scene="c2", tile=(4, 8), eps=(0.02,), frames=1, key=0, sequences=1, seed=2000),
    "sequence-16": dict(sensors=("c1",), scene="c1", tile=(4, 4), eps=(0.02,), frames=10, key=0, sequences=1,
                        seed=3000),
    "batch-uneven": dict(sensors=tuple(f"{b}x{w}" for b, w in ((16, 1024), (16, 2048), (32, 1024), (32, 2048),
                                                                (64, 1024), (64, 2048), (128, 1024), (128, 2048))),
                         scene="c1", tile=None, eps=(0.01, 0.02), frames=10, key=5, sequences=96, seed=4000),
    "learned-128": dict(sensors=("c5",), scene="c2", tile=(4, 8), eps=(0.02,), frames=10, key=5, sequences=200,
                        seed=900000),
}


def workload_sensor(name: str) -> Sensor:
    """A WORKLOADS sensor name: a SENSORS key, or "BxW" for the uneven batch."""
    if name in SENSORS:
        return SENSORS[name]
    b, w = name.split("x")
    return mixed_sensor(int(b), int(w))


def mixed_sensor(beams: int, width: int) -> Sensor:
    """Sensors of the uneven batch: 16 beams span +-15 deg, 64 beams the HDL-64E
    fan, 32 and 128 beams span +15..-25 deg."""
    if beams == 16:
        return Sensor(16, width, 15.0, -15.0)
    if beams == 64:
        return Sensor(64, width, 2.0, -24.8)
    if beams in (32, 128):
        return Sensor(beams, width, 15.0, -25.0)
    raise ValueError(f"no preset for {beams} beams")


# The uneven batch: every beam count with every azimuth resolution.
MIXED = tuple((b, w) for b in (16, 32, 64, 128) for w in (1024, 2048))


def mixed_sequence(q: int, seed0: int = 4000, n_frames: int = 10, key_index: int = 5):
    """Sequence q of the uneven batch: sensor MIXED[q % 8] (so any run of 8
    consecutive sequences holds every sensor), a config-1 style scene with
    the moving cars of the sequences, seed seed0 + q."""
    s = mixed_sensor(*MIXED[q % len(MIXED)])
    return make_sequence(s, "c1", seed0 + q, n_frames=n_frames, key_index=key_index, moving=5, shuffle=True)


def pixel_directions(sensor: Sensor) -> np.ndarray:
    """Unit ray directions (H, W, 3) in FP64 at the pixel centres, sensor frame."""
    e = sensor.elevations().astype(np.float64)
    a = sensor.az0 - (np.arange(sensor.W, dtype=np.float64) + 0.5) * (2.0 * math.pi / sensor.W)
    ce, se = np.cos(e)[:, None], np.sin(e)[:, None]
    d = np.empty((sensor.H, sensor.W, 3), dtype=np.float64)
    d[..., 0] = ce * np.cos(a)[None, :]
    d[..., 1] = ce * np.sin(a)[None, :]
    d[..., 2] = np.broadcast_to(se, (sensor.H, sensor.W))
    return d


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
@dataclass
class Scene:
    boxes_lo: np.ndarray            # (B, 3) world-frame lower corners
    boxes_hi: np.ndarray            # (B, 3) upper corners
    boxes_vel: np.ndarray           # (B, 3) metres per frame (0 for static boxes)
    cyl: np.ndarray                 # (C, 5) cx, cy, radius, z0, z1
    sigma: float                    # range noise (m)
    dropout: float                  # Bernoulli dropout probability
    cap: float = 120.0              # no return beyond this range
    ground_z: float = GROUND_Z


def _place_boxes(rng, n, sizes, dist, existing, corridor):
    """Rejection-sample ``n`` axis-aligned boxes that overlap neither each other,
    ``existing`` boxes, the sensor origin nor the ego corridor."""
    lo, hi = [], []
    tries = 0
    while len(lo) < n:
        tries += 1
        if tries > 20000:
            raise RuntimeError("could not place boxes")
        sx, sy, sz = (rng.uniform(*s) for s in sizes)
        if rng.uniform() < 0.5:       # random footprint orientation (axis aligned)
            sx, sy = sy, sx
        r = rng.uniform(*dist)
        az = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = r * math.cos(az), r * math.sin(az)
        blo = np.array([cx - sx / 2, cy - sy / 2, GROUND_Z])
        bhi = np.array([cx + sx / 2, cy + sy / 2, GROUND_Z + sz])
        if blo[0] < 1.0 and bhi[0] > -1.0 and blo[1] < 1.0 and bhi[1] > -1.0:
            continue
        if corridor is not None:
            cx0, cx1, cy0, cy1 = corridor
            if blo[0] < cx1 and bhi[0] > cx0 and blo[1] < cy1 and bhi[1] > cy0:
                continue
        ok = True
        for (l2, h2) in list(zip(lo, hi)) + list(existing):
            if blo[0] < h2[0] + 0.3 and bhi[0] > l2[0] - 0.3 and blo[1] < h2[1] + 0.3 and bhi[1] > l2[1] - 0.3:
                ok = False
                break
        if ok:
            lo.append(blo)
            hi.append(bhi)
    return lo, hi


def make_scene(kind: str, rng: np.random.Generator, moving: int = 0, corridor=None) -> Scene:
    """Scene recipes.

    ``"c1"``: ground + 4 boxes, footprint sides U(2,6) m, height U(1.5,4) m,
    centre distance U(5,30) m; sigma 1 cm, 3 % dropout.
    ``"c2"``: ground + 20 car-like boxes (1.6-2.0 x 3.8-4.8 x 1.4-1.8 m at
    5-40 m) + 20 building-like boxes (6-20 m sides, 4-15 m tall at 15-100 m)
    + 30 vertical cylinders (r U(0.1,0.3) m, height U(2,6) m at 3-60 m);
    sigma 2 cm, 5 % dropout.
    ``moving`` car-sized boxes are added with a constant horizontal velocity of
    magnitude U(0,1) m/frame.
    """
    existing = []
    if kind == "c1":
        lo, hi = _place_boxes(rng, 4, [(2, 6), (2, 6), (1.5, 4)], (5, 30), existing, corridor)
        cyl = np.zeros((0, 5))
        sigma, dropout = 0.01, 0.03
    elif kind == "c2":
        lo, hi = _place_boxes(rng, 20, [(1.6, 2.0), (3.8, 4.8), (1.4, 1.8)], (5, 40), existing, corridor)
        existing = list(zip(lo, hi))
        lo2, hi2 = _place_boxes(rng, 20, [(6, 20), (6, 20), (4, 15)], (15, 100), existing, corridor)
        lo, hi = lo + lo2, hi + hi2
        c = []
        while len(c) < 30:
            r = rng.uniform(3, 60)
            az = rng.uniform(0, 2 * math.pi)
            rad = rng.uniform(0.1, 0.3)
            h = rng.uniform(2, 6)
            cx, cy = r * math.cos(az), r * math.sin(az)
            if corridor is not None:
                x0, x1, y0, y1 = corridor
                if x0 - rad < cx < x1 + rad and y0 - rad < cy < y1 + rad:
                    continue
            inside = any(l[0] - rad < cx < h_[0] + rad and l[1] - rad < cy < h_[1] + rad for l, h_ in zip(lo, hi))
            if inside:
                continue
            c.append([cx, cy, rad, GROUND_Z, GROUND_Z + h])
        cyl = np.array(c)
        sigma, dropout = 0.02, 0.05
    else:
        raise ValueError(kind)
    vel = [np.zeros(3)] * len(lo)
    if moving:
        mlo, mhi = _place_boxes(rng, moving, [(1.6, 2.0), (3.8, 4.8), (1.4, 1.8)], (6, 30),
                                list(zip(lo, hi)), corridor)
        for _ in range(moving):
            speed = rng.uniform(0.0, 1.0)
            ang = rng.uniform(0, 2 * math.pi)
            vel.append(np.array([speed * math.cos(ang), speed * math.sin(ang), 0.0]))
        lo, hi = lo + mlo, hi + mhi
    return Scene(np.array(lo).reshape(-1, 3), np.array(hi).reshape(-1, 3),
                 np.array(vel).reshape(-1, 3), cyl, sigma, dropout)


# --------------------------------------------------------------------------
# ray casting
# --------------------------------------------------------------------------
def _column_window(sensor: Sensor, center_xy, radius):
    """Columns whose rays can reach a vertical object of xy bounding radius
    ``radius`` centred at ``center_xy`` (sensor frame); wraps at W."""
    W = sensor.W
    dist = math.hypot(center_xy[0], center_xy[1])
    if dist <= radius + 0.5:
        return np.arange(W)
    psi = math.atan2(center_xy[1], center_xy[0])
    half = math.asin(min(1.0, radius / dist))
    dth = 2 * math.pi / W
    uc = (sensor.az0 - psi) / dth - 0.5
    lo = int(math.floor(uc - half / dth)) - 2
    hi = int(math.ceil(uc + half / dth)) + 2
    if hi - lo + 1 >= W:
        return np.arange(W)
    return np.arange(lo, hi + 1) % W


def render(sensor: Sensor, scene: Scene, R: np.ndarray, P: np.ndarray, frame: int,
           rng: np.random.Generator):
    """Ray-cast one frame from pose (R, P) (sensor-to-world rotation and position).

    Returns ``(points, rows, cols)``: FP32 points (N, 3) in the sensor frame in
    raster order of the pixel they were cast from, and that pixel's indices.
    """
    H, W = sensor.H, sensor.W
    d = pixel_directions(sensor)                          # (H, W, 3) sensor frame
    dw = d @ R.T                                          # world-frame directions
    t_best = np.full((H, W), np.inf)
    # ground plane z = ground_z (the sensor moves in a horizontal plane)
    dz = dw[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < -1e-12, (scene.ground_z - P[2]) / dz, np.inf)
    t_best = np.minimum(t_best, np.where(tg > 0, tg, np.inf))
    Rt = R.T
    # boxes (axis aligned in the world frame, translated by velocity * frame)
    for lo, hi, v in zip(scene.boxes_lo, scene.boxes_hi, scene.boxes_vel):
        lo = lo + v * frame
        hi = hi + v * frame
        c = Rt @ ((lo + hi) / 2 - P)
        rad = 0.5 * math.hypot(hi[0] - lo[0], hi[1] - lo[1])
        cols = _column_window(sensor, c[:2], rad)
        D = dw[:, cols, :]
        Dn = np.where(np.abs(D) < 1e-15, 1e-15, D)
        t1 = (lo - P) / Dn
        t2 = (hi - P) / Dn
        tmin = np.max(np.minimum(t1, t2), axis=-1)
        tmax = np.min(np.maximum(t1, t2), axis=-1)
        hit = (tmax >= tmin) & (tmax > 1e-6)
        th = np.where(tmin > 1e-6, tmin, tmax)
        th = np.where(hit, th, np.inf)
        t_best[:, cols] = np.minimum(t_best[:, cols], th)
    # vertical cylinders (side surface)
    for cx, cy, rad, z0, z1 in scene.cyl:
        c = Rt @ (np.array([cx, cy, (z0 + z1) / 2]) - P)
        cols = _column_window(sensor, c[:2], rad)
        D = dw[:, cols, :]
        ox, oy = P[0] - cx, P[1] - cy
        a = D[..., 0] ** 2 + D[..., 1] ** 2
        b = 2 * (D[..., 0] * ox + D[..., 1] * oy)
        cc = ox * ox + oy * oy - rad * rad
        disc = b * b - 4 * a * cc
        with np.errstate(invalid="ignore", divide="ignore"):
            sq = np.sqrt(np.maximum(disc, 0))
            t0 = (-b - sq) / (2 * a)
        z = P[2] + t0 * D[..., 2]
        ok = (disc > 0) & (t0 > 1e-6) & (z >= z0) & (z <= z1)
        t_best[:, cols] = np.minimum(t_best[:, cols], np.where(ok, t0, np.inf))
    hit = np.isfinite(t_best) & (t_best <= scene.cap)
    noise = rng.normal(0.0, scene.sigma, size=(H, W))
    keep = hit & (rng.uniform(size=(H, W)) >= scene.dropout)
    tn = t_best + noise
    keep &= tn > 0.05
    rows, cols = np.nonzero(keep)
    pts = (tn[rows, cols][:, None] * d[rows, cols, :]).astype(np.float32)
    return pts, rows.astype(np.int32), cols.astype(np.int32)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def make_frame(sensor: Sensor, kind: str, seed: int):
    """One key frame in the sensor's own coordinates (no ego-motion)."""
    scene = make_scene(kind, _rng(seed, 0))
    pts, rows, cols = render(sensor, scene, np.eye(3), np.zeros(3), 0, _rng(seed, 1))
    return pts, rows, cols


def rotz(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


@dataclass
class Sequence:
    sensor: Sensor
    frames: list                    # FP32 (N_i, 3) points in each frame's sensor frame
    transforms: np.ndarray          # (n, 4, 4) FP32: frame i -> key frame coordinates
    key_index: int
    poses: list = field(default_factory=list)   # (R, P) FP64 sensor-to-world


def make_sequence(sensor: Sensor, kind: str, seed: int, n_frames: int = 10,
                  key_index: int | None = None, moving: int = 5, shuffle: bool = False,
                  imu_noise: float = 0.0, corridor_frames: int | None = None) -> Sequence:
    """A group of consecutive frames with ego-motion 0.8-1.2 m forward and a
    yaw change of U(-0.5, 0.5) deg per frame, plus ``moving`` independently
    moving car-sized boxes.  The transform of frame i into the key frame is
    ``pose_K^-1 pose_i`` in FP64, rounded to FP32; with ``imu_noise`` = s > 0
    it is perturbed by N(0, s x 5 cm) translation (a fifth of that in z) and
    N(0, s x 0.1 deg) yaw (True counts as s = 1).  The track's obstacle-free
    corridor is sized for ``corridor_frames`` frames (default ``n_frames``), so
    sequences of different lengths can share one scene distribution."""
    if key_index is None:
        key_index = n_frames // 2
    rng = _rng(seed, 0)
    nc = n_frames if corridor_frames is None else max(n_frames, corridor_frames)
    corridor = (-2.0 * nc - 5, 2.0 * nc + 5, -3.0, 3.0)
    scene = make_scene(kind, rng, moving=moving, corridor=corridor)
    poses = []
    heading, pos = 0.0, np.zeros(3)
    # frame k sits at the origin-centred middle of the track so the scene
    # surrounds the whole sequence
    steps = [(rng.uniform(0.8, 1.2), rng.uniform(-0.5, 0.5) * DEG) for _ in range(n_frames)]
    for i in range(n_frames):
        poses.append((rotz(heading), pos.copy()))
        fwd, dyaw = steps[i]
        pos = pos + fwd * np.array([math.cos(heading), math.sin(heading), 0.0])
        heading += dyaw
    # recentre so the key frame is at the world origin
    Rk0, Pk0 = poses[key_index]
    poses = [(Rk0.T @ R, Rk0.T @ (P - Pk0)) for (R, P) in poses]
    # scene boxes move with frame index relative to the key frame
    frames = []
    Ms = np.zeros((n_frames, 4, 4), dtype=np.float32)
    RK, PK = poses[key_index]
    for i, (R, P) in enumerate(poses):
        pts, _, _ = render(sensor, scene, R, P, i - key_index, _rng(seed, 1 + i))
        if shuffle:
            pts = pts[_rng(seed, 10_000 + i).permutation(len(pts))]
        frames.append(np.ascontiguousarray(pts))
        M = np.eye(4)
        M[:3, :3] = RK.T @ R
        M[:3, 3] = RK.T @ (P - PK)
        if imu_noise and i != key_index:
            sc = float(imu_noise)
            nr = _rng(seed, 20_000 + i)
            M[:3, :3] = rotz(nr.normal(0, 0.1 * DEG) * sc) @ M[:3, :3]
            M[:3, 3] += nr.normal(0, 0.05, size=3) * np.array([1, 1, 0.2]) * sc
        Ms[i] = M.astype(np.float32)
    return Sequence(sensor, frames, Ms, key_index, poses)
