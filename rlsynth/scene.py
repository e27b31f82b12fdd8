"""Seeded synthetic RGB-D rooms: the stand-in for the paper's indoor RGB-D
sequences (7-Scenes / Stanford 4 Scenes), which are not available here.

This module only *generates inputs*: room geometry, camera poses, rendered
depth/colour frames and the dropout/noise models the paper uses in its
robustness study (missing depth: zero a pixel iff r <= p with r ~ U[0,1];
depth-dependent noise d + n*d with n ~ N(0, sigma^2); Sec. "Robustness to
Missing/Noisy Depth").  It contains none of the relocaliser's arithmetic, so
the oracle and the GPU path may both consume its output.

Conventions
-----------
* World frame: metres, z up.  The room is the box [0,4]x[0,4]x[0,3].
* Camera frame: OpenCV (x right, y down, z forward).
* A pose is a 4x4 float64 camera-to-world matrix (the paper's hypotheses map
  camera space to world space, Sec. 3.2.3).
* Depth is the camera-space z of the first surface hit, float32 metres,
  0.0 = invalid.  RGB is uint8 (h, w, 3).
* Pixel (u, v) is the integer column/row; its ray is K^-1 (u, v, 1)^T.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOM_MIN = np.array([0.0, 0.0, 0.0])
ROOM_MAX = np.array([4.0, 4.0, 3.0])
DEPTH_MIN = 0.5
DEPTH_MAX = 4.0


@dataclasses.dataclass
class Surface:
    p0: np.ndarray          # a point on the plane (quad centre for quads)
    n: np.ndarray           # unit normal
    e1: np.ndarray          # in-plane unit axis
    e2: np.ndarray          # in-plane unit axis (n x e1)
    half: tuple | None      # (half_a, half_b) for quads, None for infinite walls
    base: np.ndarray        # (3,) texture base colour
    lam: np.ndarray         # (3,) wavelengths lambda1..3 (m)
    phi: np.ndarray         # (3,) phases
    amp1: np.ndarray        # (3,) square-wave amplitude per channel
    amp2: np.ndarray        # (3,) sinusoid amplitude per channel
    theta: float            # sinusoid orientation
    cell: float = 0.15      # value-noise lattice spacing (m)
    lattice: np.ndarray = None   # (G, G, 3) value-noise lattice, coarse octave
    lattice2: np.ndarray = None  # (G2, G2, 3) value-noise lattice, fine octave


@dataclasses.dataclass
class Room:
    seed: int
    surfaces: list

    @property
    def walls(self):
        return [s for s in self.surfaces if s.half is None]

    @property
    def quads(self):
        return [s for s in self.surfaces if s.half is not None]


def _frame_axes(n):
    helper = np.array([0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(n, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    return e1, e2


LATTICE_EXTENT = 6.0   # plane coordinates covered by the noise lattice: [-6, 6] m


def _texture(rng):
    cell = float(rng.uniform(0.08, 0.25))
    g = int(math.ceil(2 * LATTICE_EXTENT / cell)) + 2
    g2 = int(math.ceil(2 * LATTICE_EXTENT / (cell / 3))) + 2
    return dict(
        base=rng.integers(48, 208, size=3).astype(np.float64),
        lam=rng.uniform(0.1, 0.5, size=3),
        phi=rng.uniform(0.0, 2 * math.pi, size=3),
        amp1=rng.uniform(20.0, 60.0, size=3),
        amp2=rng.uniform(10.0, 40.0, size=3),
        theta=float(rng.uniform(0.0, math.pi)),
        cell=cell,
        lattice=rng.uniform(-70.0, 70.0, size=(g, g, 3)),
        lattice2=rng.uniform(-25.0, 25.0, size=(g2, g2, 3)),
    )


def _value_noise(lat, cell, a, b):
    """Bilinear interpolation of a random lattice with spacing ``cell``."""
    fa = (np.clip(a, -LATTICE_EXTENT, LATTICE_EXTENT) + LATTICE_EXTENT) / cell
    fb = (np.clip(b, -LATTICE_EXTENT, LATTICE_EXTENT) + LATTICE_EXTENT) / cell
    ia = np.minimum(np.floor(fa).astype(np.int64), lat.shape[0] - 2)
    ib = np.minimum(np.floor(fb).astype(np.int64), lat.shape[1] - 2)
    ta = (fa - ia)[:, None]
    tb = (fb - ib)[:, None]
    return ((1 - ta) * (1 - tb) * lat[ia, ib] + ta * (1 - tb) * lat[ia + 1, ib]
            + (1 - ta) * tb * lat[ia, ib + 1] + ta * tb * lat[ia + 1, ib + 1])


def make_room(seed: int, n_quads: int = 6) -> Room:
    """Box room [0,4]x[0,4]x[0,3] (6 walls) plus ``n_quads`` random quads.

    Quad centre ~ U([0.5,3.5]^2 x [0.3,2.7]), normal uniform on S^2,
    half-extents ~ U[0.2,0.8] m.  Every surface carries its own seeded
    procedural texture (see :func:`shade`).
    """
    rng = np.random.default_rng(10_000 + seed)
    surfaces = []
    walls = [
        (np.array([0.0, 0, 0]), np.array([1.0, 0, 0])),
        (np.array([4.0, 0, 0]), np.array([-1.0, 0, 0])),
        (np.array([0.0, 0, 0]), np.array([0, 1.0, 0])),
        (np.array([0.0, 4, 0]), np.array([0, -1.0, 0])),
        (np.array([0.0, 0, 0]), np.array([0, 0, 1.0])),
        (np.array([0.0, 0, 3]), np.array([0, 0, -1.0])),
    ]
    for p0, n in walls:
        e1, e2 = _frame_axes(n)
        surfaces.append(Surface(p0=p0, n=n, e1=e1, e2=e2, half=None, **_texture(rng)))
    for _ in range(n_quads):
        c = np.array([rng.uniform(0.5, 3.5), rng.uniform(0.5, 3.5), rng.uniform(0.3, 2.7)])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        e1, e2 = _frame_axes(n)
        half = (float(rng.uniform(0.2, 0.8)), float(rng.uniform(0.2, 0.8)))
        surfaces.append(Surface(p0=c, n=n, e1=e1, e2=e2, half=half, **_texture(rng)))
    return Room(seed=seed, surfaces=surfaces)


def surface_records(room: Room) -> np.ndarray:
    """The room's geometry as the library's analytic scene model: 16 float32
    per surface (point, unit normal, in-plane axes, half-extents; 0 for the
    infinite walls), the layout of rl_surface."""
    out = np.zeros((len(room.surfaces), 16), dtype=np.float32)
    for i, s in enumerate(room.surfaces):
        out[i, 0:3], out[i, 3:6], out[i, 6:9], out[i, 9:12] = s.p0, s.n, s.e1, s.e2
        if s.half is not None:
            out[i, 12:14] = s.half
    return out


def intrinsics(w: int, h: int):
    """fx = fy = 585 * w / 640, principal point at the image centre."""
    f = 585.0 * w / 640.0
    return (np.float32(f), np.float32(f), np.float32(w / 2.0), np.float32(h / 2.0))


TEXTURE = "noise"   # "noise" (non-periodic value noise) or "periodic"


def shade(surf: Surface, a: np.ndarray, b: np.ndarray, texture: str | None = None) -> np.ndarray:
    """Procedural texture at plane coordinates (a, b), clamped to uint8.

    "noise": per-surface base colour plus two octaves of value noise (random
    lattice, spacing ``cell`` and ``cell/3``): locally unique appearance, as
    in real indoor scenes.  "periodic": base colour plus a square-wave
    checker and an oriented sinusoid (strongly aliased)."""
    texture = texture or TEXTURE
    if texture == "noise":
        col = (surf.base[None, :] + _value_noise(surf.lattice, surf.cell, a, b)
               + _value_noise(surf.lattice2, surf.cell / 3, a, b))
        return np.clip(np.rint(col), 0, 255).astype(np.uint8)
    sq = np.sign(np.sin(2 * math.pi * a / surf.lam[0] + surf.phi[0])
                 * np.sin(2 * math.pi * b / surf.lam[1] + surf.phi[1]))
    sn = np.sin(2 * math.pi * (a * math.cos(surf.theta) + b * math.sin(surf.theta)) / surf.lam[2]
                + surf.phi[2])
    col = surf.base[None, :] + sq[:, None] * surf.amp1[None, :] + sn[:, None] * surf.amp2[None, :]
    return np.clip(np.rint(col), 0, 255).astype(np.uint8)


def raycast(room: Room, pose: np.ndarray, w: int, h: int, K=None):
    """Noise-free render: returns (depth float64 (h,w) with inf for no hit,
    rgb uint8 (h,w,3), surface index int (h,w), -1 for no hit)."""
    fx, fy, cx, cy = [float(v) for v in (K if K is not None else intrinsics(w, h))]
    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    dc = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1).reshape(-1, 3)
    R = pose[:3, :3]
    o = pose[:3, 3]
    dw = dc @ R.T
    best = np.full(dw.shape[0], np.inf)
    idx = np.full(dw.shape[0], -1, dtype=np.int64)
    for si, s in enumerate(room.surfaces):
        denom = dw @ s.n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = ((s.p0 - o) @ s.n) / denom
        ok = (np.abs(denom) > 1e-12) & (t > 1e-6)
        if s.half is not None:
            hit = o[None, :] + t[:, None] * dw
            rel = hit - s.p0[None, :]
            a = rel @ s.e1
            b = rel @ s.e2
            ok &= (np.abs(a) <= s.half[0]) & (np.abs(b) <= s.half[1])
        upd = ok & (t < best)
        best[upd] = t[upd]
        idx[upd] = si
    rgb = np.zeros((dw.shape[0], 3), dtype=np.uint8)
    for si, s in enumerate(room.surfaces):
        m = idx == si
        if not np.any(m):
            continue
        hit = o[None, :] + best[m][:, None] * dw[m]
        rel = hit - s.p0[None, :]
        rgb[m] = shade(s, rel @ s.e1, rel @ s.e2)
    # ray parameter t equals the camera-space depth because dc has z = 1
    return best.reshape(h, w), rgb.reshape(h, w, 3), idx.reshape(h, w)


def render(room: Room, pose: np.ndarray, w: int, h: int, seed: int,
           noise_sigma: float = 0.002, dropout: float = 0.05,
           depth_rel_sigma: float = 0.0, K=None):
    """Render a noisy RGB-D frame.

    Depth outside [0.5, 4] m becomes 0; valid depth gets additive
    N(0, noise_sigma^2) noise and optionally depth-dependent noise
    d + n*d, n ~ N(0, depth_rel_sigma^2); then each pixel is zeroed iff
    r <= dropout, r ~ U[0,1].  Returns (depth float32 (h,w), rgb uint8 (h,w,3)).
    """
    z, rgb, _ = raycast(room, pose, w, h, K)
    return corrupt(z, seed, noise_sigma, dropout, depth_rel_sigma), rgb


def corrupt(z: np.ndarray, seed: int, noise_sigma: float = 0.002, dropout: float = 0.05,
            depth_rel_sigma: float = 0.0) -> np.ndarray:
    """The sensor model of render() applied to a noise-free depth map z
    (inf where no surface): float32 depth, 0 = invalid."""
    rng = np.random.default_rng(seed)
    valid = np.isfinite(z) & (z >= DEPTH_MIN) & (z <= DEPTH_MAX)
    d = np.where(valid, z, 0.0)
    if noise_sigma > 0:
        d = np.where(valid, d + rng.normal(0.0, noise_sigma, size=d.shape), 0.0)
    if depth_rel_sigma > 0:
        d = np.where(valid, d + rng.normal(0.0, depth_rel_sigma, size=d.shape) * d, 0.0)
    if dropout > 0:
        r = rng.uniform(0.0, 1.0, size=d.shape)
        d = np.where(r <= dropout, 0.0, d)
    d = np.where(d > 0, d, 0.0)
    return d.astype(np.float32)


def _rot_axis(axis, ang):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * kx + (1 - math.cos(ang)) * kx @ kx


def look_pose(pos, yaw, pitch, roll):
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    right = np.cross(f, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f], axis=1)
    R = _rot_axis(f, roll) @ R
    H = np.eye(4)
    H[:3, :3] = R
    H[:3, 3] = pos
    return H


def valid_fraction(room, pose, w=40, h=30):
    z, _, _ = raycast(room, pose, w, h, intrinsics(w, h))
    return float(np.mean(np.isfinite(z) & (z >= DEPTH_MIN) & (z <= DEPTH_MAX)))


def random_pose(room: Room, rng, min_valid=0.8):
    """Position U([0.6,3.4]^2 x [1.0,2.0]); yaw U[0,2pi); pitch U[-30,15] deg;
    roll U[-10,10] deg; re-drawn until >= min_valid of the pixels lie in range."""
    while True:
        pos = np.array([rng.uniform(0.6, 3.4), rng.uniform(0.6, 3.4), rng.uniform(1.0, 2.0)])
        H = look_pose(pos, rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(-30, 15)),
                      math.radians(rng.uniform(-10, 10)))
        if valid_fraction(room, H) >= min_valid:
            return H


def near_pose(room: Room, base: np.ndarray, rng, max_t: float, max_deg: float,
              min_t: float = 0.0, min_deg: float = 0.0, min_valid=0.8, max_tries=1000):
    """A pose within [min_t, max_t] metres and [min_deg, max_deg] degrees of
    ``base`` (random direction / random rotation axis)."""
    for _ in range(max_tries):
        d = rng.normal(size=3)
        d *= rng.uniform(min_t, max_t) / np.linalg.norm(d)
        ang = math.radians(rng.uniform(min_deg, max_deg))
        H = np.eye(4)
        H[:3, :3] = _rot_axis(rng.normal(size=3), ang) @ base[:3, :3]
        H[:3, 3] = base[:3, 3] + d
        p = H[:3, 3]
        if np.all(p > ROOM_MIN + 0.3) and np.all(p < ROOM_MAX - 0.3) and valid_fraction(room, H) >= min_valid:
            return H
    raise RuntimeError("near_pose: no valid pose found")


def pose_error(Ha: np.ndarray, Hb: np.ndarray):
    """(translation error in metres, rotation error in degrees)."""
    dt = float(np.linalg.norm(Ha[:3, 3] - Hb[:3, 3]))
    Rd = Ha[:3, :3].T @ Hb[:3, :3]
    c = np.clip((np.trace(Rd) - 1) / 2, -1.0, 1.0)
    return dt, math.degrees(math.acos(c))
