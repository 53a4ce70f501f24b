"""Seeded synthetic inputs for the probe update and probe query.

This module produces only *inputs*: triangle scenes, lights, probe-volume
descriptions, per-frame random rotations and query points.  It contains
none of the method's arithmetic (no ray traversal of the triangle scene, no
octahedral mapping, no blending, no query weights), so that the same inputs
can be handed both to the GPU library and to the independent CPU oracle.

Random numbers come from SplitMix64 used as a counter-based generator:
output i of stream s of workload c is ``mix(seed + (i + 1) * GAMMA)`` with
``seed = 1000 * c + s``; a uniform double is ``(x >> 11) * 2**-53``.

Streams: 1 geometry, 2 lights, 3 rotations, 4 queries, 5 camera,
6 target perturbation.

Conventions (shared by every consumer of these inputs):
  * triangles are counter-clockwise seen from their front side; the front
    normal is ``(v1 - v0) x (v2 - v0)``;
  * ``tri_object`` is 0 for static triangles, k > 0 for dynamic object k;
  * rotations are row-major 3x3 float32 matrices;
  * probe ``q`` of a grid with counts (nx, ny, nz) has grid index
    ``(i, j, k)`` with ``q = i + nx * (j + ny * k)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# probe states (numeric codes shared with the C ABI)
OFF, SLEEPING, NEWLY_AWAKE, NEWLY_VIGILANT, AWAKE, VIGILANT = 0, 1, 2, 3, 4, 5

STREAM_GEOMETRY, STREAM_LIGHTS, STREAM_ROTATIONS = 1, 2, 3
STREAM_QUERIES, STREAM_CAMERA, STREAM_TARGET = 4, 5, 6


def splitmix64(seed: int, start: int, n: int) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of SplitMix64 seeded with ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class Stream:
    """Sequential reader over one SplitMix64 stream."""

    def __init__(self, config: int, stream: int):
        self.seed = 1000 * config + stream
        self.pos = 0

    def bits(self, n: int) -> np.ndarray:
        out = splitmix64(self.seed, self.pos, n)
        self.pos += n
        return out

    def uniform(self, n: int, lo=0.0, hi=1.0) -> np.ndarray:
        u = (self.bits(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)

    def unit_vectors(self, n: int) -> np.ndarray:
        z = self.uniform(n, -1.0, 1.0)
        phi = self.uniform(n, 0.0, 2.0 * np.pi)
        r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def shoemake_rotation(u1: float, u2: float, u3: float) -> np.ndarray:
    """Haar-uniform rotation from three uniforms (Shoemake 1992), float32."""
    a = math.sqrt(1.0 - u1)
    b = math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
    return R.astype(np.float32)


def rotations(config: int, n: int, start_frame: int = 0) -> np.ndarray:
    """Per-frame rotations [n, 9] (three draws of stream 3 per frame)."""
    s = Stream(config, STREAM_ROTATIONS)
    s.pos = 3 * start_frame
    u = s.uniform(3 * n).reshape(n, 3)
    return np.stack([shoemake_rotation(*row).reshape(9) for row in u])


# --------------------------------------------------------------------------
# containers


@dataclasses.dataclass
class Scene:
    vertices: np.ndarray       # float32 [V, 3]
    indices: np.ndarray        # uint32 [T, 3]
    tri_material: np.ndarray   # uint32 [T]
    tri_object: np.ndarray     # uint32 [T]
    albedo: np.ndarray         # float32 [M, 3]
    emission: np.ndarray       # float32 [M, 3]
    specular: np.ndarray = None  # float32 [M, 3] mirror reflectance (second-order glossy); None = 0

    def specular_or_zero(self) -> np.ndarray:
        if self.specular is None:
            return np.zeros_like(self.albedo)
        return np.asarray(self.specular, dtype=np.float32).reshape(-1, 3)

    @property
    def n_triangles(self) -> int:
        return int(self.indices.shape[0])


@dataclasses.dataclass
class Lights:
    dir_to_light: np.ndarray     # float32 [nd, 3], unit vectors toward the light
    dir_irradiance: np.ndarray   # float32 [nd, 3], irradiance normal to the light
    point_pos: np.ndarray        # float32 [np, 3]
    point_intensity: np.ndarray  # float32 [np, 3], W/sr
    sky: np.ndarray              # float32 [3], radiance of rays that miss


@dataclasses.dataclass
class VolumeDesc:
    origin: tuple
    spacing: tuple
    counts: tuple
    rays_per_probe: int = 64
    hysteresis_irr: float = 0.97
    hysteresis_dist: float = 0.97
    cos_power: float = 50.0
    self_shadow_bias: float = 0.3
    max_distance: float = 0.0    # 0 -> 1.5 * |spacing|
    cheb_power: int = 1
    atlas_f16: bool = False
    blend: str = "f32"           # "f32" | "bf16" | "f16" (matrix cores) | "f32_valu"
    irradiance_gamma: float = 1.0   # perception encoding exponent (1 = linear texels)
    texel_thresholds: bool = False  # per-texel irradiance hysteresis thresholds
    tracking: bool = False       # window that follows the camera, camera-centred blend weight

    @property
    def n_probes(self) -> int:
        return int(self.counts[0] * self.counts[1] * self.counts[2])

    def resolved_max_distance(self) -> float:
        if self.max_distance > 0:
            return float(self.max_distance)
        return float(np.float32(1.5 * math.sqrt(sum(float(s) ** 2 for s in self.spacing))))


@dataclasses.dataclass
class Queries:
    pos: np.ndarray   # float32 [Q, 3]
    nrm: np.ndarray   # float32 [Q, 3]
    view: np.ndarray  # float32 [Q, 3] unit, from the point toward the viewer

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    scene: Scene
    lights: Lights
    volumes: List[VolumeDesc]
    queries: Optional[Queries] = None
    classify_rotations: Optional[np.ndarray] = None   # [K, 9]
    info: dict = dataclasses.field(default_factory=dict)

    def frame_rotation(self, frame: int) -> np.ndarray:
        return rotations(self.config, 1, start_frame=frame)[0]


# --------------------------------------------------------------------------
# geometry builders


class MeshBuilder:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.i: List[np.ndarray] = []
        self.mat: List[np.ndarray] = []
        self.obj: List[np.ndarray] = []
        self.nv = 0

    def add(self, verts, tris, material: int, obj: int = 0):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.v.append(verts)
        self.i.append(tris + self.nv)
        self.mat.append(np.full(len(tris), material, dtype=np.uint32))
        self.obj.append(np.full(len(tris), obj, dtype=np.uint32))
        self.nv += len(verts)

    def grid_quad(self, origin, u, v, nu: int, nv: int, material: int, obj: int = 0):
        """Planar parallelogram origin + a*u + b*v, a,b in [0,1], split into
        nu x nv cells of two triangles each; the front side is u x v."""
        origin, u, v = (np.asarray(x, dtype=np.float64) for x in (origin, u, v))
        a = np.linspace(0.0, 1.0, nu + 1)
        b = np.linspace(0.0, 1.0, nv + 1)
        A, B = np.meshgrid(a, b, indexing="ij")
        verts = origin + A[..., None] * u + B[..., None] * v
        idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
        p00 = idx[:-1, :-1].ravel()
        p10 = idx[1:, :-1].ravel()
        p11 = idx[1:, 1:].ravel()
        p01 = idx[:-1, 1:].ravel()
        tris = np.concatenate([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)])
        self.add(verts.reshape(-1, 3), tris, material, obj)

    def box(self, lo, hi, material: int, obj: int = 0, inward: bool = False,
            cell: float = 0.0, faces=("+x", "-x", "+y", "-y", "+z", "-z")):
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        ext = hi - lo
        ex, ey, ez = np.diag(ext)
        spec = {
            "+x": ((hi[0], lo[1], lo[2]), ey, ez),
            "-x": ((lo[0], lo[1], lo[2]), ez, ey),
            "+y": ((lo[0], hi[1], lo[2]), ez, ex),
            "-y": ((lo[0], lo[1], lo[2]), ex, ez),
            "+z": ((lo[0], lo[1], hi[2]), ex, ey),
            "-z": ((lo[0], lo[1], lo[2]), ey, ex),
        }
        for f in faces:
            o, u, v = spec[f]
            if inward:
                u, v = v, u
            nu = max(1, int(round(np.linalg.norm(u) / cell))) if cell > 0 else 1
            nv = max(1, int(round(np.linalg.norm(v) / cell))) if cell > 0 else 1
            self.grid_quad(o, u, v, nu, nv, material, obj)

    def build(self, albedo, emission) -> Scene:
        return Scene(
            vertices=np.concatenate(self.v).astype(np.float32),
            indices=np.concatenate(self.i).astype(np.uint32),
            tri_material=np.concatenate(self.mat),
            tri_object=np.concatenate(self.obj),
            albedo=np.asarray(albedo, dtype=np.float32).reshape(-1, 3),
            emission=np.asarray(emission, dtype=np.float32).reshape(-1, 3),
        )


def no_lights(sky=(0.0, 0.0, 0.0)) -> Lights:
    z = np.zeros((0, 3), dtype=np.float32)
    return Lights(z, z, z, z, np.asarray(sky, dtype=np.float32))


def _near_any(x: float, planes: np.ndarray, margin: float) -> bool:
    return bool(np.any(np.abs(planes - x) < margin))


# --------------------------------------------------------------------------
# workloads


def config0(n_queries: int = 4096) -> Workload:
    """Closed 8 m room (12 triangles, inward), two seeded boxes (24
    triangles; box B is a dynamic object), an emissive ceiling quad of
    radiance 5 and a directional light that the closed room occludes.
    4x4x4 probes at 2 m spacing from (1,1,1); 64 rays per probe."""
    c = 0
    g = Stream(c, STREAM_GEOMETRY)
    probe_planes = np.array([1.0, 3.0, 5.0, 7.0])
    boxes = []
    while len(boxes) < 2:
        size = g.uniform(3, 1.0, 2.5)
        lo = np.array([g.uniform(1, 0.25, 7.75 - size[0])[0],
                       g.uniform(1, 0.01, 7.75 - size[1])[0],
                       g.uniform(1, 0.25, 7.75 - size[2])[0]])
        hi = lo + size
        ok = all(not _near_any(lo[a], probe_planes, 0.05) and
                 not _near_any(hi[a], probe_planes, 0.05) for a in range(3))
        for (blo, bhi) in boxes:
            if np.all(lo < bhi + 0.05) and np.all(blo < hi + 0.05):
                ok = False
        if ok:
            boxes.append((lo, hi))
    box_albedo = g.uniform(6, 0.2, 0.9).reshape(2, 3)

    mb = MeshBuilder()
    # materials: 0 room, 1 box A, 2 box B, 3 emissive quad
    mb.box((0, 0, 0), (8, 8, 8), material=0, inward=True)
    mb.box(boxes[0][0], boxes[0][1], material=1, obj=0)
    mb.box(boxes[1][0], boxes[1][1], material=2, obj=1)
    # emissive quad facing down at y = 7.99
    mb.grid_quad((3.0, 7.99, 3.0), (2.0, 0.0, 0.0), (0.0, 0.0, 2.0), 1, 1, material=3)
    albedo = [[0.7, 0.7, 0.7], box_albedo[0], box_albedo[1], [0.0, 0.0, 0.0]]
    emission = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [5.0, 5.0, 5.0]]
    scene = mb.build(albedo, emission)

    sun = np.array([0.3, 1.0, 0.2])
    sun /= np.linalg.norm(sun)
    lights = Lights(sun.reshape(1, 3).astype(np.float32),
                    np.full((1, 3), 2.0, dtype=np.float32),
                    np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                    np.zeros(3, np.float32))
    vol = VolumeDesc(origin=(1.0, 1.0, 1.0), spacing=(2.0, 2.0, 2.0), counts=(4, 4, 4),
                     rays_per_probe=64)
    q = Stream(c, STREAM_QUERIES)
    pos = q.uniform(3 * n_queries, 0.0, 8.0).reshape(-1, 3)
    nrm = q.unit_vectors(n_queries)
    queries = Queries(pos.astype(np.float32), nrm.astype(np.float32), nrm.astype(np.float32))
    w = Workload("room-4x4x4-64rays", c, scene, lights, [vol], queries,
                 classify_rotations=rotations(c, 5, start_frame=1000))
    w.info["boxes"] = [(lo.tolist(), hi.tolist()) for lo, hi in boxes]
    return w


def _city_buildings(g: Stream, lots=8, lot=2.0, probe_off=0.5, margin=0.06):
    planes = np.arange(0, 64) + probe_off
    out = []
    for li in range(lots):
        for lk in range(lots):
            while True:
                w = g.uniform(2, 0.8, 1.6)
                ox = g.uniform(1, 0.1, lot - 0.1 - w[0])[0]
                oz = g.uniform(1, 0.1, lot - 0.1 - w[1])[0]
                h = float(np.clip(np.exp(math.log(4.0) + 0.5 * g.normal(1)[0]), 1.0, 20.0))
                lo = np.array([li * lot + ox, 0.0, lk * lot + oz])
                hi = np.array([lo[0] + w[0], h, lo[2] + w[1]])
                if any(_near_any(x, planes, margin) for x in (lo[0], hi[0], lo[2], hi[2], hi[1])):
                    continue
                out.append((lo, hi))
                break
    return out


def config1(n_emissive: int = 32, target_triangles: int = 100_000, config: int = 1,
            width: int = 1920, height: int = 1080, gbuffer: bool = True) -> Workload:
    """Procedural city: 16 m ground (64x64 quads), 8x8 lots of extruded
    boxes with log-normal heights (median 4 m), emissive wall quads of
    radiance U[1,10], 8 point lights.  16x8x16 probes at 1 m; 256 rays.
    Queries: a 1920x1080 G-buffer from a seeded pinhole camera."""
    c = config
    g = Stream(c, STREAM_GEOMETRY)
    buildings = _city_buildings(g)
    area = sum(2 * (hi[0] - lo[0] + hi[2] - lo[2]) * hi[1] + (hi[0] - lo[0]) * (hi[2] - lo[2])
               for lo, hi in buildings)
    ground_tris = 64 * 64 * 2
    cell = math.sqrt(2.0 * area / max(1, target_triangles - ground_tris))

    mb = MeshBuilder()
    n_mat = 1 + len(buildings) + n_emissive
    albedo = np.zeros((n_mat, 3))
    emission = np.zeros((n_mat, 3))
    albedo[0] = 0.5
    mb.grid_quad((0.0, 0.0, 0.0), (0.0, 0.0, 16.0), (16.0, 0.0, 0.0), 64, 64, material=0)
    balb = g.uniform(3 * len(buildings), 0.2, 0.9).reshape(-1, 3)
    for b, (lo, hi) in enumerate(buildings):
        albedo[1 + b] = balb[b]
        mb.box(lo, hi, material=1 + b, cell=cell, faces=("+x", "-x", "+y", "+z", "-z"))
    # emissive quads, 0.5 m, 1 cm proud of a wall, facing out
    emq = []
    for e in range(n_emissive):
        b = int(g.uniform(1, 0, len(buildings))[0])
        lo, hi = buildings[b]
        side = int(g.uniform(1, 0, 4)[0])
        y0 = g.uniform(1, 0.3, max(0.31, hi[1] - 0.8))[0]
        m = 1 + len(buildings) + e
        rad = g.uniform(1, 1.0, 10.0)[0]
        emission[m] = rad
        if side < 2:  # x walls
            x = hi[0] + 0.01 if side == 0 else lo[0] - 0.01
            z0 = g.uniform(1, lo[2], max(lo[2] + 1e-3, hi[2] - 0.5))[0]
            if side == 0:
                mb.grid_quad((x, y0, z0), (0, 0.5, 0), (0, 0, 0.5), 1, 1, material=m)
            else:
                mb.grid_quad((x, y0, z0), (0, 0, 0.5), (0, 0.5, 0), 1, 1, material=m)
            emq.append(("x", x, (y0, y0 + 0.5), (z0, z0 + 0.5), 1.0 if side == 0 else -1.0))
        else:
            z = hi[2] + 0.01 if side == 2 else lo[2] - 0.01
            x0 = g.uniform(1, lo[0], max(lo[0] + 1e-3, hi[0] - 0.5))[0]
            if side == 2:
                mb.grid_quad((x0, y0, z), (0.5, 0, 0), (0, 0.5, 0), 1, 1, material=m)
            else:
                mb.grid_quad((x0, y0, z), (0, 0.5, 0), (0.5, 0, 0), 1, 1, material=m)
            emq.append(("z", z, (y0, y0 + 0.5), (x0, x0 + 0.5), 1.0 if side == 2 else -1.0))
    scene = mb.build(albedo, emission)

    lg = Stream(c, STREAM_LIGHTS)
    pts, inten = [], []
    while len(pts) < 8:
        p = np.array([lg.uniform(1, 1, 15)[0], lg.uniform(1, 0.5, 8)[0], lg.uniform(1, 1, 15)[0]])
        inside = any(np.all(p > lo - 0.1) and np.all(p < hi + 0.1) for lo, hi in buildings)
        if not inside:
            pts.append(p)
            inten.append(lg.uniform(1, 5, 40)[0])
    lights = Lights(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                    np.array(pts, np.float32), np.repeat(np.array(inten)[:, None], 3, 1).astype(np.float32),
                    np.zeros(3, np.float32))
    vol = VolumeDesc(origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0), counts=(16, 8, 16),
                     rays_per_probe=256)
    w = Workload("city-16x8x16-256rays", c, scene, lights, [vol],
                 classify_rotations=rotations(c, 5, start_frame=1000))
    w.info["buildings"] = [(lo.tolist(), hi.tolist()) for lo, hi in buildings]
    w.info["cell"] = cell
    if gbuffer:
        cam = Stream(c, STREAM_CAMERA)
        eye = np.array([8.0 + cam.uniform(1, -1, 1)[0], 9.0, 1.0])
        w.queries, w.info["gbuffer_misses"] = camera_gbuffer(
            eye, np.array([8.0, 0.0, 9.0]), 50.0, width, height, buildings, emq, ground=16.0)
    return w


def camera_gbuffer(eye, target, vfov_deg, width, height, boxes, quads, ground):
    """G-buffer of a pinhole camera over the analytic city description
    (ground rectangle y=0, axis-aligned building boxes, axis-aligned emissive
    rectangles), returned as query points (position, normal, direction to the
    camera).  Pixels that see nothing are dropped; their count is returned."""
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    tw = th * width / height
    px = (np.arange(width) + 0.5) / width * 2 - 1
    py = 1 - (np.arange(height) + 0.5) / height * 2
    X, Y = np.meshgrid(px, py)
    d = fwd + X[..., None] * tw * right + Y[..., None] * th * up
    d = (d / np.linalg.norm(d, axis=-1, keepdims=True)).reshape(-1, 3)
    n_pix = d.shape[0]
    best = np.full(n_pix, np.inf)
    nrm = np.zeros((n_pix, 3))
    # ground plane y = 0 over [0, ground]^2, normal +y
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -eye[1] / d[:, 1]
    p = eye + t[:, None] * d
    ok = (t > 0) & (p[:, 0] >= 0) & (p[:, 0] <= ground) & (p[:, 2] >= 0) & (p[:, 2] <= ground)
    best = np.where(ok, t, best)
    nrm[ok] = (0.0, 1.0, 0.0)
    inv = 1.0 / np.where(d == 0, 1e-30, d)
    pix_x = np.tile(np.arange(width), height)
    pix_y = np.repeat(np.arange(height), width)

    def candidates(lo, hi):
        # pixels inside the screen rectangle spanned by the box's corners
        cs = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])]) - eye
        zc = cs @ fwd
        if np.any(zc <= 1e-6):
            return np.arange(n_pix)
        sx = (cs @ right) / (zc * tw)
        sy = (cs @ up) / (zc * th)
        x0 = int(np.floor((sx.min() + 1) / 2 * width)) - 1
        x1 = int(np.ceil((sx.max() + 1) / 2 * width)) + 1
        y0 = int(np.floor((1 - sy.max()) / 2 * height)) - 1
        y1 = int(np.ceil((1 - sy.min()) / 2 * height)) + 1
        x0, y0 = max(x0, 0), max(y0, 0)
        x1, y1 = min(x1, width), min(y1, height)
        if x0 >= x1 or y0 >= y1:
            return np.zeros(0, dtype=np.int64)
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        return (yy * width + xx).ravel()

    for lo, hi in boxes:
        lo = np.asarray(lo)
        hi = np.asarray(hi)
        idx = candidates(lo, hi)
        if idx.size == 0:
            continue
        t0 = (lo - eye) * inv[idx]
        t1 = (hi - eye) * inv[idx]
        tmin = np.minimum(t0, t1)
        tmax = np.maximum(t0, t1)
        tn = tmin.max(axis=1)
        tf = tmax.min(axis=1)
        hit = (tn <= tf) & (tn > 0) & (tn < best[idx])
        if not np.any(hit):
            continue
        hi_idx = idx[hit]
        axis = tmin[hit].argmax(axis=1)
        n = np.zeros((hi_idx.size, 3))
        n[np.arange(hi_idx.size), axis] = -np.sign(d[hi_idx, axis])
        best[hi_idx] = tn[hit]
        nrm[hi_idx] = n
    for (ax, c0, (a0, a1), (b0, b1), s) in quads:
        k = 0 if ax == "x" else 2
        other = 2 if ax == "x" else 0
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (c0 - eye[k]) / d[:, k]
        p = eye + t[:, None] * d
        hit = (t > 0) & (t < best) & (p[:, 1] >= a0) & (p[:, 1] <= a1) & (p[:, other] >= b0) & (p[:, other] <= b1)
        hit &= (d[:, k] * s) < 0
        n = np.zeros(3)
        n[k] = s
        best = np.where(hit, t, best)
        nrm[hit] = n
    seen = np.isfinite(best)
    pos = eye + best[seen, None] * d[seen]
    view = -d[seen]
    return Queries(pos.astype(np.float32), nrm[seen].astype(np.float32), view.astype(np.float32)), int(n_pix - seen.sum())


def config2(**kw) -> Workload:
    """Config 1 with the blend on MFMA (bf16 or f16) and FP16 atlases."""
    w = config1(config=1, **kw)
    w.name = "city-16x8x16-256rays-mfma"
    return w


# ----- terrain (config 3)


def _value_noise(x, z, seed: int, octave: int):
    ix = np.floor(x).astype(np.int64)
    iz = np.floor(z).astype(np.int64)
    fx = x - ix
    fz = z - iz

    def lat(a, b):
        key = ((a & 0xFFFFF) << 20 | (b & 0xFFFFF)).astype(np.uint64) + np.uint64(octave << 40)
        with np.errstate(over="ignore"):
            zz = np.uint64(seed) + (key + np.uint64(1)) * GAMMA
            zz = (zz ^ (zz >> np.uint64(30))) * _M1
            zz = (zz ^ (zz >> np.uint64(27))) * _M2
            zz = zz ^ (zz >> np.uint64(31))
        return (zz >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2 - 1

    sx = fx * fx * (3 - 2 * fx)
    sz = fz * fz * (3 - 2 * fz)
    v00, v10 = lat(ix, iz), lat(ix + 1, iz)
    v01, v11 = lat(ix, iz + 1), lat(ix + 1, iz + 1)
    return (v00 * (1 - sx) + v10 * sx) * (1 - sz) + (v01 * (1 - sx) + v11 * sx) * sz


def terrain_height(x, z, seed: int, amplitude=24.0, base_freq=1.0 / 64.0, octaves=6):
    h = np.zeros_like(np.asarray(x, dtype=np.float64))
    amp, f = 1.0, base_freq
    for o in range(octaves):
        h += amp * _value_noise(np.asarray(x) * f, np.asarray(z) * f, seed, o)
        amp *= 0.5
        f *= 2.0
    return amplitude * h


def config3(grid_vertices: int = 708, size: float = 256.0, n_buildings: int = 400,
            cascade_counts=(32, 16, 32), spacings=(1.0, 2.0, 4.0, 8.0), rays: int = 192,
            config: int = 3, center_height: float = 6.0) -> Workload:
    """fBm heightfield terrain (grid_vertices^2 vertices over size^2 m)
    plus extruded buildings; four concentric cascades with doubling
    spacing; 192 rays; a directional sun at 40 deg elevation whose azimuth
    moves 1 deg per frame (see ``sun_for_frame``)."""
    c = config
    g = Stream(c, STREAM_GEOMETRY)
    seed = 1000 * c + STREAM_GEOMETRY
    n = grid_vertices
    xs = np.linspace(0.0, size, n)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    H = terrain_height(X, Z, seed)
    verts = np.stack([X, H, Z], -1).reshape(-1, 3)
    idx = np.arange(n * n).reshape(n, n)
    p00 = idx[:-1, :-1].ravel()
    p10 = idx[1:, :-1].ravel()
    p11 = idx[1:, 1:].ravel()
    p01 = idx[:-1, 1:].ravel()
    # front side +y: (v1 - v0) x (v2 - v0) with v0=(x,z), v1=(x,z+1), v2=(x+1,z+1)
    tris = np.concatenate([np.stack([p00, p01, p11], 1), np.stack([p00, p11, p10], 1)])
    mb = MeshBuilder()
    mb.add(verts, tris, material=0)
    albedo = [[0.45, 0.42, 0.35]]
    emission = [[0, 0, 0]]
    for b in range(n_buildings):
        w = g.uniform(2, 3.0, 10.0)
        x0 = g.uniform(1, 4.0, size - 4.0 - w[0])[0]
        z0 = g.uniform(1, 4.0, size - 4.0 - w[1])[0]
        hgt = float(np.clip(np.exp(math.log(8.0) + 0.5 * g.normal(1)[0]), 3.0, 40.0))
        corners_x = np.array([x0, x0 + w[0], x0, x0 + w[0]])
        corners_z = np.array([z0, z0, z0 + w[1], z0 + w[1]])
        hs = terrain_height(corners_x, corners_z, seed)
        base = float(hs.min()) - 1.0
        top = float(hs.max()) + hgt
        alb = g.uniform(3, 0.2, 0.8)
        albedo.append(alb.tolist())
        emission.append([0, 0, 0])
        mb.box((x0, base, z0), (x0 + w[0], top, z0 + w[1]), material=len(albedo) - 1,
               cell=2.0, faces=("+x", "-x", "+y", "+z", "-z"))
    scene = mb.build(albedo, emission)
    cy = float(terrain_height(np.array([size / 2]), np.array([size / 2]), seed)[0]) + center_height
    C = np.array([size / 2, cy, size / 2])
    vols = []
    counts = np.array(cascade_counts)
    for s in spacings:
        ext = (counts - 1) * s
        o = C - ext / 2
        vols.append(VolumeDesc(origin=tuple(float(np.float32(x)) for x in o), spacing=(s, s, s),
                               counts=tuple(int(x) for x in counts), rays_per_probe=rays))
    lights = sun_for_frame(0)
    w = Workload("terrain-4x32x16x32-192rays", c, scene, lights, vols,
                 classify_rotations=rotations(c, 5, start_frame=1000))
    w.info["center"] = C.tolist()
    return w


def sun_for_frame(frame: int, elevation_deg=40.0, azimuth0_deg=30.0, E=3.0, sky=0.3) -> Lights:
    el = math.radians(elevation_deg)
    az = math.radians(azimuth0_deg + frame)
    d = np.array([math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az)])
    return Lights(d.reshape(1, 3).astype(np.float32), np.full((1, 3), E, np.float32),
                  np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                  np.full(3, sky, np.float32))


def surface_points(scene: Scene, n: int, config: int, stream: int = STREAM_QUERIES,
                   front_of=None) -> Queries:
    """Area-weighted random points on the scene's triangles with their front
    normals; the view direction equals the normal."""
    s = Stream(config, stream)
    v = scene.vertices.astype(np.float64)
    t = scene.indices.astype(np.int64)
    a, b, cc = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(b - a, cc - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    cdf = np.cumsum(area) / area.sum()
    pick = np.minimum(np.searchsorted(cdf, s.uniform(n)), len(area) - 1)
    u = s.uniform(n)
    w = s.uniform(n)
    su = np.sqrt(u)
    b0, b1, b2 = 1 - su, su * (1 - w), su * w
    pos = b0[:, None] * a[pick] + b1[:, None] * b[pick] + b2[:, None] * cc[pick]
    nrm = cr[pick] / np.linalg.norm(cr[pick], axis=1, keepdims=True)
    return Queries(pos.astype(np.float32), nrm.astype(np.float32), nrm.astype(np.float32))


def config4(n_points: int = 65536) -> Workload:
    """Config 1 city with 64 emissive quads; query points sampled by area on
    the scene's triangles; a seeded +/-30 % perturbation of the emitter
    radiances defines the target (``target_emission``)."""
    w = config1(n_emissive=64, config=4, gbuffer=False)
    w.name = "city-64emitters-grad"
    w.queries = surface_points(w.scene, n_points, 4)
    return w


def target_emission(w: Workload) -> np.ndarray:
    s = Stream(w.config, STREAM_TARGET)
    em = w.scene.emission.astype(np.float64)
    delta = s.uniform(em.size, -0.3, 0.3).reshape(em.shape)
    return (em * (1.0 + delta)).astype(np.float32)


# ----- small scenes used as pins


def sphere_mesh(radius: float, subdiv: int, center=(0.0, 0.0, 0.0), inward=True):
    """Icosphere with vertices on the sphere; faces wound toward the centre
    when ``inward``."""
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    for _ in range(subdiv):
        cache = {}
        NF = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = V[i] + V[j]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        for (a, b, c) in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            NF += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = NF
    verts = np.array(V) * radius + np.asarray(center)
    tris = np.array(F, dtype=np.int64)
    if inward:
        tris = tris[:, [0, 2, 1]]
    return verts, tris


def sphere_scene(radius=3.0, subdiv=3, emission=0.0, albedo=0.0, center=(0.0, 0.0, 0.0)) -> Scene:
    verts, tris = sphere_mesh(radius, subdiv, center)
    mb = MeshBuilder()
    mb.add(verts, tris, material=0)
    return mb.build([[albedo] * 3 if np.isscalar(albedo) else albedo],
                    [[emission] * 3 if np.isscalar(emission) else emission])


def empty_scene() -> Scene:
    return Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.uint32), np.zeros(0, np.uint32),
                 np.zeros(0, np.uint32), np.full((1, 3), 0.5, np.float32), np.zeros((1, 3), np.float32))


def random_triangle_soup(n: int, config: int = 90, extent=4.0, size=0.8) -> Scene:
    s = Stream(config, STREAM_GEOMETRY)
    centers = s.uniform(3 * n, -extent, extent).reshape(n, 1, 3)
    offs = s.uniform(9 * n, -size, size).reshape(n, 3, 3)
    verts = (centers + offs).reshape(-1, 3)
    tris = np.arange(3 * n).reshape(n, 3)
    mb = MeshBuilder()
    mb.add(verts, tris, material=0)
    sc = mb.build([[0.5, 0.5, 0.5]], [[0, 0, 0]])
    sc.tri_object = (np.arange(n) % 5 == 0).astype(np.uint32)
    return sc
