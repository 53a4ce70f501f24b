"""FP64 CPU oracle of the probe update and probe query (TEST INFRASTRUCTURE).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``liborc.so`` (built from
``irf_oracle.c`` by ``oracle/build.py``) with ctypes and keeps all state in
numpy float64 arrays owned by Python.  ``f32=True`` selects ``liborc32.so``,
the same source built as a float32 evaluation of the value path; it is used
only to check the oracle's float32 sensitivity estimates (kappa).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional

import numpy as np

from . import build as _build

OFF, SLEEPING, NEWLY_AWAKE, NEWLY_VIGILANT, AWAKE, VIGILANT = 0, 1, 2, 3, 4, 5
F_GRAZE, F_TIE, F_NEARMISS, F_EDGEON, F_SHADOW, F_FORCED, F_FORCE_INVALID = 1, 2, 4, 8, 16, 32, 64
F_AMBIGUOUS = F_GRAZE | F_TIE | F_NEARMISS | F_EDGEON | F_SHADOW
CAGE = 16

_lib = None
_lib32 = None


def lib(f32: bool = False):
    """The oracle library (f32=True: its float32 build)."""
    global _lib, _lib32
    if (_lib32 if f32 else _lib) is None:
        path = _build.LIB32 if f32 else _build.LIB
        if not os.path.exists(path):
            _build.build()
        if not _build.stamp_ok(path):
            raise RuntimeError(f"{path} was not built from the oracle's sources beside it: rebuild it with "
                               "`python oracle/build.py`")
        L = C.CDLL(path)
        _declare(L)
        if f32:
            _lib32 = L
        else:
            _lib = L
    return _lib32 if f32 else _lib


class Hit(C.Structure):
    _fields_ = [("tri", C.c_int32), ("flags", C.c_int32), ("t", C.c_double), ("bmin", C.c_double)]


class RayRecord(C.Structure):
    _fields_ = [("tri", C.c_int32), ("flags", C.c_int32), ("t", C.c_double), ("rgb", C.c_double * 3),
                ("d", C.c_double), ("vis", C.c_uint32), ("n_cage", C.c_int32),
                ("cage", C.c_int32 * CAGE), ("kappa", C.c_double * 3), ("cosi", C.c_double),
                ("d_kappa", C.c_double)]


RECORD_DTYPE = np.dtype([("tri", np.int32), ("flags", np.int32), ("t", np.float64), ("rgb", np.float64, 3),
                         ("d", np.float64), ("vis", np.uint32), ("n_cage", np.int32),
                         ("cage", np.int32, CAGE), ("kappa", np.float64, 3), ("cosi", np.float64),
                         ("d_kappa", np.float64)], align=True)
assert RECORD_DTYPE.itemsize == C.sizeof(RayRecord)
HIT_DTYPE = np.dtype([("tri", np.int32), ("flags", np.int32), ("t", np.float64), ("bmin", np.float64)], align=True)


class Lights(C.Structure):
    _fields_ = [("n_dir", C.c_int32), ("dir_to_light", C.c_void_p), ("dir_irradiance", C.c_void_p),
                ("n_point", C.c_int32), ("point_pos", C.c_void_p), ("point_intensity", C.c_void_p),
                ("sky", C.c_float * 3)]


class VolumeStruct(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("spacing", C.c_float * 3), ("counts", C.c_int32 * 3),
                ("rays", C.c_int32), ("alpha_irr", C.c_float), ("alpha_dist", C.c_float),
                ("cos_power", C.c_float), ("bias", C.c_float), ("dmax", C.c_float), ("cheb_power", C.c_int32),
                ("irr", C.c_void_p), ("dist", C.c_void_p), ("states", C.c_void_p), ("offsets", C.c_void_p),
                ("irr_kappa", C.c_void_p), ("dist_kappa", C.c_void_p), ("gamma", C.c_float),
                ("texel_thresholds", C.c_int32), ("phase", C.c_int32 * 3), ("tracking", C.c_int32),
                ("camera", C.c_float * 3)]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _declare(L):
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    L.orc_scene_create.restype = vp
    L.orc_scene_create.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, i32]
    L.orc_scene_free.argtypes = [vp]
    L.orc_scene_set_emission.argtypes = [vp, dp]
    L.orc_scene_set_specular.argtypes = [vp, dp]
    L.orc_scene_bvh_nodes.restype = i64
    L.orc_scene_bvh_nodes.argtypes = [vp]
    for name in ("orc_oct_encode", "orc_oct_decode"):
        getattr(L, name).argtypes = [dp, dp]
    L.orc_texel_direction.argtypes = [i32, i32, i32, dp]
    L.orc_border_source.argtypes = [i32, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.orc_sample_tile.argtypes = [dp, i32, i32, dp, dp]
    L.orc_sf_direction.argtypes = [i32, i32, vp, dp]
    L.orc_trace_batch.argtypes = [vp, i64, dp, dp, i32, i32, vp]
    L.orc_blend_probe.argtypes = [i32, dp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_blend_probe_ex.argtypes = [i32, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, i32, dp, dp]
    L.orc_query_batch.argtypes = [vp, i32, i64, vp, vp, vp, dp, dp]
    L.orc_query_look.argtypes = [vp, i32, dp, dp, dp, dp, dp, dp, vp, vp]
    L.orc_glossy_batch.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp, vp]
    L.orc_classify.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.orc_state_step.argtypes = [vp, vp, i32]
    L.orc_optimize_offsets.argtypes = [vp, vp, vp, i32, C.c_double, vp]
    L.orc_track_volume.argtypes = [vp, vp, vp, vp, i32, vp]
    L.orc_update_frame.restype = i64
    L.orc_update_frame.argtypes = [vp, vp, vp, i32, vp, vp, i64]
    L.orc_update_frame_forced.restype = i64
    L.orc_update_frame_forced.argtypes = [vp, vp, vp, i32, vp, vp, i64, i64, vp, vp, vp]
    L.orc_shade_ray.argtypes = [vp, vp, vp, i32, dp, dp, C.c_double, vp]
    L.orc_query_backward.argtypes = [vp, i32, dp, dp, dp, dp, vp]
    L.orc_update_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, dp]


# ---------------------------------------------------------------- wrappers


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def oct_encode(v) -> np.ndarray:
    v = _d(v, 3)
    p = np.zeros(2)
    lib().orc_oct_encode(_p(v), _p(p))
    return p


def oct_decode(p) -> np.ndarray:
    p = _d(p, 2)
    v = np.zeros(3)
    lib().orc_oct_decode(_p(p), _p(v))
    return v


def texel_direction(m: int, x: int, y: int) -> np.ndarray:
    v = np.zeros(3)
    lib().orc_texel_direction(m, x, y, _p(v))
    return v


def border_source(m: int, x: int, y: int):
    sx, sy = C.c_int32(), C.c_int32()
    lib().orc_border_source(m, x, y, C.byref(sx), C.byref(sy))
    return sx.value, sy.value


def sample_tile(tile: np.ndarray, v) -> np.ndarray:
    tile = _d(tile)
    m, nch = tile.shape[0], tile.shape[2]
    out = np.zeros(nch)
    lib().orc_sample_tile(_p(tile), m, nch, _p(_d(v, 3)), _p(out))
    return out


def sf_directions(n: int, R) -> np.ndarray:
    R = np.ascontiguousarray(R, dtype=np.float32).reshape(9)
    out = np.zeros((n, 3))
    for i in range(n):
        lib().orc_sf_direction(i, n, _p(R), _p(out[i]))
    return out


def blend_probe(omega, rgb, d, cos_power, alpha_irr, alpha_dist, irr_tile, dist_tile):
    """In-place blend of one probe's tiles ([8,8,3] and [16,16,2] float64)."""
    omega, rgb, d = _d(omega), _d(rgb), _d(d)
    assert irr_tile.dtype == np.float64 and irr_tile.flags.c_contiguous
    assert dist_tile.dtype == np.float64 and dist_tile.flags.c_contiguous
    lib().orc_blend_probe(len(d), _p(omega), _p(rgb), _p(d), cos_power, alpha_irr, alpha_dist,
                          _p(irr_tile), _p(dist_tile))


def blend_probe_ex(omega, rgb, d, cos_power, alpha_irr, alpha_dist, gamma, thresholds, irr_tile, dist_tile):
    """blend_probe with the perception encoding exponent (1 = linear) and
    the per-texel irradiance hysteresis thresholds."""
    omega, rgb, d = _d(omega), _d(rgb), _d(d)
    assert irr_tile.dtype == np.float64 and irr_tile.flags.c_contiguous
    assert dist_tile.dtype == np.float64 and dist_tile.flags.c_contiguous
    lib().orc_blend_probe_ex(len(d), _p(omega), _p(rgb), _p(d), cos_power, alpha_irr, alpha_dist, float(gamma),
                             int(bool(thresholds)), _p(irr_tile), _p(dist_tile))


class Scene:
    """Oracle-side copy of a scene (FP64 triangles plus the oracle's own
    median-split BVH, an exact accelerator).  f32=True: a scene of the
    float32 build; every call made with it runs that build."""

    def __init__(self, scene, f32: bool = False):
        self.f32 = bool(f32)
        self.L = lib(self.f32)
        self._keep = [np.ascontiguousarray(x) for x in (scene.vertices, scene.indices, scene.tri_material,
                                                        scene.tri_object, scene.albedo, scene.emission)]
        v, i, m, o, a, e = self._keep
        self.n_triangles = int(i.shape[0])
        self.handle = self.L.orc_scene_create(_p(v), v.shape[0], _p(i), i.shape[0], _p(m), _p(o),
                                              _p(a), _p(e), a.shape[0])
        spec = getattr(scene, "specular", None)
        if spec is not None:
            self.set_specular(spec)

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "L", None) is not None:
            self.L.orc_scene_free(self.handle)
            self.handle = None

    def set_specular(self, specular) -> None:
        sp = np.ascontiguousarray(specular, dtype=np.float64).reshape(-1, 3)
        self.L.orc_scene_set_specular(self.handle, _p(sp))

    def set_emission(self, emission) -> None:
        e = np.ascontiguousarray(emission, dtype=np.float64).reshape(-1, 3)
        self.L.orc_scene_set_emission(self.handle, _p(e))

    def trace(self, origins, dirs, static_only=False, brute=False) -> np.ndarray:
        o = _d(origins).reshape(-1, 3)
        d = _d(dirs).reshape(-1, 3)
        hits = np.zeros(o.shape[0], dtype=HIT_DTYPE)
        self.L.orc_trace_batch(self.handle, o.shape[0], _p(o), _p(d), int(static_only), int(brute), _p(hits))
        return hits


def make_lights(lights) -> Lights:
    L = Lights()
    keep = [np.ascontiguousarray(x, dtype=np.float32) for x in
            (lights.dir_to_light, lights.dir_irradiance, lights.point_pos, lights.point_intensity)]
    L.n_dir = keep[0].shape[0]
    L.dir_to_light, L.dir_irradiance = _p(keep[0]), _p(keep[1])
    L.n_point = keep[2].shape[0]
    L.point_pos, L.point_intensity = _p(keep[2]), _p(keep[3])
    for c in range(3):
        L.sky[c] = float(lights.sky[c])
    L._keep = keep
    return L


class Volume:
    """Oracle volume: FP64 atlases irr[P,8,8,3], dist[P,16,16,2], uint8
    states[P], float32 offsets[P,3]."""

    def __init__(self, desc, states=None):
        self.desc = desc
        P = desc.n_probes
        self.irr = np.zeros((P, 8, 8, 3))
        self.dist = np.zeros((P, 16, 16, 2))
        self.states = np.full(P, NEWLY_VIGILANT if states is None else 0, dtype=np.uint8)
        if states is not None:
            self.states[:] = states
        self.offsets = np.zeros((P, 3), dtype=np.float32)
        # float32 sensitivity of every texel (units of 2^-24), carried by the blend
        self.irr_kappa = np.zeros((P, 8, 8, 3))
        self.dist_kappa = np.zeros((P, 16, 16, 2))
        # tracking window (Section "Tracking Windows"): current origin, circular
        # buffer phase, camera for the blend weight (initially the window centre)
        self.origin = np.asarray(desc.origin, dtype=np.float32).copy()
        self.phase = np.zeros(3, dtype=np.int32)
        self.tracking = bool(getattr(desc, "tracking", False))
        self.camera = (self.origin + 0.5 * (np.asarray(desc.counts) - 1) * np.asarray(desc.spacing)).astype(np.float32)

    def struct(self) -> VolumeStruct:
        d = self.desc
        s = VolumeStruct()
        for a in range(3):
            s.origin[a] = self.origin[a]
            s.spacing[a] = d.spacing[a]
            s.counts[a] = d.counts[a]
            s.phase[a] = self.phase[a]
            s.camera[a] = self.camera[a]
        s.tracking = int(self.tracking)
        s.rays = d.rays_per_probe
        s.alpha_irr, s.alpha_dist = d.hysteresis_irr, d.hysteresis_dist
        s.cos_power, s.bias = d.cos_power, d.self_shadow_bias
        s.dmax = d.resolved_max_distance()
        s.cheb_power = d.cheb_power
        s.gamma = float(getattr(d, "irradiance_gamma", 1.0))
        s.texel_thresholds = int(bool(getattr(d, "texel_thresholds", False)))
        for arr in (self.irr, self.dist, self.states, self.offsets):
            assert arr.flags.c_contiguous
        s.irr, s.dist, s.states, s.offsets = _p(self.irr), _p(self.dist), _p(self.states), _p(self.offsets)
        s.irr_kappa, s.dist_kappa = _p(self.irr_kappa), _p(self.dist_kappa)
        return s


def _vol_array(vols: List[Volume]):
    arr = (VolumeStruct * max(1, len(vols)))()
    for i, v in enumerate(vols):
        arr[i] = v.struct()
    return arr


def classify(scene: Scene, vols: List[Volume], rotations: np.ndarray):
    R = np.ascontiguousarray(rotations, dtype=np.float32).reshape(-1, 9)
    total = sum(v.desc.n_probes for v in vols)
    n_back = np.zeros(total, np.int32)
    n_flag = np.zeros(total, np.int32)
    t_front = np.zeros(total)
    arr = _vol_array(vols)
    scene.L.orc_classify(scene.handle, arr, len(vols), _p(R), R.shape[0], _p(n_back), _p(n_flag), _p(t_front))
    return n_back, n_flag, t_front


def optimize_offsets(scene: Scene, vol: Volume, rotations, offset_limit: float = 0.45) -> np.ndarray:
    """Probe relocation (Section "Probe Position Adjustment"): one iteration
    per rotation; updates vol.offsets in place; returns the per-probe
    ambiguity bits (bit i: iteration i)."""
    R = np.ascontiguousarray(rotations, dtype=np.float32).reshape(-1, 9)
    amb = np.zeros(vol.desc.n_probes, dtype=np.int32)
    arr = _vol_array([vol])
    scene.L.orc_optimize_offsets(scene.handle, C.byref(arr[0]), _p(R), len(R), float(offset_limit), _p(amb))
    return amb


def track_volume(scene: Scene, vol: Volume, camera, rotations) -> np.ndarray:
    """Tracking window (Section "Tracking Windows"): moves the window toward
    the camera, reinitialises the planes that enter (classification with the
    given rotations), stores the camera; returns the shift in cells."""
    cam = np.ascontiguousarray(camera, dtype=np.float32).reshape(3)
    R = np.ascontiguousarray(rotations, dtype=np.float32).reshape(-1, 9)
    arr = _vol_array([vol])
    shift = np.zeros(3, dtype=np.int32)
    scene.L.orc_track_volume(scene.handle, C.byref(arr[0]), _p(cam), _p(R), len(R), _p(shift))
    for a in range(3):
        vol.origin[a] = arr[0].origin[a]
        vol.phase[a] = arr[0].phase[a]
        vol.camera[a] = arr[0].camera[a]
    return shift


def state_step(scene: Scene, vols: List[Volume]):
    scene.L.orc_state_step(scene.handle, _vol_array(vols), len(vols))


def update_frame(scene: Scene, lights, vols: List[Volume], R, records: bool = True, force=None):
    """One update frame of all volumes (in place).  force: None, or
    (mask uint8[n], tri int32[n], vis uint32[n]) over record indices -- bit 0
    of mask adopts tri as the ray's hit (-1: miss), bit 1 adopts vis as its
    shadow bits (see orc_update_frame_forced)."""
    R = np.ascontiguousarray(R, dtype=np.float32).reshape(9)
    L = make_lights(lights)
    # states change inside; the number of active probes is known after the
    # state step, so size the record buffer for every probe
    cap = sum(v.desc.n_probes * v.desc.rays_per_probe for v in vols) if records else 0
    rec = np.zeros(cap, dtype=RECORD_DTYPE)
    arr = _vol_array(vols)
    if force is None:
        n = scene.L.orc_update_frame(scene.handle, C.byref(L), arr, len(vols), _p(R),
                                     _p(rec) if records else None, cap)
    else:
        fm = np.ascontiguousarray(force[0], dtype=np.uint8)
        ft = np.ascontiguousarray(force[1], dtype=np.int32)
        fv = np.ascontiguousarray(force[2], dtype=np.uint32)
        assert fm.shape == ft.shape == fv.shape
        n = scene.L.orc_update_frame_forced(scene.handle, C.byref(L), arr, len(vols), _p(R),
                                            _p(rec) if records else None, cap, fm.shape[0], _p(fm), _p(ft), _p(fv))
    return rec[:n] if records else None


def query(vols: List[Volume], pos, nrm, view, f32: bool = False):
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, dtype=np.float32).reshape(-1, 3)
    view = np.ascontiguousarray(view, dtype=np.float32).reshape(-1, 3)
    out = np.zeros((pos.shape[0], 3))
    kap = np.zeros((pos.shape[0], 3))
    lib(f32).orc_query_batch(_vol_array(vols), len(vols), pos.shape[0], _p(pos), _p(nrm), _p(view), _p(out),
                             _p(kap))
    return out, kap


def query_look(vols: List[Volume], X, n, wo, look, f32: bool = False):
    """One query with the texels sampled in direction `look` (the probes'
    filtered radiance); returns (value[3], kappa[3])."""
    out, kap = np.zeros(3), np.zeros(3)
    lib(f32).orc_query_look(_vol_array(vols), len(vols), _p(_d(X, 3)), _p(_d(n, 3)), _p(_d(wo, 3)),
                            _p(_d(look, 3)), _p(out), _p(kap), None, None)
    return out, kap


def glossy(scene: Scene, lights, vols: List[Volume], pos, nrm, view) -> np.ndarray:
    """Second-order glossy (Section "Second Order Glossy"): per surface point
    the record of its mirror ray (hit, shadow visibility, radiance toward the
    point, float32 sensitivity)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, dtype=np.float32).reshape(-1, 3)
    view = np.ascontiguousarray(view, dtype=np.float32).reshape(-1, 3)
    rec = np.zeros(pos.shape[0], dtype=RECORD_DTYPE)
    L = make_lights(lights)
    scene.L.orc_glossy_batch(scene.handle, C.byref(L), _vol_array(vols), len(vols), pos.shape[0], _p(pos),
                             _p(nrm), _p(view), _p(rec))
    return rec


def shade_ray(scene: Scene, lights, vols: List[Volume], o, w, dmax) -> np.ndarray:
    L = make_lights(lights)
    rec = np.zeros(1, dtype=RECORD_DTYPE)
    scene.L.orc_shade_ray(scene.handle, C.byref(L), _vol_array(vols), len(vols), _p(_d(o, 3)), _p(_d(w, 3)),
                          float(dmax), _p(rec))
    return rec[0]


# ------------------------------------------------------------------ adjoint


def _ptr_array(arrs):
    a = (C.c_void_p * len(arrs))()
    for i, x in enumerate(arrs):
        assert x.dtype == np.float64 and x.flags.c_contiguous
        a[i] = x.ctypes.data
    return a


def _linear_only(vols):
    for v in vols:
        if getattr(v.desc, "irradiance_gamma", 1.0) != 1.0 or getattr(v.desc, "texel_thresholds", False):
            raise ValueError("the adjoint covers linear irradiance texels without per-texel thresholds")


class _Grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("g_irr", "g_dist", "a_irr", "a_dist", "s_irr", "s_dist")]


def _grads(g_irr, g_dist, a_irr=None, a_dist=None, s_irr=None, s_dist=None):
    """orc_grads over per-volume float64 arrays (None: not wanted); the
    pointer arrays are kept alive on the returned structure."""
    G = _Grads()
    keep = []
    for name, arrs in (("g_irr", g_irr), ("g_dist", g_dist), ("a_irr", a_irr), ("a_dist", a_dist),
                       ("s_irr", s_irr), ("s_dist", s_dist)):
        if arrs is None:
            continue
        pa = _ptr_array(arrs)
        keep.append(pa)
        setattr(G, name, C.cast(pa, C.c_void_p))
    G._keep = keep
    return G


def query_backward(vols: List[Volume], pos, nrm, view, gout, g_irr, g_dist, a_irr=None, a_dist=None, s_irr=None,
                   s_dist=None):
    """Accumulates dLoss/d(texels) of the query into float64 arrays shaped
    like each volume's irr / dist atlases; optionally the per-texel sum of
    term magnitudes (a_*) and float32 sensitivity (s_*)."""
    _linear_only(vols)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1, 3)
    view = np.ascontiguousarray(view, dtype=np.float64).reshape(-1, 3)
    gout = np.ascontiguousarray(gout, dtype=np.float64).reshape(-1, 3)
    arr = _vol_array(vols)
    G = _grads(g_irr, g_dist, a_irr, a_dist, s_irr, s_dist)
    for i in range(pos.shape[0]):
        lib().orc_query_backward(arr, len(vols), _p(pos[i]), _p(nrm[i]), _p(view[i]), _p(gout[i]), C.byref(G))


def update_backward(scene: Scene, prev: List[Volume], R, records, g_new_irr, g_new_dist, g_prev_irr, g_prev_dist,
                    g_emission, a_new_irr=None, a_new_dist=None, a_prev_irr=None, a_prev_dist=None, s_prev_irr=None,
                    s_prev_dist=None):
    """Backward of one update frame (see orc_update_backward): accumulates
    dLoss/d(input atlases) and dLoss/d(emission); a_new_* are magnitude
    bounds of the upstream gradient (default |g_new|)."""
    _linear_only(prev)
    R = np.ascontiguousarray(R, dtype=np.float32).reshape(9)
    rec = np.ascontiguousarray(records)
    assert rec.dtype == RECORD_DTYPE
    assert g_emission.dtype == np.float64 and g_emission.flags.c_contiguous
    Gn = _grads(g_new_irr, g_new_dist, a_new_irr, a_new_dist)
    Gp = _grads(g_prev_irr, g_prev_dist, a_prev_irr, a_prev_dist, s_prev_irr, s_prev_dist)
    scene.L.orc_update_backward(scene.handle, _vol_array(prev), len(prev), _p(R), _p(rec), C.byref(Gn),
                                C.byref(Gp), _p(g_emission))


def copy_volumes(vols: List[Volume]) -> List[Volume]:
    out = []
    for v in vols:
        c = Volume(v.desc, states=v.states)
        c.origin[:] = v.origin
        c.phase[:] = v.phase
        c.camera[:] = v.camera
        c.irr[:] = v.irr
        c.dist[:] = v.dist
        c.offsets[:] = v.offsets
        c.irr_kappa[:] = v.irr_kappa
        c.dist_kappa[:] = v.dist_kappa
        out.append(c)
    return out
