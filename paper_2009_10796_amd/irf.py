"""Python binding of the irf C ABI (``include/irf.h``).

Argument marshalling only: every step of the probe update and query runs in
the HIP kernels of ``libirf.so``.  PyTorch provides device memory (the
volume buffers, query inputs and outputs) and the current HIP stream.  If
the library is missing or the GPU is unavailable, calls raise instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libirf.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_STATE, E_UNSUPPORTED = range(6)
OFF, SLEEPING, NEWLY_AWAKE, NEWLY_VIGILANT, AWAKE, VIGILANT = range(6)
ATLAS_F32, ATLAS_F16 = 0, 1
BLEND = {"f32": 0, "bf16": 1, "f16": 2, "f32_valu": 3}
MAX_VOLUMES, MAX_LIGHTS, MAX_ROTATIONS = 8, 32, 8


class IrfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("n_vertices", C.c_int64), ("indices", C.c_void_p),
                ("n_triangles", C.c_int64), ("tri_material", C.c_void_p), ("tri_object", C.c_void_p),
                ("albedo", C.c_void_p), ("emission", C.c_void_p), ("n_materials", C.c_int32),
                ("specular", C.c_void_p)]


class LightsDesc(C.Structure):
    _fields_ = [("dir_to_light", C.c_void_p), ("dir_irradiance", C.c_void_p), ("n_dir", C.c_int32),
                ("point_pos", C.c_void_p), ("point_intensity", C.c_void_p), ("n_point", C.c_int32),
                ("sky", C.c_float * 3)]


class VolumeDescC(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("spacing", C.c_float * 3), ("counts", C.c_int32 * 3),
                ("rays_per_probe", C.c_int32), ("hysteresis_irr", C.c_float), ("hysteresis_dist", C.c_float),
                ("cos_power", C.c_float), ("self_shadow_bias", C.c_float), ("max_distance", C.c_float),
                ("cheb_power", C.c_int32), ("atlas_dtype", C.c_int32), ("blend", C.c_int32),
                ("irradiance_gamma", C.c_float), ("texel_thresholds", C.c_int32), ("tracking", C.c_int32)]


class BufferSizes(C.Structure):
    _fields_ = [("n_probes", C.c_int64), ("irradiance_bytes", C.c_int64), ("distance_bytes", C.c_int64),
                ("states_bytes", C.c_int64), ("offsets_bytes", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("trace_blocks", C.c_int32), ("shadow_blocks", C.c_int32), ("shade_blocks", C.c_int32),
                ("blend_blocks", C.c_int32), ("shadow_refill", C.c_int32), ("blend_rsplit", C.c_int32),
                ("query_shadow", C.c_int32)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


RECORD_DTYPE = np.dtype([("tri", np.int32), ("t", np.float32), ("rgb", np.float32, 3), ("d", np.float32),
                         ("vis", np.uint32), ("probe", np.int32)])

# every function the header declares, with (restype, argtypes)
_vp, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64
SIGNATURES = {
    "irf_status_str": (C.c_char_p, [C.c_int]),
    "irf_last_error": (C.c_char_p, []),
    "irf_version": (C.c_char_p, []),
    "irf_create": (C.c_int, [_i32, C.POINTER(_vp)]),
    "irf_destroy": (None, [_vp]),
    "irf_set_scene": (C.c_int, [_vp, C.POINTER(SceneDesc)]),
    "irf_set_lights": (C.c_int, [_vp, C.POINTER(LightsDesc)]),
    "irf_create_volume": (C.c_int, [_vp, C.POINTER(VolumeDescC), C.POINTER(_i32)]),
    "irf_volume_sizes": (C.c_int, [_vp, _i32, C.POINTER(BufferSizes)]),
    "irf_bind_volume": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "irf_classify": (C.c_int, [_vp, _vp, _i32, _vp]),
    "irf_update_probes": (C.c_int, [_vp, _vp, _vp]),
    "irf_update_probes_after": (C.c_int, [_vp, _vp, _vp, _vp]),
    "irf_update_probes_noalloc": (C.c_int, [_vp, _vp, _vp]),
    "irf_query_irradiance": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "irf_update_probes_query": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "irf_ray_records": (C.c_int, [_vp, _i32, _vp, _i64, C.POINTER(_i64), _vp]),
    "irf_frame_stats": (C.c_int, [_vp, C.POINTER(_i64 * 4), _vp]),
    "irf_traversal_stats": (C.c_int, [_vp, C.POINTER(_i64 * 4), _vp]),
    "irf_set_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "irf_get_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "irf_graph_capture": (C.c_int, [_vp, _vp, C.POINTER(_vp)]),
    "irf_graph_capture_query": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp, C.POINTER(_vp)]),
    "irf_graph_launch": (C.c_int, [_vp, _vp, _vp, _vp]),
    "irf_graph_destroy": (None, [_vp]),
    "irf_optimize_probes": (C.c_int, [_vp, _vp, _i32, C.c_float, _vp]),
    "irf_track_volume": (C.c_int, [_vp, _i32, _vp, _vp, _i32, _vp, _vp]),
    "irf_volume_window": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "irf_trace_glossy": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "irf_set_differentiable": (C.c_int, [_vp, _i32]),
    "irf_set_emission": (C.c_int, [_vp, _vp, _vp]),
    "irf_query_backward": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "irf_update_backward": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "irf_profile_enable": (C.c_int, [_vp, _i32]),
    "irf_profile_read": (C.c_int, [_vp, _vp, _i32, C.POINTER(_i32), _i32]),
    "irf_validate_volume_desc": (C.c_int, [C.POINTER(VolumeDescC)]),
    "irf_bvh_stats": (C.c_int, [C.POINTER(SceneDesc), C.POINTER(C.c_double * 5)]),
}

_lib = None


def load() -> C.CDLL:
    """Loads libirf.so (building it first only if it is absent).  A library
    built from other sources than the ones beside it (its build stamp does
    not match them) is refused: rebuild it."""
    global _lib
    if _lib is None:
        from . import build as _build
        if not os.path.exists(LIB_PATH):
            _build.build()
        stamp = open(_build.STAMP).read().strip() if os.path.exists(_build.STAMP) else None
        if stamp != _build.source_hash():
            raise RuntimeError(f"{LIB_PATH} was not built from the sources beside it "
                               f"({'no build stamp' if stamp is None else 'sources changed since'}): rebuild it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != OK:
        raise IrfError(status, load().irf_last_error().decode())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def scene_desc(scene):
    spec = scene.specular_or_zero() if hasattr(scene, "specular_or_zero") else np.zeros_like(scene.albedo)
    keep = [_np(scene.vertices, np.float32), _np(scene.indices, np.uint32), _np(scene.tri_material, np.uint32),
            _np(scene.tri_object, np.uint32), _np(scene.albedo, np.float32), _np(scene.emission, np.float32),
            _np(spec, np.float32)]
    d = SceneDesc(_ptr(keep[0]), keep[0].shape[0], _ptr(keep[1]), keep[1].shape[0], _ptr(keep[2]),
                  _ptr(keep[3]), keep[4].ctypes.data_as(C.c_void_p), keep[5].ctypes.data_as(C.c_void_p),
                  keep[4].shape[0], keep[6].ctypes.data_as(C.c_void_p))
    return d, keep


def volume_desc(desc) -> VolumeDescC:
    d = VolumeDescC()
    for a in range(3):
        d.origin[a] = desc.origin[a]
        d.spacing[a] = desc.spacing[a]
        d.counts[a] = desc.counts[a]
    d.rays_per_probe = desc.rays_per_probe
    d.hysteresis_irr = desc.hysteresis_irr
    d.hysteresis_dist = desc.hysteresis_dist
    d.cos_power = desc.cos_power
    d.self_shadow_bias = desc.self_shadow_bias
    d.max_distance = desc.max_distance
    d.cheb_power = desc.cheb_power
    d.atlas_dtype = ATLAS_F16 if desc.atlas_f16 else ATLAS_F32
    d.blend = BLEND[desc.blend]
    d.irradiance_gamma = float(getattr(desc, "irradiance_gamma", 1.0))
    d.texel_thresholds = int(bool(getattr(desc, "texel_thresholds", False)))
    d.tracking = int(bool(getattr(desc, "tracking", False)))
    return d


def validate_volume_desc(desc) -> None:
    d = volume_desc(desc)
    _check(load().irf_validate_volume_desc(C.byref(d)))


def bvh_stats(scene) -> dict:
    d, keep = scene_desc(scene)
    out = (C.c_double * 5)()
    _check(load().irf_bvh_stats(C.byref(d), C.byref(out)))
    return {"nodes": int(out[0]), "leaves": int(out[1]), "depth": int(out[2]), "sah": out[3], "valid": out[4] == 1.0}


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Volume:
    """Caller-owned (torch) device buffers of one probe volume."""

    def __init__(self, ctx: "Context", vid: int, desc, torch, device):
        self.ctx, self.id, self.desc = ctx, vid, desc
        sz = BufferSizes()
        _check(load().irf_volume_sizes(ctx.handle, vid, C.byref(sz)))
        P = int(sz.n_probes)
        dt = torch.float16 if desc.atlas_f16 else torch.float32
        self.irradiance = torch.zeros((P, 8, 8, 4), dtype=dt, device=device)
        self.distance = torch.zeros((P, 16, 16, 2), dtype=dt, device=device)
        self.states = torch.full((P,), NEWLY_VIGILANT, dtype=torch.uint8, device=device)
        self.offsets = torch.zeros((P, 3), dtype=torch.float32, device=device)
        assert self.irradiance.numel() * self.irradiance.element_size() == sz.irradiance_bytes
        assert self.distance.numel() * self.distance.element_size() == sz.distance_bytes
        self.rebind()

    def rebind(self):
        _check(load().irf_bind_volume(self.ctx.handle, self.id, C.c_void_p(self.irradiance.data_ptr()),
                                      C.c_void_p(self.distance.data_ptr()), C.c_void_p(self.states.data_ptr()),
                                      C.c_void_p(self.offsets.data_ptr())))

    @property
    def n_probes(self) -> int:
        return int(self.states.shape[0])


class Context:
    """One irf context on one GPU."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise IrfError(E_HIP, "no GPU available for the irf library")
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        _check(load().irf_create(device, C.byref(h)))
        self.handle = h
        self.volumes: List[Volume] = []
        self.n_lights = 0
        self.frames = 0          # update frames run (eager or replayed)

    def close(self):
        if getattr(self, "handle", None):
            load().irf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scene(self, scene) -> None:
        d, keep = scene_desc(scene)
        _check(load().irf_set_scene(self.handle, C.byref(d)))

    def set_lights(self, lights) -> None:
        keep = [_np(lights.dir_to_light, np.float32).reshape(-1, 3), _np(lights.dir_irradiance, np.float32).reshape(-1, 3),
                _np(lights.point_pos, np.float32).reshape(-1, 3), _np(lights.point_intensity, np.float32).reshape(-1, 3)]
        d = LightsDesc(_ptr(keep[0]), _ptr(keep[1]), keep[0].shape[0], _ptr(keep[2]), _ptr(keep[3]), keep[2].shape[0])
        for a in range(3):
            d.sky[a] = float(lights.sky[a])
        _check(load().irf_set_lights(self.handle, C.byref(d)))
        self.n_lights = keep[0].shape[0] + keep[2].shape[0]

    def create_volume(self, desc) -> Volume:
        d = volume_desc(desc)
        vid = C.c_int32()
        _check(load().irf_create_volume(self.handle, C.byref(d), C.byref(vid)))
        v = Volume(self, vid.value, desc, self.torch, self.device)
        self.volumes.append(v)
        return v

    def classify(self, rotations) -> None:
        R = _np(rotations, np.float32).reshape(-1, 9)
        _check(load().irf_classify(self.handle, _ptr(R), R.shape[0], _stream(self.torch)))

    def optimize_probes(self, rotations, offset_limit: float = 0.45) -> None:
        """Probe relocation: one pass per rotation (run before classify)."""
        R = _np(rotations, np.float32).reshape(-1, 9)
        _check(load().irf_optimize_probes(self.handle, _ptr(R), len(R), float(offset_limit), _stream(self.torch)))

    def track_volume(self, vol: int, camera, rotations) -> np.ndarray:
        """Moves a tracking volume's window toward the camera (entering planes
        reset and classified with `rotations`); returns the shift in cells."""
        cam = _np(camera, np.float32).reshape(3)
        R = _np(rotations, np.float32).reshape(-1, 9)
        shift = np.zeros(3, dtype=np.int32)
        _check(load().irf_track_volume(self.handle, vol, _ptr(cam), _ptr(R), len(R), _ptr(shift),
                                       _stream(self.torch)))
        return shift

    def volume_window(self, vol: int):
        """(origin, phase, camera) of a volume's window."""
        o = np.zeros(3, np.float32)
        ph = np.zeros(3, np.int32)
        cam = np.zeros(3, np.float32)
        _check(load().irf_volume_window(self.handle, vol, _ptr(o), _ptr(ph), _ptr(cam)))
        return o, ph, cam

    def update_probes(self, rotation, after=None) -> None:
        """One update frame on the current stream.  `after`: a recorded
        torch.cuda.Event (e.g. after the previous frame's queries on another
        stream) that the frame's atlas writes wait for."""
        R = _np(rotation, np.float32).reshape(9)
        if after is None:
            _check(load().irf_update_probes(self.handle, _ptr(R), _stream(self.torch)))
        else:
            _check(load().irf_update_probes_after(self.handle, _ptr(R), _stream(self.torch),
                                                  C.c_void_p(after.cuda_event)))
        self.frames += 1

    def update_probes_noalloc(self, rotation) -> None:
        """One update frame that allocates nothing (its scratch is the
        library's static per-GPU array; see irf_update_probes_noalloc)."""
        R = _np(rotation, np.float32).reshape(9)
        _check(load().irf_update_probes_noalloc(self.handle, _ptr(R), _stream(self.torch)))
        self.frames += 1

    def _query_args(self, pos, nrm, view, out):
        torch = self.torch
        n = int(pos.shape[0])
        for t in (pos, nrm, view):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (n, 3):
                raise IrfError(E_INVALID, "query inputs must be contiguous float32 CUDA tensors of shape [n, 3]")
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
        elif out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or tuple(out.shape) != (n, 3):
            raise IrfError(E_INVALID, "the query output must be a contiguous float32 CUDA tensor of shape [n, 3]")
        return n, out

    def update_probes_query(self, rotation, pos, nrm, view, out=None):
        """One update frame that also answers the queries against the atlases
        the previous frame left (inside the frame's probe-ray and shadow-ray
        launches, split by the tuning's query_shadow); returns `out`, equal
        to query_irradiance() called before update_probes()."""
        n, out = self._query_args(pos, nrm, view, out)
        R = _np(rotation, np.float32).reshape(9)
        _check(load().irf_update_probes_query(self.handle, _ptr(R), C.c_void_p(pos.data_ptr()),
                                              C.c_void_p(nrm.data_ptr()), C.c_void_p(view.data_ptr()), n,
                                              C.c_void_p(out.data_ptr()), _stream(self.torch)))
        self.frames += 1
        return out

    def query_irradiance(self, pos, nrm, view, out=None):
        n, out = self._query_args(pos, nrm, view, out)
        _check(load().irf_query_irradiance(self.handle, C.c_void_p(pos.data_ptr()), C.c_void_p(nrm.data_ptr()),
                                           C.c_void_p(view.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                           _stream(self.torch)))
        return out

    def glossy(self, pos, nrm, view, records: bool = False):
        """Second-order glossy: radiance along each point's mirror direction
        [n, 3] (and the per-point records when asked)."""
        torch = self.torch
        n = int(pos.shape[0])
        out = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        rec = torch.empty((max(1, n) * RECORD_DTYPE.itemsize,), dtype=torch.uint8, device=self.device) if records else None
        _check(load().irf_trace_glossy(self.handle, C.c_void_p(pos.data_ptr()), C.c_void_p(nrm.data_ptr()),
                                       C.c_void_p(view.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                       C.c_void_p(rec.data_ptr()) if rec is not None else None, _stream(torch)))
        if not records:
            return out
        torch.cuda.current_stream().synchronize()
        return out, rec[: n * RECORD_DTYPE.itemsize].cpu().numpy().view(RECORD_DTYPE)

    # ---- adjoint

    def set_differentiable(self, enable: bool = True) -> None:
        _check(load().irf_set_differentiable(self.handle, int(enable)))

    def set_emission(self, emission) -> None:
        e = emission.detach().to(self.device, self.torch.float32).contiguous()
        _check(load().irf_set_emission(self.handle, C.c_void_p(e.data_ptr()), _stream(self.torch)))
        self._emission_keep = e

    @staticmethod
    def _ptrs(tensors):
        a = (C.c_void_p * len(tensors))()
        for i, t in enumerate(tensors):
            assert t.is_contiguous() and t.dtype.is_floating_point
            a[i] = t.data_ptr()
        return a

    def query_backward(self, pos, nrm, view, grad_out, grad_irr, grad_dist) -> None:
        n = int(pos.shape[0])
        g = grad_out.contiguous()
        _check(load().irf_query_backward(self.handle, C.c_void_p(pos.data_ptr()), C.c_void_p(nrm.data_ptr()),
                                         C.c_void_p(view.data_ptr()), n, C.c_void_p(g.data_ptr()),
                                         self._ptrs(grad_irr), self._ptrs(grad_dist), _stream(self.torch)))

    def update_backward(self, g_new_irr, g_new_dist, g_prev_irr, g_prev_dist, g_emission) -> None:
        _check(load().irf_update_backward(self.handle, self._ptrs(g_new_irr), self._ptrs(g_new_dist),
                                          self._ptrs(g_prev_irr), self._ptrs(g_prev_dist),
                                          C.c_void_p(g_emission.data_ptr()), _stream(self.torch)))

    def frame_stats(self) -> dict:
        out = (C.c_int64 * 4)()
        _check(load().irf_frame_stats(self.handle, C.byref(out), _stream(self.torch)))
        return {"active_probes": out[0], "probe_rays": out[1], "shadow_rays": out[2], "front_hits": out[3]}

    def traversal_stats(self) -> dict:
        out = (C.c_int64 * 4)()
        _check(load().irf_traversal_stats(self.handle, C.byref(out), _stream(self.torch)))
        return {"probe_nodes": out[0], "probe_tris": out[1], "shadow_nodes": out[2], "shadow_tris": out[3]}

    def set_tuning(self, **kw) -> None:
        t = Tuning()
        _check(load().irf_get_tuning(self.handle, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(load().irf_set_tuning(self.handle, C.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().irf_get_tuning(self.handle, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def capture_frame(self, stream=None) -> "FrameGraph":
        """Captures one update frame as a HIP graph on `stream` (a torch
        stream other than the default one)."""
        st = stream or self.torch.cuda.current_stream()
        g = C.c_void_p()
        _check(load().irf_graph_capture(self.handle, C.c_void_p(st.cuda_stream), C.byref(g)))
        return FrameGraph(self, g, st)

    def capture_frame_query(self, pos, nrm, view, out, stream=None) -> "FrameGraph":
        """Captures the frame of update_probes_query: each launch also writes
        into `out` the queries at pos/nrm/view (tensors fixed at capture, their
        contents may change) against the atlases the previous frame left."""
        n, out = self._query_args(pos, nrm, view, out)
        st = stream or self.torch.cuda.current_stream()
        g = C.c_void_p()
        _check(load().irf_graph_capture_query(self.handle, C.c_void_p(st.cuda_stream), C.c_void_p(pos.data_ptr()),
                                              C.c_void_p(nrm.data_ptr()), C.c_void_p(view.data_ptr()), n,
                                              C.c_void_p(out.data_ptr()), C.byref(g)))
        graph = FrameGraph(self, g, st)
        graph.tensors = (pos, nrm, view, out)   # kept alive while the graph is
        return graph

    def profile(self, enable: bool = True) -> None:
        _check(load().irf_profile_enable(self.handle, int(enable)))

    def profile_read(self, reset: bool = True) -> dict:
        n = C.c_int32()
        _check(load().irf_profile_read(self.handle, None, 0, C.byref(n), 0))
        arr = (KernelTime * max(1, n.value))()
        _check(load().irf_profile_read(self.handle, arr, n.value, C.byref(n), int(reset)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}

    def ray_records(self, vol: int) -> np.ndarray:
        torch = self.torch
        cnt = C.c_int64()
        _check(load().irf_ray_records(self.handle, vol, None, 0, C.byref(cnt), _stream(torch)))
        n = int(cnt.value)
        buf = torch.empty((max(1, n) * RECORD_DTYPE.itemsize,), dtype=torch.uint8, device=self.device)
        _check(load().irf_ray_records(self.handle, vol, C.c_void_p(buf.data_ptr()), n, C.byref(cnt), _stream(torch)))
        torch.cuda.current_stream().synchronize()
        return buf[: n * RECORD_DTYPE.itemsize].cpu().numpy().view(RECORD_DTYPE)


class FrameGraph:
    """A captured update frame; launch(rotation) replays it with the
    context's current lights."""

    def __init__(self, ctx: Context, handle, stream):
        self.ctx, self.handle, self.stream = ctx, handle, stream

    def launch(self, rotation) -> None:
        R = _np(rotation, np.float32).reshape(9)
        _check(load().irf_graph_launch(self.ctx.handle, self.handle, _ptr(R), C.c_void_p(self.stream.cuda_stream)))
        self.ctx.frames += 1

    def close(self):
        if getattr(self, "handle", None):
            load().irf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_workload(w, device: int = 0):
    """Context with the workload's scene, lights and volumes (in order)."""
    ctx = Context(device)
    ctx.set_scene(w.scene)
    ctx.set_lights(w.lights)
    for d in w.volumes:
        ctx.create_volume(d)
    return ctx
