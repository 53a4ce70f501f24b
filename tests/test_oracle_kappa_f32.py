"""The oracle's float32 sensitivity estimates (kappa) checked as error
bounds.

kappa (units of u = 2^-24) decides how far a float32 result may sit from
the FP64 oracle before the parity protocol (tests/parity.py) calls it wrong.
Here it is checked against an actual float32 evaluation of the same steps:
the oracle's own source built with its value path in float32
(``liborc32.so``: octahedral map, ray directions, hit shading, blend, query
in float, nearest-hit search exact for the float32 ray) is run through the
same protocol as the GPU library, and every ray, texel and query must lie
within 1e-5 s + 8 u kappa of the FP64 oracle (s = max(|o|, tau)).  The
workloads are those of the GPU parity tests: the room, the room with
perception encoding, thresholds and a lighting change, the reduced terrain
cascades with a moving sun (64 and 32 rays, the latter above 4,096 probes),
the city, and second-order glossy.

This pins kappa to something other than itself: a dropped term (the hit
point's coordinate rounding, the normal's rounding, the distance of a
grazing hit) shows up here as an element beyond its bound.
"""
import numpy as np
import pytest

import oracle
from paper_2009_10796_amd import scenes as S
from tests import parity as P


def _pair(w):
    osc, osc32 = oracle.Scene(w.scene), oracle.Scene(w.scene, f32=True)
    ov = [oracle.Volume(d) for d in w.volumes]
    ov32 = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    for a, b in zip(ov32, ov):
        a.states[:] = b.states
    return osc, osc32, ov, ov32


def _frames(w, schedule, lights_of=None):
    """schedule: (frame, emission or None); returns (verdicts, reports, ov, ov32)."""
    osc, osc32, ov, ov32 = _pair(w)
    verdicts, reports = [], []
    for f, em in schedule:
        if em is not None:
            osc.set_emission(em.astype(np.float64))
            osc32.set_emission(em.astype(np.float64))
        L = lights_of(f) if lights_of else w.lights
        R = w.frame_rotation(f)
        r32 = oracle.update_frame(osc32, L, ov32, R)
        rec, rep = P.oracle_frame(osc, L, ov, R, r32["tri"], r32["vis"])
        assert rep.unflagged_flips == 0, rep.line()
        vs, t_bad = P.ray_checks(f"frame {f}", r32["rgb"], r32["d"], r32["t"], rec,
                                 P.origin_magnitude(ov, P.active_counts(ov)))
        assert t_bad == 0
        for v, (a, b) in enumerate(zip(ov32, ov)):
            assert np.array_equal(a.states, b.states)
            vs += P.texel_checks(f"frame {f} volume {v}", a.irr, a.dist, b)
        verdicts += vs
        reports.append(rep)
        print(f"[kappa] frame {f}: {rep.line()}", flush=True)
    return verdicts, reports, ov, ov32


def _queries(ov, ov32, q, n=None):
    n = q.n if n is None else min(n, q.n)
    pos, nrm, view = q.pos[:n], q.nrm[:n], q.view[:n]
    e32, _ = oracle.query(ov32, pos, nrm, view, f32=True)
    e64, k64 = oracle.query(ov, pos, nrm, view)
    out = [P.compare("query end-to-end", e32, e64, k64)]
    # stage: both sides on the FP64 atlas rounded to float32
    ovr = oracle.copy_volumes(ov)
    for a in ovr:
        a.irr[:] = a.irr.astype(np.float32)
        a.dist[:] = a.dist.astype(np.float32)
        a.irr_kappa[:] = 0.0
        a.dist_kappa[:] = 0.0
    e32, _ = oracle.query(ovr, pos, nrm, view, f32=True)
    e64, k64 = oracle.query(ovr, pos, nrm, view)
    out.append(P.compare("query stage", e32, e64, k64))
    return out


def _assert(verdicts):
    for v in verdicts:
        print("[kappa]", v.line(), flush=True)
    bad = [v for v in verdicts if not v.ok]
    assert not bad, [(v.name, v.fail, v.worst_allowed, v.where[:3]) for v in bad]


def small_terrain(cascade_counts=(8, 4, 8), rays=64):
    return S.config3(grid_vertices=97, size=48.0, n_buildings=12, cascade_counts=cascade_counts,
                     spacings=(1.0, 2.0, 4.0, 8.0), rays=rays, center_height=3.0)


def test_kappa_bounds_float32_room():
    w = S.config0()
    vs, _, ov, ov32 = _frames(w, [(1, None), (2, None), (3, None)])
    _assert(vs + _queries(ov, ov32, w.queries))


def test_kappa_bounds_float32_encoded_room_with_lighting_change():
    w = S.config0()
    for d in w.volumes:
        d.irradiance_gamma = 5.0
        d.texel_thresholds = True
    em = w.scene.emission.astype(np.float32)
    dim = (em * np.float32(0.05)).astype(np.float32)
    vs, _, ov, ov32 = _frames(w, [(1, None), (2, None), (3, dim), (4, dim), (5, em), (6, em)])
    _assert(vs + _queries(ov, ov32, w.queries)[:1])


@pytest.mark.parametrize("counts,rays", [((8, 4, 8), 64), ((16, 8, 16), 32)])
def test_kappa_bounds_float32_terrain_cascades(counts, rays):
    w = small_terrain(counts, rays)
    vs, _, ov, ov32 = _frames(w, [(f, None) for f in (1, 2, 3)], lights_of=S.sun_for_frame)
    _assert(vs + _queries(ov, ov32, S.surface_points(w.scene, 20000, 3)))


def test_kappa_bounds_float32_city():
    w = S.config1()
    vs, reps, ov, ov32 = _frames(w, [(1, None), (2, None)])
    # the float32 build decides a few rays of this city otherwise: the
    # substitution path is exercised
    assert sum(r.substituted for r in reps) > 0
    _assert(vs + _queries(ov, ov32, w.queries, n=300000))


@pytest.mark.parametrize("name", ["room", "city"])
def test_kappa_bounds_float32_glossy(name):
    w = S.config0() if name == "room" else S.config1()
    M = w.scene.albedo.shape[0]
    spec = np.full((M, 3), 0.2, np.float32)
    spec[0] = 0.5
    w.scene.specular = spec
    osc, osc32 = oracle.Scene(w.scene), oracle.Scene(w.scene, f32=True)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    for f in (1, 2):
        oracle.update_frame(osc, w.lights, ov, w.frame_rotation(f), records=False)
    for o in ov:
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
    q = w.queries
    sel = np.arange(0, q.n, max(1, q.n // 100000))
    pos, nrm, view = q.pos[sel], q.nrm[sel], q.view[sel]
    if name == "room":
        st = S.Stream(985, 1)
        view = st.unit_vectors(len(pos)).astype(np.float32)
        view = np.where((np.sum(view * nrm, 1) < 0)[:, None], -view, view).astype(np.float32)
    g32 = oracle.glossy(osc32, w.lights, ov, pos, nrm, view)
    g64 = oracle.glossy(osc, w.lights, ov, pos, nrm, view)
    flip = (g32["tri"] != g64["tri"]) | (g32["vis"] != g64["vis"])
    assert not np.any(flip & ((g64["flags"] & oracle.F_AMBIGUOUS) == 0))
    _assert([P.compare(f"{name} glossy", g32["rgb"][~flip], g64["rgb"][~flip], g64["kappa"][~flip])])


def test_checker_catches_planted_errors():
    """The comparison fails on a texel moved by three times its allowance
    and on a swapped pair of texels, and counts a texel moved beyond 1e-5 s
    but within its kappa allowance as widened."""
    w = S.config0()
    vs, _, ov, ov32 = _frames(w, [(1, None), (2, None)])
    _assert(vs)
    o, k = ov[0].irr, ov[0].irr_kappa
    s = np.maximum(np.abs(o), P.channel_tau(o))
    allowed = np.minimum(P.REL * s + 8 * P.U32 * k, P.CAP * s)
    big = np.abs(o) > 0.1 * np.abs(o).max()
    i = np.unravel_index(np.argmin(np.where(big, allowed / s, np.inf)), o.shape)
    base = P.compare("unchanged", ov32[0].irr, o, k)
    irr = ov32[0].irr.copy()
    irr[i] = o[i] + 3 * allowed[i]
    assert P.compare("planted", irr, o, k).fail == 1
    j = np.unravel_index(np.argmax(np.where(big & (allowed > 3 * P.REL * s), allowed / s, 0)), o.shape)
    irr = ov32[0].irr.copy()
    irr[j] = o[j] + 2 * P.REL * s[j]
    v = P.compare("planted within kappa", irr, o, k)
    assert v.ok and v.widened == base.widened + (abs(ov32[0].irr[j] - o[j]) <= P.REL * s[j])
    q, y, x = i[:3]
    irr = ov32[0].irr.copy()
    irr[q, y, x], irr[q, y, x + 1] = ov32[0].irr[q, y, x + 1], ov32[0].irr[q, y, x]
    if np.abs(o[q, y, x] - o[q, y, x + 1]).max() > 1e-3 * np.abs(o[q, y, x]).max():
        assert not P.compare("swapped", irr, o, k).ok


def test_forced_hit_adopts_the_given_triangle():
    """orc_update_frame_forced: a ray forced onto another triangle records it
    with the exact plane distance and the forced flag; a ray forced to a miss
    sees the sky; forced shadow bits replace the oracle's."""
    w = S.config1()
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    saved = oracle.copy_volumes(ov)
    R = w.frame_rotation(1)
    rec = oracle.update_frame(osc, w.lights, ov, R)
    P.restore(ov, saved)
    n = len(rec)
    hits = np.nonzero(rec["tri"] >= 0)[0]
    i, j = hits[0], hits[1]
    mask = np.zeros(n, np.uint8)
    tri = rec["tri"].copy()
    vis = rec["vis"].copy()
    mask[i] = 1
    tri[i] = -1
    mask[j] = 2
    vis[j] = 0
    rec2 = oracle.update_frame(osc, w.lights, ov, R, force=(mask, tri, vis))
    assert rec2[i]["tri"] == -1 and rec2[i]["flags"] & oracle.F_FORCED
    assert np.allclose(rec2[i]["rgb"], w.lights.sky)
    assert rec2[j]["vis"] == 0 and rec2[j]["tri"] == rec[j]["tri"]
    others = np.ones(n, bool)
    others[[i, j]] = False
    assert np.array_equal(rec2["tri"][others], rec["tri"][others])
    assert np.array_equal(rec2["rgb"][others], rec["rgb"][others])
    # a ray forced onto its own triangle's neighbour along the same plane
    # keeps the plane distance
    P.restore(ov, saved)
    k = hits[2]
    mask = np.zeros(n, np.uint8)
    mask[k] = 1
    rec3 = oracle.update_frame(osc, w.lights, ov, R, force=(mask, rec["tri"], rec["vis"]))
    assert rec3[k]["tri"] == rec[k]["tri"] and rec3[k]["t"] == rec[k]["t"]


def test_kappa_bounds_float32_open_air_window():
    """The dynamic-states workload: a window of probes in open air over the
    city's rooftops, whose distance texels sit at the clamp, so many
    hit-shading queries rest on a Chebyshev variance below float32's
    resolution; a building moves before frame 3."""
    from tests.test_gpu_dynamic_states import city_with_dynamic_building
    w, scene_a = city_with_dynamic_building()
    _, scene_b = city_with_dynamic_building((4.0, 0.0, 0.0))
    w.scene = scene_a
    w.volumes = [S.VolumeDesc(origin=(3.5, 5.5, 4.5), spacing=(1.0, 1.0, 1.0), counts=(10, 4, 6), rays_per_probe=64)]
    osc, osc32, ov, ov32 = _pair(w)
    sb, sb32 = oracle.Scene(scene_b), oracle.Scene(scene_b, f32=True)
    verdicts = []
    for f in (1, 2, 3, 4):
        a, b = (osc, osc32) if f < 3 else (sb, sb32)
        R = w.frame_rotation(f)
        r32 = oracle.update_frame(b, w.lights, ov32, R)
        rec, rep = P.oracle_frame(a, w.lights, ov, R, r32["tri"], r32["vis"])
        assert rep.unflagged_flips == 0
        vs, t_bad = P.ray_checks(f"frame {f}", r32["rgb"], r32["d"], r32["t"], rec,
                                 P.origin_magnitude(ov, P.active_counts(ov)))
        assert t_bad == 0
        vs += P.texel_checks(f"frame {f}", ov32[0].irr, ov32[0].dist, ov[0])
        verdicts += vs
    _assert(verdicts)
    beyond = max(v.beyond_cap / v.n for v in verdicts)
    print(f"[kappa] open-air window: largest share beyond 1e-3 {beyond:.3f}", flush=True)
