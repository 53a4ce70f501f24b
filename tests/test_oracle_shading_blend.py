"""Pins of the oracle's hit shading and probe blend.

Shading (paper, Section "Probe Update" and the backface rule at the end of
the self-shadow-bias section): misses see the sky; backfaces record zero
radiance and 20 % of their distance; front faces are Lambertian.  The blend
is Eq. U read as a normalised weighted average with hysteresis.
"""
import math

import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S


def _plane_scene(albedo=0.6, emission=0.0, half=50.0):
    mb = S.MeshBuilder()
    # y = 0 plane, front side +y
    mb.grid_quad((-half, 0, -half), (0, 0, 2 * half), (2 * half, 0, 0), 1, 1, material=0)
    return mb.build([[albedo] * 3], [[emission] * 3])


def _lights(point=None, intensity=None, sun=None, E=None, sky=0.0):
    z = np.zeros((0, 3), np.float32)
    L = S.Lights(z, z, z, z, np.full(3, sky, np.float32))
    if point is not None:
        L.point_pos = np.array([point], np.float32)
        L.point_intensity = np.array([intensity], np.float32)
    if sun is not None:
        s = np.asarray(sun, float)
        L.dir_to_light = (s / np.linalg.norm(s)).reshape(1, 3).astype(np.float32)
        L.dir_irradiance = np.array([E], np.float32)
    return L


def test_point_light_over_a_plane(orc):
    """L = rho * I * cos(theta) / (pi * dist^2) for a Lambertian plane under a
    point light of intensity I (W/sr)."""
    rho, I = 0.6, np.array([10.0, 20.0, 5.0])
    sc = orc.Scene(_plane_scene(rho))
    for lx, h in [(0.0, 2.0), (1.5, 3.0), (-4.0, 1.0)]:
        L = _lights(point=(lx, h, 0.0), intensity=I)
        rec = orc.shade_ray(sc, L, [], [0.0, 1.0, 0.0], [0.0, -1.0, 0.0], 10.0)
        dist = math.hypot(lx, h)
        exp = rho * I * (h / dist) / (math.pi * dist * dist)
        assert rec["tri"] >= 0 and rec["d"] == pytest.approx(1.0)
        assert np.allclose(rec["rgb"], exp, rtol=2e-4)  # shadow-ray origin is lifted by 1e-4 m
        assert rec["vis"] == 1


def test_directional_light_and_shadow(orc):
    rho, E = 0.5, np.array([3.0, 3.0, 3.0])
    sun = np.array([0.4, 1.0, -0.2])
    sc = orc.Scene(_plane_scene(rho))
    rec = orc.shade_ray(sc, _lights(sun=sun, E=E), [], [0.3, 2.0, 0.1], [0.0, -1.0, 0.0], 10.0)
    cos = (sun / np.linalg.norm(sun))[1]
    assert np.allclose(rec["rgb"], rho * E * cos / math.pi, rtol=1e-12)
    # a blocker between the hit and the sun removes the direct term
    mb = S.MeshBuilder()
    mb.grid_quad((-50, 0, -50), (0, 0, 100), (100, 0, 0), 1, 1, material=0)
    mb.grid_quad((-3, 1.0, -3), (0, 0, 6), (6, 0, 0), 1, 1, material=0)   # roof at y = 1
    sc2 = orc.Scene(mb.build([[rho] * 3], [[0, 0, 0]]))
    rec = orc.shade_ray(sc2, _lights(sun=sun, E=E), [], [0.3, 0.5, 0.1], [0.0, -1.0, 0.0], 10.0)
    assert np.all(rec["rgb"] == 0) and rec["vis"] == 0


def test_backface_miss_and_emission(orc):
    sc = orc.Scene(_plane_scene(0.7, emission=2.5))
    # from below the plane looking up: the back side
    rec = orc.shade_ray(sc, _lights(sky=0.3), [], [0.0, -2.0, 0.0], [0.0, 1.0, 0.0], 10.0)
    assert np.all(rec["rgb"] == 0) and rec["d"] == pytest.approx(0.2 * 2.0, abs=1e-15)
    # backface distance is clamped too
    rec = orc.shade_ray(sc, _lights(sky=0.3), [], [0.0, -20.0, 0.0], [0.0, 1.0, 0.0], 3.0)
    assert rec["d"] == 3.0
    # miss: sky radiance at the clamp distance
    rec = orc.shade_ray(sc, _lights(sky=0.3), [], [0.0, 2.0, 0.0], [0.0, 1.0, 0.0], 7.5)
    assert rec["tri"] < 0 and np.allclose(rec["rgb"], 0.3) and rec["d"] == 7.5
    # front face of an emitter with no lights and no probes: its emission
    rec = orc.shade_ray(sc, _lights(), [], [0.0, 2.0, 0.0], [0.0, -1.0, 0.0], 10.0)
    assert np.allclose(rec["rgb"], 2.5) and rec["d"] == pytest.approx(2.0)


def test_sun_in_closed_room_is_occluded(orc):
    w = S.config0()
    sc = orc.Scene(w.scene)
    st = S.Stream(907, 1)
    dirs = st.unit_vectors(300)
    for d in dirs:
        rec = orc.shade_ray(sc, w.lights, [], [3.0, 1.0, 1.0], d, 5.0)
        assert rec["vis"] == 0


# ------------------------------------------------------------------ blend


def _blend(orc, omega, rgb, d, p=50.0, ai=0.0, ad=0.0, irr=None, dist=None):
    irr = np.zeros((8, 8, 3)) if irr is None else irr.copy()
    dist = np.zeros((16, 16, 2)) if dist is None else dist.copy()
    orc.blend_probe(omega, rgb, d, p, ai, ad, irr, dist)
    return irr, dist


@pytest.mark.parametrize("n", [64, 256])
def test_uniform_sky_gives_its_radiance(orc, n):
    omega = orc.sf_directions(n, S.rotations(0, 1)[0])
    L = np.array([0.3, 1.7, 2.2])
    irr, dist = _blend(orc, omega, np.tile(L, (n, 1)), np.full(n, 4.5))
    assert np.allclose(irr, L, rtol=1e-13)
    assert np.allclose(dist[..., 0], 4.5, rtol=1e-13) and np.allclose(dist[..., 1], 4.5 ** 2, rtol=1e-13)


def test_linear_sky_converges_to_the_lobe_mean(orc):
    """Radiance a + b w_z: the cosine-weighted hemisphere mean about n is
    a + (2/3) b n_z, the cos^p-weighted mean is a + b n_z (p+1)/(p+2)."""
    a, b, p = 1.0, 0.8, 50.0
    errs_i, errs_d = [], []
    for n in (1024, 4096, 16384):
        omega = orc.sf_directions(n, S.rotations(0, 1, start_frame=3)[0])
        f = a + b * omega[:, 2]
        irr, dist = _blend(orc, omega, np.repeat(f[:, None], 3, 1), f, p=p)
        ei = ed = 0.0
        for y in range(1, 7):
            for x in range(1, 7):
                nz = orc.texel_direction(8, x, y)[2]
                ei = max(ei, abs(irr[y, x, 0] - (a + 2 / 3 * b * nz)))
        for y in range(1, 15):
            for x in range(1, 15):
                nz = orc.texel_direction(16, x, y)[2]
                ed = max(ed, abs(dist[y, x, 0] - (a + b * nz * (p + 1) / (p + 2))))
        errs_i.append(ei)
        errs_d.append(ed)
    assert errs_i[-1] < 2e-4 and errs_d[-1] < 2e-3
    assert errs_i[-1] < errs_i[0] and errs_d[-1] < errs_d[0]


def test_hysteresis(orc):
    """texel' = alpha * texel + (1 - alpha) * new; alpha = 1 keeps the texel."""
    n = 64
    omega = orc.sf_directions(n, np.eye(3, dtype=np.float32))
    st = S.Stream(908, 1)
    old_i = st.uniform(8 * 8 * 3).reshape(8, 8, 3)
    old_d = st.uniform(16 * 16 * 2).reshape(16, 16, 2)
    irr, dist = _blend(orc, omega, np.full((n, 3), 2.0), np.full(n, 3.0), ai=1.0, ad=1.0, irr=old_i, dist=old_d)
    for y in range(1, 7):
        for x in range(1, 7):
            assert np.array_equal(irr[y, x], old_i[y, x])
    irr, dist = _blend(orc, omega, np.full((n, 3), 2.0), np.full(n, 3.0), ai=0.97, ad=0.9, irr=old_i, dist=old_d)
    assert np.allclose(irr[3, 4], 0.97 * old_i[3, 4] + 0.03 * 2.0, rtol=1e-14)
    assert np.allclose(dist[5, 9], [0.9 * old_d[5, 9, 0] + 0.1 * 3.0, 0.9 * old_d[5, 9, 1] + 0.1 * 9.0], rtol=1e-14)


def test_border_repeats_blended_interior(orc):
    n = 128
    omega = orc.sf_directions(n, S.rotations(0, 1, start_frame=5)[0])
    st = S.Stream(909, 1)
    irr, dist = _blend(orc, omega, st.uniform(3 * n).reshape(n, 3), st.uniform(n, 0.5, 3))
    for m, t in ((8, irr), (16, dist)):
        for y in range(m):
            for x in range(m):
                sx, sy = orc.border_source(m, x, y)
                assert np.array_equal(t[y, x], t[sy, sx])


def test_zero_weight_keeps_old_texel(orc):
    # a single ray straight up: texels facing down have no positive weight
    omega = np.array([[0.0, 0.0, 1.0]])
    old = np.full((8, 8, 3), 7.0)
    irr, _ = _blend(orc, omega, np.array([[1.0, 1.0, 1.0]]), np.array([2.0]), irr=old)
    for y in range(1, 7):
        for x in range(1, 7):
            nz = orc.texel_direction(8, x, y)[2]
            assert np.allclose(irr[y, x], 7.0 if nz <= 0 else 1.0)
