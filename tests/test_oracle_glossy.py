"""Pins of the oracle's second-order glossy pass (paper, Section "Second
Order Glossy"): the mirror ray of a surface point, its hit shaded as a
probe-ray hit plus the hit's mirror reflectance times the probes' filtered
radiance in the hit's own mirror direction.  Geometry and lighting are
solved here in closed form; the probe terms are pinned by constant and
direction-dependent atlases."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

S2 = np.sqrt(2.0)


def _wall_scene(orc, albedo=0.0, emission=(0.0, 0.0, 0.0), specular=0.0):
    """A 6 x 2 m wall in the plane x = 3 facing -x, from y = 0 to 6."""
    mb = S.MeshBuilder()
    o, u, v = np.array([3.0, 0.0, -1.0]), np.array([0.0, 0.0, 2.0]), np.array([0.0, 6.0, 0.0])
    assert np.cross(u, v)[0] < 0
    mb.grid_quad(o, u, v, 1, 1, material=0)
    scene = mb.build([[albedo] * 3], [list(emission)])
    scene.specular = np.full((1, 3), specular, np.float32)
    return orc.Scene(scene), scene


def _point():
    X = np.array([[0.0, 0.0, 0.0]])
    n = np.array([[0.0, 1.0, 0.0]])
    v = np.array([[-1.0, 1.0, 0.0]]) / S2        # mirror direction (1, 1, 0) / sqrt 2
    return X, n, v


def test_sky_only(orc):
    sc = orc.Scene(S.empty_scene())
    st = S.Stream(980, 1)
    n = st.unit_vectors(200)
    v = st.unit_vectors(200)
    v = np.where((np.sum(n * v, 1) < 0)[:, None], -v, v)
    X = st.uniform(600, -3, 3).reshape(-1, 3)
    rec = orc.glossy(sc, S.no_lights(sky=(0.2, 0.5, 0.9)), [], X, n, v)
    assert np.all(rec["tri"] == -1)
    assert np.allclose(rec["rgb"], np.float32([0.2, 0.5, 0.9]), rtol=1e-12)


def test_mirror_ray_sees_an_emitter(orc):
    Le = (2.0, 1.0, 0.5)
    sc, _ = _wall_scene(orc, emission=Le)
    X, n, v = _point()
    rec = orc.glossy(sc, S.no_lights(), [], X, n, v)[0]
    assert rec["tri"] >= 0
    # from the point lifted by 1e-4 along n, along (1, 1, 0)/sqrt 2 to x = 3
    assert np.isclose(rec["t"], 3.0 * S2, rtol=1e-12)
    assert np.allclose(rec["rgb"], Le, rtol=1e-12)
    # seen from the back the wall is black
    X2 = np.array([[6.0, 0.0, 0.0]])
    v2 = np.array([[1.0, 1.0, 0.0]]) / S2
    rec = orc.glossy(sc, S.no_lights(), [], X2, n, v2)[0]
    assert rec["tri"] >= 0 and np.all(rec["rgb"] == 0.0)


def test_point_light_at_the_glossy_hit(orc):
    rho, I = 0.5, np.array([3.0, 2.0, 1.0])
    sc, _ = _wall_scene(orc, albedo=rho)
    P = np.array([1.0, 3.0, 0.0])
    lights = S.Lights(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), P[None].astype(np.float32),
                      I[None].astype(np.float32), np.zeros(3, np.float32))
    X, n, v = _point()
    rec = orc.glossy(sc, lights, [], X, n, v)[0]
    Y = np.array([0.0, 1e-4, 0.0]) + 3.0 * S2 * np.array([1.0, 1.0, 0.0]) / S2
    ng = np.array([-1.0, 0.0, 0.0])
    Ys = Y + 1e-4 * max(1.0, np.abs(Y).max()) * ng
    u = P.astype(np.float32).astype(np.float64) - Ys
    d = np.linalg.norm(u)
    expect = rho * I.astype(np.float32) * np.dot(ng, u / d) / (np.pi * d * d)
    assert rec["vis"] == 1
    assert np.allclose(rec["rgb"], expect, rtol=1e-10)


def _vol_around(orc, value):
    d = S.VolumeDesc(origin=(1.0, 1.0, -2.0), spacing=(2.0, 2.0, 2.0), counts=(3, 3, 3), rays_per_probe=64)
    v = orc.Volume(d, states=np.full(d.n_probes, S.VIGILANT))
    v.dist[..., 0] = 100.0
    v.dist[..., 1] = 100.0 ** 2 + 1.0
    v.irr[:] = value
    return v


def test_constant_probes_give_albedo_and_specular_terms(orc):
    rho, ks, C = 0.4, 0.3, np.array([0.8, 1.2, 2.0])
    sc, _ = _wall_scene(orc, albedo=rho, specular=ks)
    vol = _vol_around(orc, C)
    X, n, v = _point()
    rec = orc.glossy(sc, S.no_lights(), [vol], X, n, v)[0]
    rho32, ks32 = float(np.float32(rho)), float(np.float32(ks))   # materials arrive as float32
    assert np.allclose(rec["rgb"], (rho32 + ks32) * C, rtol=1e-12)


def _fill_tiles(orc, vol, f):
    for y in range(1, 7):
        for x in range(1, 7):
            vol.irr[:, y, x] = f(orc.texel_direction(8, x, y))
    for y in range(8):
        for x in range(8):
            sx, sy = orc.border_source(8, x, y)
            vol.irr[:, y, x] = vol.irr[:, sy, sx]


def test_look_direction_samples_that_texel(orc):
    vol = _vol_around(orc, 0.0)
    _fill_tiles(orc, vol, lambda w: np.array([1.0 + w[0], 2.0 + w[1], 3.0 + w[2]]))
    # at a probe position the query returns that probe's texel in the look direction
    X = np.array([3.0, 3.0, 0.0])
    nrm = np.array([0.0, 1.0, 0.0])
    look = orc.texel_direction(8, 2, 5)
    e, _ = orc.query_look([vol], X, nrm, nrm, look)
    assert np.allclose(e, [1.0 + look[0], 2.0 + look[1], 3.0 + look[2]], rtol=1e-12)
    e_n, _ = orc.query_look([vol], X, nrm, nrm, nrm)
    assert not np.allclose(e, e_n, rtol=1e-3)


def test_second_bounce_uses_the_hit_mirror_direction(orc):
    """Probes whose texels encode their direction: the specular term comes
    back close to r2 = reflect(r, ng) = (-1, 1, 0)/sqrt 2 and far from the
    ray's own direction r = (1, 1, 0)/sqrt 2 or the normal."""
    ks = 1.0
    sc, _ = _wall_scene(orc, specular=ks)
    vol = _vol_around(orc, 0.0)
    _fill_tiles(orc, vol, lambda w: 2.0 + w)       # channel k = 2 + w_k
    X, n, v = _point()
    rec = orc.glossy(sc, S.no_lights(), [vol], X, n, v)[0]
    g = np.asarray(rec["rgb"]) - 2.0
    r2 = np.array([-1.0, 1.0, 0.0]) / S2
    assert np.dot(g / np.linalg.norm(g), r2) > 0.97
    assert np.dot(g, np.array([1.0, 1.0, 0.0]) / S2) < 0.2
