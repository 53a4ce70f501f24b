"""Whole-frame pins of the oracle: trace -> shade -> blend -> states, checked
against closed forms (uniform sky, probe at the centre of a sphere, the
furnace recurrence) and hand-built state scenes (paper, Sections "Probe
Update", "Probe States" and "Full Probe Initialization Algorithm")."""
import math

import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S


def test_uniform_sky_no_geometry(orc):
    sc = orc.Scene(S.empty_scene())
    L = S.no_lights(sky=(0.4, 0.9, 1.3))
    v = orc.Volume(S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(3, 2, 2), rays_per_probe=64))
    rec = orc.update_frame(sc, L, [v], S.rotations(0, 1)[0])
    dmax = v.desc.resolved_max_distance()
    assert len(rec) == 12 * 64 and np.all(rec["tri"] < 0)
    assert np.allclose(v.irr, np.float32([0.4, 0.9, 1.3]), rtol=1e-13)   # the sky arrives as float32
    assert np.allclose(v.dist[..., 0], dmax, rtol=1e-13) and np.allclose(v.dist[..., 1], dmax ** 2, rtol=1e-13)
    assert np.all(v.states == S.VIGILANT)   # promoted after the converge frame


def test_probe_at_sphere_centre_distance(orc):
    """Mean distance and mean distance^2 of a probe at the centre of a
    tessellated sphere of radius R lie between the inscribed and
    circumscribed values; mu2 >= mu^2."""
    R = 3.0
    verts, tris = S.sphere_mesh(R, 3)
    sc = orc.Scene(S.sphere_scene(R, 3))
    # largest angle between a facet's centroid direction and its vertices
    cosmin = 1.0
    for t in tris:
        c = verts[t].mean(0)
        c /= np.linalg.norm(c)
        for k in range(3):
            cosmin = min(cosmin, float(np.dot(c, verts[t[k]] / R)))
    v = orc.Volume(S.VolumeDesc(origin=(-0.5, -0.5, -0.5), spacing=(1, 1, 1), counts=(2, 2, 2),
                                rays_per_probe=256, max_distance=10.0))
    v.offsets[0] = (0.5, 0.5, 0.5)          # probe 0 sits exactly at the centre
    orc.update_frame(sc, S.no_lights(), [v], S.rotations(0, 1, start_frame=7)[0])
    mu, mu2 = v.dist[0, 1:15, 1:15, 0], v.dist[0, 1:15, 1:15, 1]
    assert np.all(mu <= R * (1 + 1e-12)) and np.all(mu >= R * cosmin)
    assert np.all(mu2 <= R * R * (1 + 1e-12)) and np.all(mu2 >= (R * cosmin) ** 2)
    assert np.all(mu2 >= mu * mu * (1 - 1e-12))


def test_furnace_recurrence(orc):
    """Closed sphere of emission Le and albedo rho, probes inside: the atlas
    follows x_1 = Le (converge frame, alpha = 0, previous irradiance 0) and
    x_k = alpha x_{k-1} + (1 - alpha)(Le + rho x_{k-1}), whose fixed point
    is Le / (1 - rho).  Exact for any tessellation: querying a uniform atlas
    returns its value."""
    Le = np.array([1.0, 2.0, 0.5])
    rho = 0.6
    sc = orc.Scene(S.sphere_scene(4.0, 2, emission=Le.tolist(), albedo=rho))
    a = 0.9
    v = orc.Volume(S.VolumeDesc(origin=(-1, -1, -1), spacing=(1, 1, 1), counts=(3, 3, 3), rays_per_probe=64,
                                hysteresis_irr=a, hysteresis_dist=a, max_distance=20.0))
    x = np.zeros(3)
    for f in range(6):
        orc.update_frame(sc, S.no_lights(), [v], S.rotations(0, 1, start_frame=20 + f)[0])
        x = Le if f == 0 else a * x + (1 - a) * (Le + rho * x)
        assert np.allclose(v.irr, x, rtol=1e-6), f   # float32 hysteresis constants


def _box_room(cell=0.0):
    mb = S.MeshBuilder()
    mb.box((0, 0, 0), (10, 10, 10), material=0, inward=True, cell=cell)
    return mb


def test_classification_hand_scenes(orc):
    """A probe inside a closed static box is Off; a probe 0.5 m from a wall is
    Newly Vigilant; a probe in open space sleeps; a sleeping probe inside the
    box of a dynamic object grown by one cell and the bias is Newly Awake."""
    mb = _box_room()
    mb.box((1.2, 1.2, 1.2), (2.8, 2.8, 2.8), material=0, obj=0)     # closed static box around (2,2,2)
    mb.box((7.6, 7.6, 1.6), (7.9, 7.9, 1.9), material=0, obj=1)     # small dynamic object
    sc = orc.Scene(mb.build([[0.5] * 3], [[0, 0, 0]]))
    v = orc.Volume(S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(2, 2, 2), rays_per_probe=64))
    grid = np.array([[i, j, k] for k in range(2) for j in range(2) for i in range(2)], float)
    place = {0: (2.0, 2.0, 2.0),      # inside the static box
             1: (9.5, 5.0, 5.0),      # 0.5 m from the x = 10 wall
             2: (5.0, 5.0, 5.0),      # open space
             3: (7.75, 7.75, 2.5)}    # 0.6 m above the dynamic object, 2.25 m from any wall
    for q in range(8):
        v.offsets[q] = np.array(place.get(q, (5.0, 4.0 + 0.5 * q, 6.0))) - grid[q]
    orc.classify(sc, [v], S.rotations(0, 5, start_frame=40))
    assert v.states[0] == S.OFF
    assert v.states[1] == S.NEWLY_VIGILANT
    assert v.states[2] == S.SLEEPING
    # classification rays ignore dynamic geometry; the grown box wakes the probe
    assert v.states[3] == S.NEWLY_AWAKE


def test_state_step_and_promotion(orc):
    mb = _box_room()
    mb.box((4.8, 4.8, 4.8), (5.2, 5.2, 5.2), material=0, obj=1)    # dynamic object at the centre
    sc = orc.Scene(mb.build([[0.5] * 3], [[0, 0, 0]]))
    v = orc.Volume(S.VolumeDesc(origin=(3.5, 5, 5), spacing=(3, 3, 3), counts=(2, 2, 2), rays_per_probe=64))
    v.offsets[:] = 0
    # probe 0 at (3.5,5,5) is within one cell of the object; probe 7 at (6.5,8,8) too (cell=3)
    v.states[:] = [S.SLEEPING, S.AWAKE, S.VIGILANT, S.OFF, S.SLEEPING, S.AWAKE, S.NEWLY_VIGILANT, S.SLEEPING]
    v.offsets[1] = (20.0, 0, 0)                  # probe 1 moved far away: no object near it
    orc.state_step(sc, [v])
    assert v.states[0] == S.NEWLY_AWAKE and v.states[1] == S.SLEEPING
    assert v.states[2] == S.VIGILANT and v.states[3] == S.OFF and v.states[6] == S.NEWLY_VIGILANT
    orc.update_frame(sc, S.no_lights(), [v], S.rotations(0, 1)[0], records=False)
    assert v.states[0] == S.AWAKE and v.states[6] == S.VIGILANT and v.states[3] == S.OFF


def test_sleeping_and_off_probes_keep_their_texels(orc):
    sc = orc.Scene(S.empty_scene())
    v = orc.Volume(S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(2, 2, 2), rays_per_probe=32))
    v.states[:] = [S.OFF, S.SLEEPING, S.VIGILANT, S.VIGILANT, S.OFF, S.OFF, S.OFF, S.OFF]
    v.irr[:] = 9.0
    v.dist[:] = 9.0
    rec = orc.update_frame(sc, S.no_lights(sky=(1, 1, 1)), [v], S.rotations(0, 1)[0])
    assert len(rec) == 2 * 32
    assert np.all(v.irr[[0, 1, 4]] == 9.0)
    assert np.allclose(v.irr[2], 0.97 * 9 + 0.03 * 1.0, rtol=1e-6)
